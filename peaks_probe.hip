// Peak-rate probe of the GPU the transform runs on: a device-to-device copy
// (HBM bandwidth), reads of a buffer that stays in the L2 caches and of one
// that stays in the last-level (infinity) cache, independent chains of FP32
// FMA in the non-packed form the kernels are compiled to (once with a
// scalar-register operand, once with vector-register operands only: the two
// issue at different rates), exp + reciprocal pairs (the sigmoid of the
// network form's activation) and v_mfma_f32_32x32x16_bf16.  It is a
// measurement aid for the roofline denominators, not part of the library.
// Build and run from the repository root:
//
//   hipcc -x hip -O3 -std=c++17 --offload-arch=gfx950 -Xclang -target-feature \
//         -Xclang -packed-fp32-ops peaks_probe.hip -o _build/peaks_probe
//   ./_build/peaks_probe
//
// It prints one line per rate (best of three launches, HIP events).
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                              \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));               \
            std::exit(1);                                                                     \
        }                                                                                     \
    } while (0)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ void copy_kernel(const float4 *__restrict__ src, float4 *__restrict__ dst, long n) {
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Every block reads the whole buffer of n float4 `reps` times, starting at a
// block-dependent offset, so that a CU streams far more than its L1 holds
// and every access is served by the level of the hierarchy that holds the
// buffer (L2 when it fits an XCD's 4 MB L2, the last-level cache when it
// fits its 256 MB).  The sum keeps the loads alive.
template <int U>
__global__ void __launch_bounds__(256) read_kernel(const float4 *__restrict__ src, long n, int reps,
                                                   float *__restrict__ out) {
    float a[U];
    for (int u = 0; u < U; ++u) a[u] = 0.0f;
    const long start = ((long)blockIdx.x * 7919) % n;
    const long b = blockDim.x;
    for (int r = 0; r < reps; ++r) {
        // U independent loads in flight per thread
        for (long i = threadIdx.x; i + (U - 1) * b < n; i += U * b) {
            float4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                long k = start + i + u * b;
                k -= k >= n ? n : 0;
                v[u] = src[k];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] += v[u].x + v[u].y + v[u].z + v[u].w;
        }
    }
    float t = 0.0f;
    for (int u = 0; u < U; ++u) t += a[u];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

constexpr int CHAINS = 16;
// lane 0 of block 0 also records the shader-clock and the constant 100 MHz
// real-time counters around its loop (clk[0], clk[1]), giving the clock the
// FMA stream actually ran at
__global__ void __launch_bounds__(256) fma_kernel(float *out, int iters, float s, long long *clk) {
    const long long c0 = clock64(), r0 = wall_clock64();
    float a[CHAINS];
    for (int k = 0; k < CHAINS; ++k) a[k] = threadIdx.x * 1e-3f + k;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
            for (int k = 0; k < CHAINS; ++k) a[k] = fmaf(a[k], s, 0.5f);  // independent chains
    float t = 0.0f;
    for (int k = 0; k < CHAINS; ++k) t += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clk[0] = clock64() - c0;
        clk[1] = wall_clock64() - r0;
    }
}

// the same chains with every operand in a vector register (per-lane
// multiplier and addend), as in the transform's own arithmetic
__global__ void __launch_bounds__(256) fma_vgpr_kernel(float *out, int iters, float s) {
    float a[CHAINS], b[CHAINS], c[CHAINS];
    for (int k = 0; k < CHAINS; ++k) {
        a[k] = threadIdx.x * 1e-3f + k;
        b[k] = s + 1e-7f * (float)((threadIdx.x & 7) * k);
        c[k] = 0.5f + 1e-3f * (float)((threadIdx.x & 3) * k);
    }
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
            for (int k = 0; k < CHAINS; ++k) a[k] = fmaf(a[k], b[k], c[k]);
    float t = 0.0f;
    for (int k = 0; k < CHAINS; ++k) t += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

__global__ void __launch_bounds__(256) sigmoid_kernel(float *out, int iters, float s) {
    float a[CHAINS];
    for (int k = 0; k < CHAINS; ++k) a[k] = threadIdx.x * 1e-3f + k * 1e-2f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int k = 0; k < CHAINS; ++k) a[k] = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(a[k] * s));
    float t = 0.0f;
    for (int k = 0; k < CHAINS; ++k) t += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

__global__ void __launch_bounds__(256) mfma_kernel(float *out, int iters) {
    const int lane = threadIdx.x & 63;
    bf16x8 A, B;
    for (int k = 0; k < 8; ++k) {
        A[k] = (__bf16)(1e-3f * (lane + k));
        B[k] = (__bf16)(1e-3f * (lane - k));
    }
    f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int it = 0; it < iters; ++it) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, c3, 0, 0, 0);
    }
    float t = 0.0f;
    for (int k = 0; k < 16; ++k) t += c0[k] + c1[k] + c2[k] + c3[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

template <class F>
static float best_ms(F launch) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        CHECK(hipEventRecord(e0));
        launch();
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.0f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) best = ms;
    }
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return best;
}

int main() {
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const double simds = 4.0 * cus, clk = 2.4e9;  // MI355X peak engine clock
    std::printf("device %s, %d compute units, %d MHz reported clock\n", prop.gcnArchName, cus, prop.clockRate / 1000);

    const long bytes = 1L << 30, n4 = bytes / 16;
    float4 *src = nullptr, *dst = nullptr;
    CHECK(hipMalloc(&src, bytes));
    CHECK(hipMalloc(&dst, bytes));
    CHECK(hipMemset(src, 0, bytes));
    const float tc = best_ms([&] { copy_kernel<<<cus * 16, 256>>>(src, dst, n4); });
    std::printf("copy 1 GiB: %.3f ms, %.0f GB/s (read + write)\n", tc, 2.0 * bytes / (tc * 1e-3) / 1e9);
    CHECK(hipFree(src));
    CHECK(hipFree(dst));

    // cache-resident reads: 2 MiB (fits each XCD's L2) and 128 MiB (fits the
    // last-level cache, not the L2); one warm-up pass brings the buffer in
    {
        float *rout = nullptr;
        const int rblocks = cus * 8;
        CHECK(hipMalloc(&rout, sizeof(float) * rblocks * 256));
        for (long mib : {2L, 128L}) {
            const long rb = mib << 20, rn = rb / 16;
            float4 *buf = nullptr;
            CHECK(hipMalloc(&buf, rb));
            CHECK(hipMemset(buf, 0, rb));
            const int reps = mib <= 2 ? 8 : 1;
            const int nblk = rblocks;
            read_kernel<4><<<nblk, 256>>>(buf, rn, 1, rout);
            const float t4 = best_ms([&] { read_kernel<4><<<nblk, 256>>>(buf, rn, reps, rout); });
            const float t8 = best_ms([&] { read_kernel<8><<<nblk, 256>>>(buf, rn, reps, rout); });
            const double moved = (double)nblk * reps * rb;
            std::printf("read %ld MiB buffer, %d blocks x %d passes: 4 loads in flight %.3f ms, %.0f GB/s; "
                        "8 in flight %.3f ms, %.0f GB/s\n", mib, nblk, reps, t4, moved / (t4 * 1e-3) / 1e9, t8,
                        moved / (t8 * 1e-3) / 1e9);
            CHECK(hipFree(buf));
        }
        CHECK(hipFree(rout));
    }

    const int blocks = cus * 8, threads = 256;
    float *out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * blocks * threads));
    const double waves = (double)blocks * threads / 64;
    const int fit = 2000;
    long long *dclk = nullptr, hclk[2] = {0, 0};
    CHECK(hipMalloc(&dclk, sizeof(hclk)));
    const float tf = best_ms([&] { fma_kernel<<<blocks, threads>>>(out, fit, 0.999f, dclk); });
    CHECK(hipMemcpy(hclk, dclk, sizeof(hclk), hipMemcpyDeviceToHost));
    CHECK(hipFree(dclk));
    const double fmas = waves * fit * 16 * CHAINS;
    const double ghz = hclk[1] > 0 ? 0.1 * (double)hclk[0] / (double)hclk[1] : 0.0;  // real-time counter: 100 MHz
    std::printf("fp32 fma (non-packed), scalar-register operand: %.3f ms, %.3f wave instructions per SIMD per cycle "
                "at 2.4 GHz, %.1f TFLOP/s; shader clock during the loop %.2f GHz (%.3f per cycle at that clock)\n",
                tf, fmas / (simds * clk * tf * 1e-3), fmas * 64 * 2 / (tf * 1e-3) / 1e12, ghz,
                ghz > 0 ? fmas / (simds * ghz * 1e9 * tf * 1e-3) : 0.0);
    // at most eight, and at most four, waves per SIMD: the same blocks, four
    // of them per CU when each asks for 38 KiB of (unused) LDS
    for (int lds : {0, 38 * 1024}) {
        const float tv = best_ms([&] { fma_vgpr_kernel<<<blocks, threads, lds>>>(out, fit, 0.999f); });
        std::printf("fp32 fma (non-packed), vector-register operands only, %d waves per SIMD: %.3f ms, %.3f wave "
                    "instructions per SIMD per cycle at 2.4 GHz, %.1f TFLOP/s\n",
                    lds ? 4 : 8, tv, fmas / (simds * clk * tv * 1e-3), fmas * 64 * 2 / (tv * 1e-3) / 1e12);
    }
    const int sit = 500;
    const float ts = best_ms([&] { sigmoid_kernel<<<blocks, threads>>>(out, sit, 0.7f); });
    const double trans = waves * sit * 8 * CHAINS * 2;
    std::printf("exp + rcp: %.3f ms, %.3f wave transcendentals per SIMD per cycle, %.2f T lane results/s\n", ts,
                trans / (simds * clk * ts * 1e-3), trans * 64 / (ts * 1e-3) / 1e12);
    const int mit = 2000;
    const float tm = best_ms([&] { mfma_kernel<<<blocks, threads>>>(out, mit); });
    const double mflop = waves * mit * 4 * (2.0 * 32 * 32 * 16);
    std::printf("mfma 32x32x16 bf16: %.3f ms, %.1f TFLOP/s\n", tm, mflop / (tm * 1e-3) / 1e12);
    CHECK(hipFree(out));
    return 0;
}
