// ss_mlp.hip -- the learned footprint f_theta (Sec. 2.2) on gfx950 matrix cores.
//
// Network: 5 -> 64 -> 64 -> 64 -> 64 -> 1, SiLU after each hidden layer.
// Precision split: fold, frame and layer 1 in FP32 (layer 1 on the FP32
// matrix core, v_mfma_f32_32x32x2_f32); the three 64x64 layers on the BF16
// matrix core with FP32 accumulation (v_mfma_f32_32x32x16_bf16); SiLU in
// FP32; an activation feeding a BF16 layer is carried as the sum of two BF16
// numbers (its rounding to nearest even and the rounding of the remainder),
// so each such layer is two BF16 products into one FP32 accumulator and the
// activations keep about 16 significant bits; output layer in FP32.  The network value is multiplied by the indicator
// that the line meets the basis support (exact slab test), so the pair set
// equals the quadrature form's.
//
// Tile layout.  A wave evaluates 32 (line, basis) pairs at a time, pairs
// along the N (column) dimension of the MFMA.  The 32x32 accumulator of an
// MFMA puts column j in lanes j and j + 32; lane l, register r holds row
// 8 (r / 4) + 4 (l / 32) + (r % 4).  The next layer's B operand needs, in
// lane l, the K slots 8 (l / 32) + e (e < 8) of each 16-wide K step.  The
// hidden units are therefore renumbered so that K step kk of a layer reads
// accumulator block kk / 2, registers 8 (kk % 2) + e of the *same* lane: the
// K slot 16 kk + 8 h + e holds unit 16 kk + 8 (e / 4) + 4 h + (e % 4).  The
// weight image (built on the host from the blob) bakes this permutation
// into the A operands, so activations never leave their lane.
#include "ss_kernels.hpp"

#include <cstring>

namespace ss {

constexpr int HID = 64;

// Weight image, kept in LDS by the kernels (27.4 KB).
struct MlpImage {
    float w1a[2][3][64];       // layer-1 A operand: [row block][K step][lane]
    float bias[4][2][32];      // [layer][lane half][block * 16 + reg]
    uint32_t wh[3][2][4][64][4];  // hidden A operands: 8 bf16 per lane
    float wout[2][32];         // [lane half][block * 16 + reg]
    float bout;
    float pad[3];
};

// accumulator (block b, register r) of lane half hf -> hidden unit
__host__ __device__ constexpr int acc_unit(int b, int r, int hf) { return 32 * b + 8 * (r / 4) + 4 * hf + (r % 4); }
// K slot of a hidden layer's input -> hidden unit
__host__ __device__ constexpr int kslot_unit(int ks) {
    return 16 * (ks / 16) + 8 * ((ks % 8) / 4) + 4 * ((ks % 16) / 8) + (ks % 4);
}

namespace {

struct BlobHeader {
    char magic[8];
    uint32_t version, degree, in, hidden, depth, act, fold, seed;
    float rel_fp32, rel_bf16;
};
static_assert(sizeof(BlobHeader) == 48, "blob header layout");

constexpr size_t BLOB_BODY = 4 * (HID * 5 + HID) + 3 * (2 * HID * HID + 4 * HID) + 4 * (HID + 1);

}  // namespace

// The kernels carry every hidden pre-activation z as A = -log2(e) z, so that
// the SiLU of z is -ln(2) s(A) with s(A) = A / (1 + 2^A): one exp2, one add,
// one reciprocal and one multiply.  Since ln(2) log2(e) = 1, a hidden layer
// maps s(A) to the next A with its own weights and its bias times
// -log2(e); layer 1 takes W1 and b1 times -log2(e), the output layer its
// weights times -ln(2).  The BF16 hidden weights are unchanged.
constexpr double NEG_LOG2E = -1.4426950408889634074;
constexpr double NEG_LN2 = -0.69314718055994530942;
static float scaled(float v, double f) { return (float)((double)v * f); }

ss_status mlp_blob_to_image(const void *blob, size_t bytes, int degree, std::vector<unsigned char> &image) {
    if (bytes != sizeof(BlobHeader) + BLOB_BODY)
        return fail(SS_EBLOB, "weight blob has %zu bytes, expected %zu", bytes, sizeof(BlobHeader) + BLOB_BODY);
    BlobHeader hd;
    std::memcpy(&hd, blob, sizeof hd);
    static const char MAGIC[8] = {'S', 'S', 'M', 'L', 'P', 0, 0, 1};
    if (std::memcmp(hd.magic, MAGIC, 8) != 0) return fail(SS_EBLOB, "weight blob: bad magic");
    if (hd.version != 1) return fail(SS_EBLOB, "weight blob: version %u, expected 1", hd.version);
    if ((int)hd.degree != degree)
        return fail(SS_EBLOB, "weight blob trained for degree %u, context has degree %d", hd.degree, degree);
    if (hd.in != 5 || hd.hidden != HID || hd.depth != 4 || hd.act != 1 || hd.fold != 1)
        return fail(SS_EBLOB, "weight blob: unsupported architecture (in %u hidden %u depth %u act %u fold %u)",
                    hd.in, hd.hidden, hd.depth, hd.act, hd.fold);
    const unsigned char *p = (const unsigned char *)blob + sizeof(BlobHeader);
    float W1[HID][5], b1[HID], bh[3][HID], wo[HID], bo;
    uint16_t Wh[3][HID][HID];
    std::memcpy(W1, p, sizeof W1); p += sizeof W1;
    std::memcpy(b1, p, sizeof b1); p += sizeof b1;
    for (int l = 0; l < 3; ++l) {
        std::memcpy(Wh[l], p, sizeof Wh[l]); p += sizeof Wh[l];
        std::memcpy(bh[l], p, sizeof bh[l]); p += sizeof bh[l];
    }
    std::memcpy(wo, p, sizeof wo); p += sizeof wo;
    std::memcpy(&bo, p, sizeof bo);
    for (int u = 0; u < HID; ++u) {
        for (int k = 0; k < 5; ++k)
            if (!std::isfinite(W1[u][k])) return fail(SS_EBLOB, "weight blob: non-finite layer-1 weight");
        if (!std::isfinite(b1[u]) || !std::isfinite(wo[u])) return fail(SS_EBLOB, "weight blob: non-finite value");
    }
    if (!std::isfinite(bo)) return fail(SS_EBLOB, "weight blob: non-finite output bias");
    MlpImage im;
    std::memset(&im, 0, sizeof im);
    for (int b = 0; b < 2; ++b)
        for (int kk = 0; kk < 3; ++kk)
            for (int l = 0; l < 64; ++l) {
                const int unit = 32 * b + (l % 32), feat = 2 * kk + l / 32;
                im.w1a[b][kk][l] = feat < 5 ? scaled(W1[unit][feat], NEG_LOG2E) : 0.0f;
            }
    for (int hf = 0; hf < 2; ++hf)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 16; ++r) {
                const int u = acc_unit(b, r, hf);
                im.bias[0][hf][b * 16 + r] = scaled(b1[u], NEG_LOG2E);
                for (int l = 0; l < 3; ++l) im.bias[l + 1][hf][b * 16 + r] = scaled(bh[l][u], NEG_LOG2E);
                im.wout[hf][b * 16 + r] = scaled(wo[u], NEG_LN2);
            }
    for (int l = 0; l < 3; ++l)
        for (int b = 0; b < 2; ++b)
            for (int kk = 0; kk < 4; ++kk)
                for (int ln = 0; ln < 64; ++ln) {
                    const int out = 32 * b + (ln % 32);
                    uint16_t v[8];
                    for (int e = 0; e < 8; ++e) v[e] = Wh[l][out][kslot_unit(16 * kk + 8 * (ln / 32) + e)];
                    std::memcpy(im.wh[l][b][kk][ln], v, sizeof v);
                }
    im.bout = bo;
    image.resize(sizeof im);
    std::memcpy(image.data(), &im, sizeof im);
    return SS_OK;
}

// ---------------------------------------------------------------------------
// Device side
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x8 __attribute__((ext_vector_type(8)));

// s(A) = A / (1 + 2^A) for A = -log2(e) z: the SiLU of z is -ln(2) s(A),
// the factor being folded into the next layer's weights (see the image)
__device__ __forceinline__ float silu(float a) { return a * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(a)); }

// Copy the weight image into LDS (all threads of the block take part).
__device__ __forceinline__ void load_image(MlpImage &dst, const MlpImage *__restrict__ src) {
    const uint4 *s = reinterpret_cast<const uint4 *>(src);
    uint4 *d = reinterpret_cast<uint4 *>(&dst);
    constexpr int n16 = sizeof(MlpImage) / 16;
    for (int i = threadIdx.x; i < n16; i += blockDim.x) d[i] = s[i];
}

// Network value for the 32 pairs whose features sit in lanes base .. base+31
// (f0..f4 of each lane).  Every lane of the wave must be active.  Returns,
// in lanes l and l + 32, the value of the pair of lane base + (l % 32).
__device__ __forceinline__ float mlp_tile(const MlpImage &W, float f0, float f1, float f2, float f3, float f4,
                                          int base) {
    const int lane = threadIdx.x & 63, hf = lane >> 5, src = base + (lane & 31);
    // layer-1 B operand: feature 2 kk + hf of the pair
    float bop[3];
    {
        const float a0 = __shfl(f0, src), a1 = __shfl(f1, src), a2 = __shfl(f2, src);
        const float a3 = __shfl(f3, src), a4 = __shfl(f4, src);
        bop[0] = hf ? a1 : a0;
        bop[1] = hf ? a3 : a2;
        bop[2] = hf ? 0.0f : a4;
    }
    f32x16 acc0, acc1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        acc0[r] = W.bias[0][hf][r];
        acc1[r] = W.bias[0][hf][16 + r];
    }
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(W.w1a[0][kk][lane], bop[kk], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(W.w1a[1][kk][lane], bop[kk], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int L = 0; L < 3; ++L) {
        // each activation as the sum of two BF16 numbers: hi = RNE(a),
        // lo = RNE(a - hi); the layer is W hi + W lo in one FP32 accumulator
        bf16x8 Bh[4], Bl[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            f32x8 v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = silu(kk < 2 ? acc0[8 * kk + e] : acc1[8 * (kk - 2) + e]);
            Bh[kk] = __builtin_convertvector(v, bf16x8);
            const f32x8 back = __builtin_convertvector(Bh[kk], f32x8);
            Bl[kk] = __builtin_convertvector(v - back, bf16x8);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc0[r] = W.bias[L + 1][hf][r];
            acc1[r] = W.bias[L + 1][hf][16 + r];
        }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const bf16x8 A0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(W.wh[L][0][kk][lane]));
            const bf16x8 A1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(W.wh[L][1][kk][lane]));
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0, Bh[kk], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, Bh[kk], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0, Bl[kk], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, Bl[kk], acc1, 0, 0, 0);
        }
    }
    float part = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        part = fmaf(silu(acc0[r]), W.wout[hf][r], part);
        part = fmaf(silu(acc1[r]), W.wout[hf][16 + r], part);
    }
    part += __shfl_xor(part, 32);
    return part + W.bout;
}

// Both tiles of a wave: each lane gets the value of its own pair.  The two
// independent tiles are left to the scheduler, which interleaves one tile's
// matrix-core work with the other's SiLU (24 views of cone_256: forward
// 1,263 against 1,485 ms with a scheduling barrier between the tiles; the
// adjoint, whose candidate state then spills, 1,237 against 1,394 ms).
__device__ __forceinline__ float mlp_wave(const MlpImage &W, const float f[5]) {
    const int lane = threadIdx.x & 63;
    const float ra = mlp_tile(W, f[0], f[1], f[2], f[3], f[4], 0);
    const float rb = mlp_tile(W, f[0], f[1], f[2], f[3], f[4], 32);
    return lane < 32 ? ra : rb;
}

// Fold convention 1 for one line: sort |w| ascending (lower axis first on
// ties); wf = sorted |w|; u = normalise(e1 - wf1 wf), v = u x wf; U, V are u
// and v carried back to world axes, so that u . (Q x) = U . x.
struct Fold {
    float wf[3];
    float U[3], V[3];
};

__device__ __forceinline__ Fold make_fold(const double w[3]) {
    const double a[3] = {fabs(w[0]), fabs(w[1]), fabs(w[2])};
    // stable ascending order of (a0, a1, a2)
    int p0 = 0, p1 = 1, p2 = 2;
    if (a[1] < a[0]) { p0 = 1; p1 = 0; }
    {
        // insert axis 2
        const double ap0 = pick3(a, p0), ap1 = pick3(a, p1);
        if (a[2] < ap0) { p2 = p1; p1 = p0; p0 = 2; }
        else if (a[2] < ap1) { p2 = p1; p1 = 2; }
    }
    const int P[3] = {p0, p1, p2};
    double wf[3], sg[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        wf[k] = pick3(a, P[k]);
        sg[k] = pick3(w, P[k]) < 0.0 ? -1.0 : 1.0;
    }
    double u[3] = {1.0 - wf[0] * wf[0], -wf[0] * wf[1], -wf[0] * wf[2]};
    const double un = 1.0 / sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] *= un;
    const double v[3] = {u[1] * wf[2] - u[2] * wf[1], u[2] * wf[0] - u[0] * wf[2], u[0] * wf[1] - u[1] * wf[0]};
    Fold F;
    double Ud[3] = {0.0, 0.0, 0.0}, Vd[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double uk = u[k] * sg[k], vk = v[k] * sg[k];
        Ud[0] += P[k] == 0 ? uk : 0.0; Ud[1] += P[k] == 1 ? uk : 0.0; Ud[2] += P[k] == 2 ? uk : 0.0;
        Vd[0] += P[k] == 0 ? vk : 0.0; Vd[1] += P[k] == 1 ? vk : 0.0; Vd[2] += P[k] == 2 ? vk : 0.0;
        F.wf[k] = (float)wf[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) { F.U[k] = (float)Ud[k]; F.V[k] = (float)Vd[k]; }
    return F;
}

// ---------------------------------------------------------------------------
// Forward, network form.  Same slab walk and windows as the quadrature
// kernel, written as a resumable iterator: each round every lane advances to
// its next (line, basis) pair with a non-empty chord, the wave evaluates the
// 64 pairs on the matrix cores, and each lane accumulates c_q * f_theta.
// ---------------------------------------------------------------------------
template <int n>
struct Walk {
    double A1, A2, r1, r2, H1, H2;
    int j, j1, N1, N2, lo1, hi1, hi2, q1, q2;
    int64_t sd, s1, s2;  // strides of axes d, i1, i2

    __device__ __forceinline__ void window() {
        const double P1 = fma((double)j, r1, A1), P2 = fma((double)j, r2, A2);
        lo1 = (int)fmin(fmax(floor(P1 - H1) + 1.0, 0.0), (double)N1);
        hi1 = (int)fmax(fmin(ceil(P1 + H1) - 1.0, (double)(N1 - 1)), -1.0);
        q2 = (int)fmin(fmax(floor(P2 - H2) + 1.0, 0.0), (double)N2);
        hi2 = (int)fmax(fmin(ceil(P2 + H2) - 1.0, (double)(N2 - 1)), -1.0);
        q1 = lo1;
    }
    // current candidate is (j, q1, q2) when valid() holds
    __device__ __forceinline__ bool valid() const { return j <= j1 && q1 <= hi1 && q2 <= hi2; }
    __device__ __forceinline__ bool done() const { return j > j1; }
    __device__ __forceinline__ void advance() {
        ++q1;
        if (q1 > hi1) {
            q1 = lo1;
            ++q2;
            if (q2 > hi2 || lo1 > hi1) {
                ++j;
                if (j <= j1) window();
            }
        }
    }
};

template <int n>
__device__ __forceinline__ void walk_init(Walk<n> &W, const LineD &L, const int N[3], int &d, int &i1, int &i2) {
    constexpr double h = (double)Degree<n>::h;
    dominant_axis(L.w, d, i1, i2);
    const double wd = pick3(L.w, d);
    W.r1 = pick3(L.w, i1) / wd;
    W.r2 = pick3(L.w, i2) / wd;
    const double o[3] = {-0.5 * (N[0] - 1), -0.5 * (N[1] - 1), -0.5 * (N[2] - 1)};
    const double ad = pick3(L.a, d) - pick3(o, d);
    W.A1 = (pick3(L.a, i1) - pick3(o, i1)) - ad * W.r1;
    W.A2 = (pick3(L.a, i2) - pick3(o, i2)) - ad * W.r2;
    W.H1 = h * (1.0 + fabs(W.r1));
    W.H2 = h * (1.0 + fabs(W.r2));
    const int Nd = pick3(N, d);
    W.N1 = pick3(N, i1);
    W.N2 = pick3(N, i2);
    double jlo = 0.0, jhi = (double)(Nd - 1);
    const double rr[2] = {W.r1, W.r2}, AA[2] = {W.A1, W.A2}, HH[2] = {W.H1, W.H2};
    const int NN[2] = {W.N1, W.N2};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double lo = -HH[k] - AA[k], hi = (double)(NN[k] - 1) + HH[k] - AA[k];
        if (rr[k] == 0.0) {
            if (!(lo < 0.0 && hi > 0.0)) jhi = -1.0;
        } else {
            const double ta = lo / rr[k], tb = hi / rr[k];
            jlo = fmax(jlo, floor(fmin(ta, tb)));
            jhi = fmin(jhi, ceil(fmax(ta, tb)));
        }
    }
    W.j = (int)fmin(fmax(jlo, 0.0), (double)Nd);
    W.j1 = (int)fmax(fmin(jhi, (double)(Nd - 1)), -1.0);
    const int64_t strides[3] = {1, (int64_t)N[0], (int64_t)N[0] * N[1]};
    W.sd = pick3(strides, d);
    W.s1 = pick3(strides, i1);
    W.s2 = pick3(strides, i2);
    if (W.j <= W.j1) W.window();
}

// The network forward's pairs waiting to be evaluated, a ring of 128 per
// wave: the five features, the coefficient's index and the owning lane.
constexpr int FBUF = 128;
struct FwdPairBuf {
    float f[5][FBUF];
    int idx_lo[FBUF], idx_hi[FBUF];
    int owner[FBUF];
};

// The slab walk of one line per lane, with the footprint of each (line,
// basis) pair it yields taken from the network (EXACT = false) or from the
// exact piecewise Gauss-Legendre integral (EXACT = true: every round each
// lane evaluates its own next pair).  The exact variant is the reference
// point of the network: the same walk, windows and pair gating, only the
// footprint differs.  In the network variant each lane appends the pairs it
// finds to its wave's ring; whenever 64 are buffered the wave evaluates
// them on the matrix cores, one pair per lane, and adds c times the
// footprint to the owning lane's sum in LDS (atomic adds within the wave),
// so rounds stay full while some lines of the wave are done and others are
// not (about 6 % empty slots at cone_256 when each lane evaluated its own
// pairs).
template <int n, bool EXACT>
__device__ __forceinline__ void project_walk(const float *__restrict__ c, int N0, int N1, int N2,
                                             const float *__restrict__ geom, int kind, int V, int R, int C,
                                             const MlpImage *Wt, float *__restrict__ y, int v, int tr, int tc,
                                             FwdPairBuf *fbuf = nullptr, float *accw = nullptr) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = tr * 16 + (wave >> 1) * 8 + (lane >> 3);
    const int i = tc * 16 + (wave & 1) * 8 + (lane & 7);
    const bool pix = v < V && j < R && i < C;
    const int N[3] = {N0, N1, N2};
    const double centre[3] = {0.0, 0.0, 0.0};
    LineD L;
    L.ok = false;
    if (pix) L = make_line(geom + 12 * v, kind, R, C, j, i, centre);
    Walk<n> Wk;
    int d = 0, i1 = 1, i2 = 2;
    Fold F;
    Slopes S;
    float inv_wd = 0.0f;
    bool live = false;
    if (L.ok) {
        walk_init<n>(Wk, L, N, d, i1, i2);
        F = make_fold(L.w);
        S = make_slopes((float)Wk.r1, (float)Wk.r2);
        inv_wd = (float)(1.0 / fabs(pick3(L.w, d)));
        live = !Wk.done();
    } else {
        F = Fold{};
        S = make_slopes(0.0f, 0.0f);
    }
    const float Ui1 = pick3(F.U, i1), Ui2 = pick3(F.U, i2), Vi1 = pick3(F.V, i1), Vi2 = pick3(F.V, i2);
    float acc = 0.0f;
    int head = 0, wcount = 0;  // network form, wave-uniform: oldest buffered pair, how many
    if constexpr (!EXACT) {
        FwdPairBuf &B = fbuf[wave];
        accw[threadIdx.x] = 0.0f;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            B.f[q][lane] = 0.0f;
            B.f[q][lane + 64] = 0.0f;
        }
        B.idx_lo[lane] = B.idx_lo[lane + 64] = 0;
        B.idx_hi[lane] = B.idx_hi[lane + 64] = 0;
        B.owner[lane] = B.owner[lane + 64] = lane;
    }
    // network form: evaluate the cnt oldest buffered pairs (wave-uniform
    // cnt <= 64, every lane taking part) and add c times the footprint to
    // the owners' sums
    auto flush = [&](int cnt) {
        if constexpr (!EXACT) {
            const FwdPairBuf &B = fbuf[wave];
            const int e = (head + lane) & (FBUF - 1);
            const float f[5] = {B.f[0][e], B.f[1][e], B.f[2][e], B.f[3][e], B.f[4][e]};
            const int64_t idx = (int64_t)(((uint64_t)(uint32_t)B.idx_hi[e] << 32) | (uint32_t)B.idx_lo[e]);
            const int own = B.owner[e];
            const float cv = lane < cnt ? c[idx] : 0.0f;
            const float fp = mlp_wave(*Wt, f);
            if (lane < cnt)
                __hip_atomic_fetch_add(&accw[(threadIdx.x & ~63) + own], cv * fp, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };
    while (true) {
        bool have = false;
        float u1 = 0.0f, u2 = 0.0f;
        int64_t idx = 0;
        while (live && !have) {
            if (Wk.valid()) {
                const double P1 = fma((double)Wk.j, Wk.r1, Wk.A1), P2 = fma((double)Wk.j, Wk.r2, Wk.A2);
                u1 = (float)(P1 - (double)Wk.q1);
                u2 = (float)(P2 - (double)Wk.q2);
                if (chord_nonempty<n>(S, u1, u2)) {
                    have = true;
                    idx = (int64_t)Wk.j * Wk.sd + (int64_t)Wk.q1 * Wk.s1 + (int64_t)Wk.q2 * Wk.s2;
                }
            }
            Wk.advance();
            live = !Wk.done();
        }
        const uint64_t m = __ballot(have);
        if (m == 0) break;
        if constexpr (EXACT) {
            const float fp = have ? footprint_slab<n>(S, u1, u2) * inv_wd : 0.0f;
            if (have) acc = fmaf(c[idx], fp, acc);
        } else {
            if (have) {
                FwdPairBuf &B = fbuf[wave];
                const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const int slot = (head + wcount + rank) & (FBUF - 1);
                B.f[0][slot] = F.wf[0];
                B.f[1][slot] = F.wf[1];
                B.f[2][slot] = F.wf[2];
                B.f[3][slot] = fmaf(Ui1, u1, Ui2 * u2);
                B.f[4][slot] = fmaf(Vi1, u1, Vi2 * u2);
                B.idx_lo[slot] = (int)(uint32_t)idx;
                B.idx_hi[slot] = (int)(uint32_t)((uint64_t)idx >> 32);
                B.owner[slot] = lane;
            }
            wcount += __popcll(m);
            if (wcount >= 64) {
                flush(64);
                head = (head + 64) & (FBUF - 1);
                wcount -= 64;
            }
        }
    }
    if constexpr (!EXACT) {
        if (wcount > 0) flush(wcount);
        acc = accw[threadIdx.x];
    }
    if (pix) y[((int64_t)v * R + j) * C + i] = acc;
}

// two workgroups (eight waves) per CU: one wave's matrix-core layers overlap
// another's SiLU
template <int n>
__global__ void __launch_bounds__(256, 2) project_mlp_kernel(const float *__restrict__ c, int N0, int N1, int N2,
                                                          const float *__restrict__ geom, int kind, int V, int R,
                                                          int C, const MlpImage *__restrict__ img,
                                                          float *__restrict__ y) {
    __shared__ MlpImage Wt;
    __shared__ FwdPairBuf fbuf[4];  // one ring per wave of the 256-thread block
    __shared__ float accw[256];
    const int tR = (R + 15) / 16, tC = (C + 15) / 16;
    int v, tr, tc;
    if (!fwd_block_tile(V, tR, tC, v, tr, tc)) return;  // padding slot: the whole block
    load_image(Wt, img);
    __syncthreads();
    project_walk<n, false>(c, N0, N1, N2, geom, kind, V, R, C, &Wt, y, v, tr, tc, fbuf, accw);
}

template <int n>
__global__ void __launch_bounds__(256) project_pair_kernel(const float *__restrict__ c, int N0, int N1, int N2,
                                                           const float *__restrict__ geom, int kind, int V, int R,
                                                           int C, float *__restrict__ y) {
    const int tR = (R + 15) / 16, tC = (C + 15) / 16;
    int v, tr, tc;
    if (!fwd_block_tile(V, tR, tC, v, tr, tc)) return;  // padding slot: the whole block
    project_walk<n, true>(c, N0, N1, N2, geom, kind, V, R, C, nullptr, y, v, tr, tc);
}

// ---------------------------------------------------------------------------
// Adjoint, network form: the brick gather of the quadrature kernel with the
// per-line fold data added to the LDS table.
// ---------------------------------------------------------------------------
constexpr int MBX = 8, MBY = 8, MBZ = 4;
constexpr int MRAY_CAP = 384;
constexpr float MPIX_MARGIN = 1.0e-3f;  // pixels

struct RayRecM {     // 80 bytes
    float a[3];      // point of the line nearest the brick centre, relative to it
    float r1, r2, ir1, ir2;
    float y;
    float wf[3];
    float U[3], V[3];
    int d;
    float iwd;       // 1 / |w_d|
    float pad;
};

// The network adjoint's pairs waiting to be evaluated, a ring of 128 per
// wave: the five features and y of each pair and its owning thread.  A wave
// appends only its own lanes' pairs, so each ring is used by one wave.
constexpr int PBUF = 128;
struct PairBuf {
    float v[6][PBUF];
    int owner[PBUF];
};

template <int n>
__device__ __forceinline__ void fill_ray_m(RayRecM &rec, const float *__restrict__ e, int kind, int R, int C,
                                           int j, int i, const double centre[3], float yval) {
    const LineD L = make_line(e, kind, R, C, j, i, centre);
    int d, i1, i2;
    dominant_axis(L.w, d, i1, i2);
    const double wd = pick3(L.w, d);
    const Slopes S = make_slopes((float)(pick3(L.w, i1) / wd), (float)(pick3(L.w, i2) / wd));
    rec.a[0] = (float)(L.a[0] - centre[0]);
    rec.a[1] = (float)(L.a[1] - centre[1]);
    rec.a[2] = (float)(L.a[2] - centre[2]);
    rec.r1 = S.r1; rec.r2 = S.r2; rec.ir1 = S.ir1; rec.ir2 = S.ir2;
    rec.y = L.ok ? yval : 0.0f;
    const Fold F = make_fold(L.w);
#pragma unroll
    for (int k = 0; k < 3; ++k) { rec.wf[k] = F.wf[k]; rec.U[k] = F.U[k]; rec.V[k] = F.V[k]; }
    rec.d = d;
    rec.iwd = L.ok ? (float)(1.0 / fabs(wd)) : 0.0f;
}

// Coefficient-brick gather: each thread owns one coefficient and sums, view
// by view, y_m times the footprint over the pixels of its support's shadow;
// each lane finds its own pairs (the pixels whose line meets its support).
// The exact form (EXACT = true) evaluates the piecewise Gauss-Legendre
// integral of every lane's next pair in the same round.  The network form
// appends the pairs to its wave's ring and, whenever 64 are buffered,
// evaluates them together on the matrix cores, one pair per lane, adding y
// times the footprint to the owners' sums in LDS (atomic adds within the
// wave, since owner and evaluating lane differ): every round is full, and
// pairs carry over from one chunk or view to the next.
template <int n, bool EXACT>
__device__ __forceinline__ void backproject_gather(const float *__restrict__ y, int N0, int N1, int N2,
                                                   const float *__restrict__ geom, const ViewProj *__restrict__ vps,
                                                   int kind, int V, int R, int C, const MlpImage *Wt,
                                                   RayRecM *rays, ViewProj &vp, LocalProj &lp, int *sbox,
                                                   PairBuf *pbuf, float *accw, float *__restrict__ c) {
    constexpr float hf = Degree<n>::h;
    const int nbx = (N0 + MBX - 1) / MBX, nby = (N1 + MBY - 1) / MBY, nbz = (N2 + MBZ - 1) / MBZ;
    const int b = xcd_remap(blockIdx.x, nbx * nby * nbz);
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int tid = threadIdx.x;
    const int k0 = bx * MBX + (tid % MBX), k1 = by * MBY + ((tid / MBX) % MBY), k2 = bz * MBZ + tid / (MBX * MBY);
    const bool mine = k0 < N0 && k1 < N1 && k2 < N2;
    constexpr double h = (double)Degree<n>::h;
    const double o[3] = {-0.5 * (N0 - 1), -0.5 * (N1 - 1), -0.5 * (N2 - 1)};
    const double centre[3] = {o[0] + bx * MBX + 0.5 * (MBX - 1), o[1] + by * MBY + 0.5 * (MBY - 1),
                              o[2] + bz * MBZ + 0.5 * (MBZ - 1)};
    const float xq[3] = {(float)(o[0] + k0 - centre[0]), (float)(o[1] + k1 - centre[1]),
                         (float)(o[2] + k2 - centre[2])};
    float acc = 0.0f;                 // exact form: this coefficient's sum
    const int lane = tid & 63;
    int head = 0, wcount = 0;         // network form, wave-uniform: oldest buffered pair, how many
    if constexpr (!EXACT) {
        PairBuf &B = pbuf[tid >> 6];
        accw[tid] = 0.0f;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            B.v[q][lane] = 0.0f;
            B.v[q][lane + 64] = 0.0f;
        }
        B.owner[lane] = tid;
        B.owner[lane + 64] = tid;
    }
    // network form: evaluate the cnt oldest buffered pairs (wave-uniform
    // cnt <= 64, every lane of the wave taking part) and add their terms to
    // the owners' sums
    auto flush = [&](int cnt) {
        if constexpr (!EXACT) {
            const PairBuf &B = pbuf[tid >> 6];
            const int e = (head + lane) & (PBUF - 1);
            const float f[5] = {B.v[0][e], B.v[1][e], B.v[2][e], B.v[3][e], B.v[4][e]};
            const float yv = B.v[5][e];
            const int own = B.owner[e];
            const float fp = mlp_wave(*Wt, f);
            if (lane < cnt)
                __hip_atomic_fetch_add(&accw[own], yv * fp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };
    for (int v = 0; v < V; ++v) {
        const float *e = geom + 12 * v;
        __syncthreads();
        if (tid == 0) {
            vp = vps[v];
            make_localproj(vp, centre, lp);
            double lo[3], hi[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int nb = k == 0 ? MBX : k == 1 ? MBY : MBZ;
                lo[k] = centre[k] - 0.5 * (nb - 1) - h;
                hi[k] = centre[k] + 0.5 * (nb - 1) + h;
            }
            box_to_pixels(vp, lo, hi, R, C, sbox[0], sbox[1], sbox[2], sbox[3]);
        }
        __syncthreads();
        const int bi0 = sbox[0], bi1 = sbox[1], bj0 = sbox[2], bj1 = sbox[3];
        int mi0 = 0, mi1 = -1, mj0 = 0, mj1 = -1;
        if (mine) {
            // the pixels whose centre lies in the bounding rectangle of the
            // projected corners of this coefficient's support box (FP32
            // offsets from the brick centre; MPIX_MARGIN covers the rounding)
            float cmin = 3.0e38f, cmax = -3.0e38f, rmin = 3.0e38f, rmax = -3.0e38f;
            bool bad = false;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float d[3] = {xq[0] + ((k & 1) ? hf : -hf), xq[1] + ((k & 2) ? hf : -hf),
                                    xq[2] + ((k & 4) ? hf : -hf)};
                float cc, rr;
                if (!local_to_detector(lp, d, cc, rr)) bad = true;
                cmin = fminf(cmin, cc); cmax = fmaxf(cmax, cc);
                rmin = fminf(rmin, rr); rmax = fmaxf(rmax, rr);
            }
            const float oc = 0.5f * (float)(C - 1), orow = 0.5f * (float)(R - 1);
            if (bad) {
                mi0 = 0; mi1 = C - 1; mj0 = 0; mj1 = R - 1;
            } else {
                const float fi0 = fmaxf(ceilf(cmin + oc - MPIX_MARGIN), 0.0f);
                const float fi1 = fminf(floorf(cmax + oc + MPIX_MARGIN), (float)(C - 1));
                const float fj0 = fmaxf(ceilf(rmin + orow - MPIX_MARGIN), 0.0f);
                const float fj1 = fminf(floorf(rmax + orow + MPIX_MARGIN), (float)(R - 1));
                if (fi0 <= fi1 && fj0 <= fj1) {
                    mi0 = (int)fi0; mi1 = (int)fi1; mj0 = (int)fj0; mj1 = (int)fj1;
                }
            }
        }
        const int W = bi1 - bi0 + 1;
        const int rows_per_chunk = W > 0 ? max(1, MRAY_CAP / W) : 1;
        const int cols = min(max(W, 1), MRAY_CAP);
        for (int cj0 = bj0; cj0 <= bj1; cj0 += rows_per_chunk) {
            const int cj1 = min(bj1, cj0 + rows_per_chunk - 1);
            for (int ci0 = bi0; ci0 <= bi1; ci0 += cols) {
                const int ci1 = min(bi1, ci0 + cols - 1);
                const int cw = ci1 - ci0 + 1;
                const int cn = (cj1 - cj0 + 1) * cw;
                __syncthreads();
                for (int t = tid; t < cn; t += blockDim.x) {
                    const int jj = cj0 + t / cw, ii = ci0 + t % cw;
                    fill_ray_m<n>(rays[t], e, kind, R, C, jj, ii, centre, y[((int64_t)v * R + jj) * C + ii]);
                }
                __syncthreads();
                // this thread's pixels inside the chunk, visited row-major
                const int j0 = mine ? max(mj0, cj0) : 1, j1 = mine ? min(mj1, cj1) : 0;
                const int i0 = max(mi0, ci0), i1 = min(mi1, ci1);
                int jj = j0, ii = i0;
                bool live = j0 <= j1 && i0 <= i1;
                if constexpr (EXACT) {
                    // every round each lane with pixels left evaluates its next pair
                    while (true) {
                        bool have = false;
                        float yv = 0.0f, pu1 = 0.0f, pu2 = 0.0f, iwd = 0.0f;
                        Slopes PS = make_slopes(0.0f, 0.0f);
                        while (live && !have) {
                            const RayRecM &rr = rays[(jj - cj0) * cw + (ii - ci0)];
                            const int d = rr.d;
                            const int i1x = d == 0 ? 1 : 0, i2x = d == 2 ? 1 : 2;
                            const float t = pick3(xq, d) - pick3(rr.a, d);
                            const float u1 = fmaf(t, rr.r1, pick3(rr.a, i1x)) - pick3(xq, i1x);
                            const float u2 = fmaf(t, rr.r2, pick3(rr.a, i2x)) - pick3(xq, i2x);
                            Slopes S;
                            S.r1 = rr.r1; S.r2 = rr.r2; S.ir1 = rr.ir1; S.ir2 = rr.ir2;
                            if (chord_nonempty<n>(S, u1, u2)) {
                                have = true;
                                yv = rr.y;
                                pu1 = u1;
                                pu2 = u2;
                                PS = S;
                                iwd = rr.iwd;
                            }
                            ++ii;
                            if (ii > i1) { ii = i0; ++jj; }
                            live = jj <= j1;
                        }
                        if (__ballot(have) == 0) break;
                        const float fp = have ? footprint_slab<n>(PS, pu1, pu2) * iwd : 0.0f;
                        if (have) acc = fmaf(yv, fp, acc);
                    }
                } else {
                    // every round each lane with pixels left finds its next
                    // pair; the found pairs go into the ring (at most 63 + 64)
                    while (true) {
                        bool have = false;
                        float pv[6];
                        while (live && !have) {
                            const RayRecM &rr = rays[(jj - cj0) * cw + (ii - ci0)];
                            const int d = rr.d;
                            const int i1x = d == 0 ? 1 : 0, i2x = d == 2 ? 1 : 2;
                            const float t = pick3(xq, d) - pick3(rr.a, d);
                            const float u1 = fmaf(t, rr.r1, pick3(rr.a, i1x)) - pick3(xq, i1x);
                            const float u2 = fmaf(t, rr.r2, pick3(rr.a, i2x)) - pick3(xq, i2x);
                            Slopes S;
                            S.r1 = rr.r1; S.r2 = rr.r2; S.ir1 = rr.ir1; S.ir2 = rr.ir2;
                            if (chord_nonempty<n>(S, u1, u2)) {
                                have = true;
                                const float x0 = rr.a[0] - xq[0], x1 = rr.a[1] - xq[1], x2 = rr.a[2] - xq[2];
                                pv[0] = rr.wf[0]; pv[1] = rr.wf[1]; pv[2] = rr.wf[2];
                                pv[3] = fmaf(rr.U[0], x0, fmaf(rr.U[1], x1, rr.U[2] * x2));
                                pv[4] = fmaf(rr.V[0], x0, fmaf(rr.V[1], x1, rr.V[2] * x2));
                                pv[5] = rr.y;
                            }
                            ++ii;
                            if (ii > i1) { ii = i0; ++jj; }
                            live = jj <= j1;
                        }
                        const uint64_t m = __ballot(have);
                        if (m == 0) break;  // every lane has exhausted this chunk
                        if (have) {
                            PairBuf &B = pbuf[tid >> 6];
                            const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                            const int slot = (head + wcount + rank) & (PBUF - 1);
#pragma unroll
                            for (int q = 0; q < 6; ++q) B.v[q][slot] = pv[q];
                            B.owner[slot] = tid;
                        }
                        wcount += __popcll(m);
                        if (wcount >= 64) {
                            flush(64);
                            head = (head + 64) & (PBUF - 1);
                            wcount -= 64;
                        }
                    }
                }
            }
        }
    }
    if constexpr (!EXACT) {
        if (wcount > 0) flush(wcount);
        acc = accw[tid];  // the wave's atomic adds precede this read (LDS operations of a wave run in order)
    }
    if (mine) c[((int64_t)k2 * N1 + k1) * N0 + k0] = acc;
}

template <int n>
__global__ void __launch_bounds__(256, 2) backproject_mlp_kernel(const float *__restrict__ y, int N0, int N1, int N2,
                                                              const float *__restrict__ geom,
                                                              const ViewProj *__restrict__ vps, int kind, int V,
                                                              int R, int C, const MlpImage *__restrict__ img,
                                                              float *__restrict__ c) {
    __shared__ MlpImage Wt;
    __shared__ RayRecM rays[MRAY_CAP];
    __shared__ ViewProj vp;
    __shared__ LocalProj lp;
    __shared__ int sbox[4];
    __shared__ PairBuf pbuf[4];  // one ring per wave of the 256-thread block
    __shared__ float accw[256];
    load_image(Wt, img);
    backproject_gather<n, false>(y, N0, N1, N2, geom, vps, kind, V, R, C, &Wt, rays, vp, lp, sbox, pbuf, accw, c);
}

template <int n>
__global__ void __launch_bounds__(256) backproject_pair_kernel(const float *__restrict__ y, int N0, int N1, int N2,
                                                               const float *__restrict__ geom,
                                                               const ViewProj *__restrict__ vps, int kind, int V,
                                                               int R, int C, float *__restrict__ c) {
    __shared__ RayRecM rays[MRAY_CAP];
    __shared__ ViewProj vp;
    __shared__ LocalProj lp;
    __shared__ int sbox[4];
    backproject_gather<n, true>(y, N0, N1, N2, geom, vps, kind, V, R, C, nullptr, rays, vp, lp, sbox, nullptr, nullptr,
                                c);
}

// ---------------------------------------------------------------------------
// Network footprint of arbitrary pairs (diagnostics), one pair per lane.
// ---------------------------------------------------------------------------
template <int n>
__global__ void __launch_bounds__(64) footprint_mlp_kernel(const float *__restrict__ dirs,
                                                           const float *__restrict__ offs, int count,
                                                           const MlpImage *__restrict__ img,
                                                           float *__restrict__ out) {
    __shared__ MlpImage Wt;
    load_image(Wt, img);
    __syncthreads();
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    bool have = false;
    float f[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (k < count) {
        double w[3], x[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) { w[a] = dirs[3 * k + a]; x[a] = offs[3 * k + a]; }
        const double nn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        if (nn > 0.0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) w[a] /= nn;
            int d, i1, i2;
            dominant_axis(w, d, i1, i2);
            const double wd = pick3(w, d);
            const double r1 = pick3(w, i1) / wd, r2 = pick3(w, i2) / wd;
            const Slopes S = make_slopes((float)r1, (float)r2);
            const double xd = pick3(x, d);
            const float u1 = (float)(pick3(x, i1) - xd * r1), u2 = (float)(pick3(x, i2) - xd * r2);
            have = chord_nonempty<n>(S, u1, u2);
            const Fold F = make_fold(w);
            f[0] = F.wf[0]; f[1] = F.wf[1]; f[2] = F.wf[2];
            const float xf[3] = {(float)x[0], (float)x[1], (float)x[2]};
            f[3] = fmaf(F.U[0], xf[0], fmaf(F.U[1], xf[1], F.U[2] * xf[2]));
            f[4] = fmaf(F.V[0], xf[0], fmaf(F.V[1], xf[1], F.V[2] * xf[2]));
        }
    }
    const float fp = mlp_wave(Wt, f);
    if (k < count) out[k] = have ? fp : 0.0f;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int n>
static hipError_t launch_project_mlp_n(const LaunchArgs &a, hipStream_t st) {
    const int tR = (a.R + 15) / 16, tC = (a.C + 15) / 16;
    hipLaunchKernelGGL(project_mlp_kernel<n>, dim3((unsigned)fwd_blocks(tR, tC, a.V)), dim3(256), 0, st, a.coeffs, a.N[0], a.N[1],
                       a.N[2], a.geom, a.kind, a.V, a.R, a.C, (const MlpImage *)a.mlp, a.sino);
    return hipGetLastError();
}

template <int n>
static hipError_t launch_backproject_mlp_n(const LaunchArgs &a, hipStream_t st) {
    const int nb = ((a.N[0] + MBX - 1) / MBX) * ((a.N[1] + MBY - 1) / MBY) * ((a.N[2] + MBZ - 1) / MBZ);
    hipLaunchKernelGGL(backproject_mlp_kernel<n>, dim3(nb), dim3(256), 0, st, a.sino_in, a.N[0], a.N[1], a.N[2],
                       a.geom, a.vproj, a.kind, a.V, a.R, a.C, (const MlpImage *)a.mlp, a.coeffs_out);
    return hipGetLastError();
}

template <int n>
static hipError_t launch_project_pair_n(const LaunchArgs &a, hipStream_t st) {
    const int tR = (a.R + 15) / 16, tC = (a.C + 15) / 16;
    hipLaunchKernelGGL(project_pair_kernel<n>, dim3((unsigned)fwd_blocks(tR, tC, a.V)), dim3(256), 0, st, a.coeffs,
                       a.N[0], a.N[1], a.N[2], a.geom, a.kind, a.V, a.R, a.C, a.sino);
    return hipGetLastError();
}

template <int n>
static hipError_t launch_backproject_pair_n(const LaunchArgs &a, hipStream_t st) {
    const int nb = ((a.N[0] + MBX - 1) / MBX) * ((a.N[1] + MBY - 1) / MBY) * ((a.N[2] + MBZ - 1) / MBZ);
    hipLaunchKernelGGL(backproject_pair_kernel<n>, dim3(nb), dim3(256), 0, st, a.sino_in, a.N[0], a.N[1], a.N[2],
                       a.geom, a.vproj, a.kind, a.V, a.R, a.C, a.coeffs_out);
    return hipGetLastError();
}

hipError_t launch_project_pair(int degree, const LaunchArgs &a, hipStream_t st) {
    switch (degree) {
    case 0: return launch_project_pair_n<0>(a, st);
    case 1: return launch_project_pair_n<1>(a, st);
    case 2: return launch_project_pair_n<2>(a, st);
    case 3: return launch_project_pair_n<3>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_backproject_pair(int degree, const LaunchArgs &a, hipStream_t st) {
    switch (degree) {
    case 0: return launch_backproject_pair_n<0>(a, st);
    case 1: return launch_backproject_pair_n<1>(a, st);
    case 2: return launch_backproject_pair_n<2>(a, st);
    case 3: return launch_backproject_pair_n<3>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_project_mlp(int degree, const LaunchArgs &a, hipStream_t st) {
    switch (degree) {
    case 1: return launch_project_mlp_n<1>(a, st);
    case 2: return launch_project_mlp_n<2>(a, st);
    case 3: return launch_project_mlp_n<3>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_backproject_mlp(int degree, const LaunchArgs &a, hipStream_t st) {
    switch (degree) {
    case 1: return launch_backproject_mlp_n<1>(a, st);
    case 2: return launch_backproject_mlp_n<2>(a, st);
    case 3: return launch_backproject_mlp_n<3>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_footprint_mlp(int degree, const void *mlp, const float *dirs, const float *offs, int count,
                                float *out, hipStream_t st) {
    if (count == 0) return hipSuccess;
    const int nb = (count + 63) / 64;
    const MlpImage *im = (const MlpImage *)mlp;
    switch (degree) {
    case 1: hipLaunchKernelGGL(footprint_mlp_kernel<1>, dim3(nb), dim3(64), 0, st, dirs, offs, count, im, out); break;
    case 2: hipLaunchKernelGGL(footprint_mlp_kernel<2>, dim3(nb), dim3(64), 0, st, dirs, offs, count, im, out); break;
    case 3: hipLaunchKernelGGL(footprint_mlp_kernel<3>, dim3(nb), dim3(64), 0, st, dirs, offs, count, im, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ss
