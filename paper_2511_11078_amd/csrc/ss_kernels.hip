// ss_kernels.hip -- gfx950 kernels of the spline x-ray transform.
//
//   project_kernel      forward model, one line per lane (quadrature form)
//   backproject_kernel  transpose, one coefficient per lane, atomic-free
//   footprint_kernel    P phi(w, x) for arbitrary pairs (diagnostics)
//   dot / axpy / xpay / ratio kernels for the least-squares loop
//
// The network form lives in ss_mlp.hip and reuses the traversal below.
#include "ss_kernels.hpp"

namespace ss {

// ---------------------------------------------------------------------------
// Forward: the slab walk of one line.  For every slab j of the dominant axis
// (one DDA step of the paper's projection algorithm), the candidate bases
// are those with q_d = j and |q_i - P_i(j)| < h (1 + |r_i|) in the two
// transverse axes, where P(j) is where the line crosses the plane of slab j
// (the neighbour set of the crossed cells, restricted to bases the line can
// reach; see the derivation of the window in the module header of
// ss_kernels.hpp).  Each candidate is gated by the exact chord test inside
// the footprint and visited exactly once.
// ---------------------------------------------------------------------------
template <int n, class Visit>
__device__ __forceinline__ void walk_line(const LineD &L, const int N[3], Visit &&visit) {
    constexpr double h = (double)Degree<n>::h;
    int d, i1, i2;
    dominant_axis(L.w, d, i1, i2);
    const double wd = pick3(L.w, d);
    const double r1 = pick3(L.w, i1) / wd, r2 = pick3(L.w, i2) / wd;
    const double o[3] = {-0.5 * (N[0] - 1), -0.5 * (N[1] - 1), -0.5 * (N[2] - 1)};
    // crossing point of slab j in index coordinates: P_i(j) = A_i + j r_i
    const double ad = pick3(L.a, d) - pick3(o, d);
    const double A1 = (pick3(L.a, i1) - pick3(o, i1)) - ad * r1;
    const double A2 = (pick3(L.a, i2) - pick3(o, i2)) - ad * r2;
    const double H1 = h * (1.0 + fabs(r1)), H2 = h * (1.0 + fabs(r2));
    const int Nd = pick3(N, d), N1 = pick3(N, i1), N2 = pick3(N, i2);
    // slabs where both windows can be non-empty: -H < P_i(j) < N_i - 1 + H
    double jlo = 0.0, jhi = (double)(Nd - 1);
    {
        const double rr[2] = {r1, r2}, AA[2] = {A1, A2}, HH[2] = {H1, H2};
        const int NN[2] = {N1, N2};
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
    }
    const Slopes S = make_slopes((float)r1, (float)r2);
    // clamp in FP64 before converting: every index below stays in [0, N - 1]
    const int j0 = (int)fmin(fmax(jlo, 0.0), (double)Nd);
    const int j1 = (int)fmax(fmin(jhi, (double)(Nd - 1)), -1.0);
    for (int j = j0; j <= j1; ++j) {
        const double P1 = fma((double)j, r1, A1), P2 = fma((double)j, r2, A2);
        const int lo1 = (int)fmin(fmax(floor(P1 - H1) + 1.0, 0.0), (double)N1);
        const int hi1 = (int)fmax(fmin(ceil(P1 + H1) - 1.0, (double)(N1 - 1)), -1.0);
        const int lo2 = (int)fmin(fmax(floor(P2 - H2) + 1.0, 0.0), (double)N2);
        const int hi2 = (int)fmax(fmin(ceil(P2 + H2) - 1.0, (double)(N2 - 1)), -1.0);
        for (int q2 = lo2; q2 <= hi2; ++q2) {
            const float u2 = (float)(P2 - (double)q2);
            for (int q1 = lo1; q1 <= hi1; ++q1) {
                const float u1 = (float)(P1 - (double)q1);
                visit(S, u1, u2, d, j, i1, q1, i2, q2);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Forward, quadrature form: cell walk.  The footprint of a basis is the sum,
// over the knot cells its support spans, of the Gauss-Legendre integral of
// its (polynomial) restriction to the line inside the cell.  Walking the
// line cell by cell through the knot lattice (Amanatides-Woo stepping over
// the support-padded box) and adding, for every cell, c_q times that
// per-cell integral for each of the (n+1)^3 bases whose support covers the
// cell visits every (line, basis) pair of eq. (4) exactly once, through the
// same Gauss-Legendre terms as the slab-by-slab per-basis sum, evaluated
// with the node positions and per-axis weights shared by the (n+1)^3 bases.
// ---------------------------------------------------------------------------
template <int n>
__global__ void __launch_bounds__(256) project_kernel(const float *__restrict__ c, int N0, int N1, int N2,
                                                      const float *__restrict__ geom, int kind, int V, int R,
                                                      int C, float *__restrict__ y) {
    using Rule = GLRule<Degree<n>::m>;
    constexpr int NB = n + 1;
    constexpr double h = (double)Degree<n>::h;
    constexpr double kap = (double)Degree<n>::kap;
    constexpr int qoff = CellBasis<n>::qoff;
    const int tR = (R + 15) / 16, tC = (C + 15) / 16;
    const int nblocks = V * tR * tC;
    const int b = xcd_remap(blockIdx.x, nblocks);
    const int v = b / (tR * tC), rem = b % (tR * tC);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = (rem / tC) * 16 + (wave >> 1) * 8 + (lane >> 3);
    const int i = (rem % tC) * 16 + (wave & 1) * 8 + (lane & 7);
    if (v >= V || j >= R || i >= C) return;
    const int N[3] = {N0, N1, N2};
    const double centre[3] = {0.0, 0.0, 0.0};
    const LineD L = make_line(geom + 12 * v, kind, R, C, j, i, centre);
    float acc = 0.0f;
    if (L.ok) {
        // index coordinates z = x - o, o = -(N - 1)/2
        double z0[3], t0 = -1e300, t1 = 1e300;
        bool hit = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            z0[k] = L.a[k] + 0.5 * (double)(N[k] - 1);
            const double lo = -h, hi = (double)(N[k] - 1) + h;
            if (L.w[k] == 0.0) {
                if (!(z0[k] > lo && z0[k] < hi)) hit = false;
                // degree 0: the support of beta^0 is open, so a line lying in
                // a face plane between two voxels meets neither
                if (n == 0 && z0[k] - kap == floor(z0[k] - kap)) hit = false;
            } else {
                const double ta = (lo - z0[k]) / L.w[k], tb = (hi - z0[k]) / L.w[k];
                t0 = fmax(t0, fmin(ta, tb));
                t1 = fmin(t1, fmax(ta, tb));
            }
        }
        if (hit && t0 < t1) {
            // DDA state per axis
            int m[3], stp[3];
            double tmax[3], tdel[3];
            // a point just past the entry (the entry lies on a knot plane)
            const double tm0 = t0 + fmin(1e-6, 0.5 * (t1 - t0));
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double zs = fma(tm0, L.w[k], z0[k]) - kap;
                m[k] = (int)floor(fmin(fmax(zs, -8.0), (double)N[k] + 8.0));
                if (L.w[k] > 0.0) {
                    stp[k] = 1;
                    tdel[k] = 1.0 / L.w[k];
                    tmax[k] = ((double)(m[k] + 1) + kap - z0[k]) / L.w[k];
                } else if (L.w[k] < 0.0) {
                    stp[k] = -1;
                    tdel[k] = -1.0 / L.w[k];
                    tmax[k] = ((double)m[k] + kap - z0[k]) / L.w[k];
                } else {
                    stp[k] = 0;
                    tdel[k] = 0.0;
                    tmax[k] = 1e300;
                }
            }
            const int64_t s1 = N0, s2 = (int64_t)N0 * N1;
            double tc = t0;
            // every step moves one axis to its next knot plane: the walk ends
            // after at most sum_k (N_k + 2h + 2) steps
            while (tc < t1) {
                int ax = 0;
                double tn = tmax[0];
                if (tmax[1] < tn) { tn = tmax[1]; ax = 1; }
                if (tmax[2] < tn) { tn = tmax[2]; ax = 2; }
                tn = fmin(tn, t1);
                if (tn > tc) {
                    const double mid = 0.5 * (tc + tn), half = 0.5 * (tn - tc);
                    float lc[3], dl[3];
                    int q0[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        lc[k] = (float)(fma(mid, L.w[k], z0[k]) - ((double)m[k] + kap));
                        dl[k] = (float)(half * L.w[k]);
                        q0[k] = m[k] + qoff;
                    }
                    // coefficient block (zero outside the volume)
                    float cb[NB][NB][NB];
                    const bool inner = q0[0] >= 0 && q0[0] + n < N0 && q0[1] >= 0 && q0[1] + n < N1 &&
                                       q0[2] >= 0 && q0[2] + n < N2;
                    if (inner) {
                        const float *base = c + (int64_t)q0[2] * s2 + (int64_t)q0[1] * s1 + q0[0];
#pragma unroll
                        for (int a3 = 0; a3 < NB; ++a3)
#pragma unroll
                            for (int a2 = 0; a2 < NB; ++a2)
#pragma unroll
                                for (int a1 = 0; a1 < NB; ++a1) cb[a3][a2][a1] = base[a3 * s2 + a2 * s1 + a1];
                    } else {
#pragma unroll
                        for (int a3 = 0; a3 < NB; ++a3)
#pragma unroll
                            for (int a2 = 0; a2 < NB; ++a2)
#pragma unroll
                                for (int a1 = 0; a1 < NB; ++a1) {
                                    const int k1 = q0[0] + a1, k2 = q0[1] + a2, k3 = q0[2] + a3;
                                    const bool ok = k1 >= 0 && k1 < N0 && k2 >= 0 && k2 < N1 && k3 >= 0 && k3 < N2;
                                    cb[a3][a2][a1] = ok ? c[(int64_t)k3 * s2 + (int64_t)k2 * s1 + k1] : 0.0f;
                                }
                    }
                    float seg = 0.0f;
#pragma unroll
                    for (int l = 0; l < Rule::m; ++l) {
                        const float xi = Rule::x(l);
                        float w1[NB], w2[NB], w3[NB];
                        cell_weights<n>(fmaf(dl[0], xi, lc[0]), w1);
                        cell_weights<n>(fmaf(dl[1], xi, lc[1]), w2);
                        cell_weights<n>(fmaf(dl[2], xi, lc[2]), w3);
                        float f = 0.0f;
#pragma unroll
                        for (int a3 = 0; a3 < NB; ++a3) {
                            float g = 0.0f;
#pragma unroll
                            for (int a2 = 0; a2 < NB; ++a2) {
                                float r = 0.0f;
#pragma unroll
                                for (int a1 = 0; a1 < NB; ++a1) r = fmaf(w1[a1], cb[a3][a2][a1], r);
                                g = fmaf(w2[a2], r, g);
                            }
                            f = fmaf(w3[a3], g, f);
                        }
                        seg = fmaf(Rule::w(l), f, seg);
                    }
                    acc = fmaf((float)half, seg, acc);
                }
                tc = fmax(tc, tn);
                // advance the axis whose plane was reached
                if (ax == 0) { m[0] += stp[0]; tmax[0] += tdel[0]; }
                else if (ax == 1) { m[1] += stp[1]; tmax[1] += tdel[1]; }
                else { m[2] += stp[2]; tmax[2] += tdel[2]; }
            }
        }
    }
    y[((int64_t)v * R + j) * C + i] = acc;
}

// ---------------------------------------------------------------------------
// Adjoint: brick gather.  A block owns a BX x BY x BZ brick of coefficients,
// one per thread, and loops over the views.  Per view it maps the brick's
// support box to a pixel rectangle, sets those lines up once (FP64, anchor
// re-based near the brick centre) into an LDS table, then every thread sums
// y_m * footprint over the pixels of its own support's rectangle.  Each
// coefficient is written once, by its owner: no atomics, deterministic.
// ---------------------------------------------------------------------------
constexpr int BX = 8, BY = 8, BZ = 4;
constexpr int RAY_CAP = 1024;  // lines per LDS chunk

struct RayRec {      // 48 bytes
    float a[3];      // point of the line nearest the brick centre, relative to it
    float r1, r2, ir1, ir2;
    float len;       // 1 / |w_d|
    float y;
    int d;
    int pad0, pad1;
};

template <int n>
__device__ __forceinline__ void fill_ray(RayRec &rec, const float *__restrict__ e, int kind, int R, int C, int j,
                                         int i, const double centre[3], float yval) {
    const LineD L = make_line(e, kind, R, C, j, i, centre);
    int d, i1, i2;
    dominant_axis(L.w, d, i1, i2);
    const double wd = pick3(L.w, d);
    const double r1 = pick3(L.w, i1) / wd, r2 = pick3(L.w, i2) / wd;
    const Slopes S = make_slopes((float)r1, (float)r2);
    // re-based anchor (nearest point to the brick centre), relative to it
    rec.a[0] = (float)(L.a[0] - centre[0]);
    rec.a[1] = (float)(L.a[1] - centre[1]);
    rec.a[2] = (float)(L.a[2] - centre[2]);
    rec.r1 = S.r1; rec.r2 = S.r2; rec.ir1 = S.ir1; rec.ir2 = S.ir2;
    rec.len = (float)(1.0 / fabs(wd));
    rec.y = L.ok ? yval : 0.0f;
    rec.d = d;
}

template <int n>
__global__ void __launch_bounds__(256) backproject_kernel(const float *__restrict__ y, int N0, int N1, int N2,
                                                          const float *__restrict__ geom, int kind, int V, int R,
                                                          int C, float *__restrict__ c) {
    __shared__ RayRec rays[RAY_CAP];
    __shared__ ViewProj vp;
    __shared__ int sbox[4];
    const int nbx = (N0 + BX - 1) / BX, nby = (N1 + BY - 1) / BY, nbz = (N2 + BZ - 1) / BZ;
    const int b = xcd_remap(blockIdx.x, nbx * nby * nbz);
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int tid = threadIdx.x;
    const int k0 = bx * BX + (tid % BX), k1 = by * BY + ((tid / BX) % BY), k2 = bz * BZ + tid / (BX * BY);
    const bool mine = k0 < N0 && k1 < N1 && k2 < N2;
    constexpr double h = (double)Degree<n>::h;
    const double o[3] = {-0.5 * (N0 - 1), -0.5 * (N1 - 1), -0.5 * (N2 - 1)};
    // brick centre (world) and this coefficient's position relative to it
    const double centre[3] = {o[0] + bx * BX + 0.5 * (BX - 1), o[1] + by * BY + 0.5 * (BY - 1),
                              o[2] + bz * BZ + 0.5 * (BZ - 1)};
    const float xq[3] = {(float)(o[0] + k0 - centre[0]), (float)(o[1] + k1 - centre[1]),
                         (float)(o[2] + k2 - centre[2])};
    // FP32 sums within a view, accumulated across views in FP64
    double acc = 0.0;
    for (int v = 0; v < V; ++v) {
        const float *e = geom + 12 * v;
        float part = 0.0f;
        if (tid == 0) {
            make_viewproj(e, kind, vp);
            double lo[3], hi[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int nb = k == 0 ? BX : k == 1 ? BY : BZ;
                lo[k] = centre[k] - 0.5 * (nb - 1) - h;
                hi[k] = centre[k] + 0.5 * (nb - 1) + h;
            }
            box_to_pixels(vp, lo, hi, R, C, sbox[0], sbox[1], sbox[2], sbox[3]);
        }
        __syncthreads();
        const int bi0 = sbox[0], bi1 = sbox[1], bj0 = sbox[2], bj1 = sbox[3];
        // this coefficient's own rectangle
        int mi0 = 0, mi1 = -1, mj0 = 0, mj1 = -1;
        if (mine) {
            double lo[3], hi[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                lo[k] = centre[k] + (double)xq[k] - h;
                hi[k] = centre[k] + (double)xq[k] + h;
            }
            box_to_pixels(vp, lo, hi, R, C, mi0, mi1, mj0, mj1);
        }
        const int W = bi1 - bi0 + 1;
        const int rows_per_chunk = W > 0 ? max(1, RAY_CAP / W) : 1;
        for (int cj0 = bj0; cj0 <= bj1; cj0 += rows_per_chunk) {
            const int cj1 = min(bj1, cj0 + rows_per_chunk - 1);
            const int cnt = (cj1 - cj0 + 1) * W;
            // W can exceed RAY_CAP only for absurd geometries; then split columns
            const int cols = min(W, RAY_CAP);
            for (int ci0 = bi0; ci0 <= bi1; ci0 += cols) {
                const int ci1 = min(bi1, ci0 + cols - 1);
                const int cw = ci1 - ci0 + 1;
                const int cn = min(cnt, (cj1 - cj0 + 1) * cw);
                __syncthreads();
                for (int t = tid; t < cn; t += blockDim.x) {
                    const int jj = cj0 + t / cw, ii = ci0 + t % cw;
                    fill_ray<n>(rays[t], e, kind, R, C, jj, ii, centre, y[((int64_t)v * R + jj) * C + ii]);
                }
                __syncthreads();
                if (mine) {
                    const int j0 = max(mj0, cj0), j1 = min(mj1, cj1);
                    const int i0 = max(mi0, ci0), i1 = min(mi1, ci1);
                    for (int jj = j0; jj <= j1; ++jj) {
                        for (int ii = i0; ii <= i1; ++ii) {
                            const RayRec &rr = rays[(jj - cj0) * cw + (ii - ci0)];
                            const int d = rr.d;
                            const int i1x = d == 0 ? 1 : 0, i2x = d == 2 ? 1 : 2;
                            const float ad = d == 0 ? rr.a[0] : d == 1 ? rr.a[1] : rr.a[2];
                            const float xd = d == 0 ? xq[0] : d == 1 ? xq[1] : xq[2];
                            const float a1 = i1x == 0 ? rr.a[0] : rr.a[1];
                            const float x1 = i1x == 0 ? xq[0] : xq[1];
                            const float a2 = i2x == 1 ? rr.a[1] : rr.a[2];
                            const float x2 = i2x == 1 ? xq[1] : xq[2];
                            const float t = xd - ad;
                            const float u1 = fmaf(t, rr.r1, a1) - x1;
                            const float u2 = fmaf(t, rr.r2, a2) - x2;
                            Slopes S;
                            S.r1 = rr.r1; S.r2 = rr.r2; S.ir1 = rr.ir1; S.ir2 = rr.ir2;
                            const float f = footprint_slab<n>(S, u1, u2);
                            if (f != 0.0f) part = fmaf(rr.y * rr.len, f, part);
                        }
                    }
                }
            }
        }
        __syncthreads();
        acc += (double)part;
    }
    if (mine) c[((int64_t)k2 * N1 + k1) * N0 + k0] = (float)acc;
}

// ---------------------------------------------------------------------------
// Footprint of arbitrary pairs (diagnostics): w unit, x any point of the
// line relative to the basis centre.
// ---------------------------------------------------------------------------
template <int n>
__global__ void footprint_kernel(const float *__restrict__ dirs, const float *__restrict__ offs, int count,
                                 float *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    double w[3], x[3];
    for (int a = 0; a < 3; ++a) { w[a] = dirs[3 * k + a]; x[a] = offs[3 * k + a]; }
    int d, i1, i2;
    dominant_axis(w, d, i1, i2);
    const double wd = pick3(w, d);
    if (wd == 0.0) { out[k] = 0.0f; return; }
    const double r1 = pick3(w, i1) / wd, r2 = pick3(w, i2) / wd;
    const Slopes S = make_slopes((float)r1, (float)r2);
    const double xd = pick3(x, d);
    const float u1 = (float)(pick3(x, i1) - xd * r1), u2 = (float)(pick3(x, i2) - xd * r2);
    const double nrm = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    out[k] = footprint_slab<n>(S, u1, u2) * (float)(nrm / fabs(wd));
}

// ---------------------------------------------------------------------------
// FP64-accumulated inner product (two passes, fixed grid: deterministic),
// FP64 ratio, FP32 vector updates with a device scalar.
// ---------------------------------------------------------------------------
constexpr int DOT_BLOCKS = 1024, DOT_THREADS = 256;

__global__ void __launch_bounds__(DOT_THREADS) dot_partial_kernel(const float *__restrict__ a,
                                                                  const float *__restrict__ b, int64_t n,
                                                                  double *__restrict__ part) {
    __shared__ double red[DOT_THREADS];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        s = fma((double)a[i], (double)b[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = DOT_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(DOT_THREADS) dot_final_kernel(const double *__restrict__ part, int np,
                                                                double *__restrict__ out) {
    __shared__ double red[DOT_THREADS];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += DOT_THREADS) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = DOT_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void ratio_kernel(const double *__restrict__ num, const double *__restrict__ den,
                             double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double dd = *den;
        *out = dd != 0.0 ? *num / dd : 0.0;
    }
}

__global__ void axpy_kernel(const double *__restrict__ alpha, float sign, const float *__restrict__ x,
                            float *__restrict__ yv, int64_t n) {
    const float a = sign * (float)(*alpha);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        yv[i] = fmaf(a, x[i], yv[i]);
}

__global__ void xpay_kernel(const double *__restrict__ beta, const float *__restrict__ x, float *__restrict__ yv,
                            int64_t n) {
    const float bt = (float)(*beta);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        yv[i] = fmaf(bt, yv[i], x[i]);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <int n>
static hipError_t launch_project_n(const LaunchArgs &a, hipStream_t st) {
    const int tR = (a.R + 15) / 16, tC = (a.C + 15) / 16;
    const int nb = a.V * tR * tC;
    hipLaunchKernelGGL(project_kernel<n>, dim3(nb), dim3(256), 0, st, a.coeffs, a.N[0], a.N[1], a.N[2], a.geom,
                       a.kind, a.V, a.R, a.C, a.sino);
    return hipGetLastError();
}

template <int n>
static hipError_t launch_backproject_n(const LaunchArgs &a, hipStream_t st) {
    const int nb = ((a.N[0] + BX - 1) / BX) * ((a.N[1] + BY - 1) / BY) * ((a.N[2] + BZ - 1) / BZ);
    hipLaunchKernelGGL(backproject_kernel<n>, dim3(nb), dim3(256), 0, st, a.sino_in, a.N[0], a.N[1], a.N[2],
                       a.geom, a.kind, a.V, a.R, a.C, a.coeffs_out);
    return hipGetLastError();
}

hipError_t launch_project_quad(int degree, const LaunchArgs &a, hipStream_t st) {
    switch (degree) {
    case 0: return launch_project_n<0>(a, st);
    case 1: return launch_project_n<1>(a, st);
    case 2: return launch_project_n<2>(a, st);
    case 3: return launch_project_n<3>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_backproject_quad(int degree, const LaunchArgs &a, hipStream_t st) {
    switch (degree) {
    case 0: return launch_backproject_n<0>(a, st);
    case 1: return launch_backproject_n<1>(a, st);
    case 2: return launch_backproject_n<2>(a, st);
    case 3: return launch_backproject_n<3>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_footprint_quad(int degree, const float *dirs, const float *offs, int count, float *out,
                                 hipStream_t st) {
    const int nb = (count + 255) / 256;
    if (count == 0) return hipSuccess;
    switch (degree) {
    case 0: hipLaunchKernelGGL(footprint_kernel<0>, dim3(nb), dim3(256), 0, st, dirs, offs, count, out); break;
    case 1: hipLaunchKernelGGL(footprint_kernel<1>, dim3(nb), dim3(256), 0, st, dirs, offs, count, out); break;
    case 2: hipLaunchKernelGGL(footprint_kernel<2>, dim3(nb), dim3(256), 0, st, dirs, offs, count, out); break;
    case 3: hipLaunchKernelGGL(footprint_kernel<3>, dim3(nb), dim3(256), 0, st, dirs, offs, count, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dot(const float *a, const float *b, int64_t n, double *partials, double *out, hipStream_t st) {
    hipLaunchKernelGGL(dot_partial_kernel, dim3(DOT_BLOCKS), dim3(DOT_THREADS), 0, st, a, b, n, partials);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(DOT_THREADS), 0, st, partials, DOT_BLOCKS, out);
    return hipGetLastError();
}

int dot_partials_needed() { return DOT_BLOCKS; }

hipError_t launch_ratio(const double *num, const double *den, double *out, hipStream_t st) {
    hipLaunchKernelGGL(ratio_kernel, dim3(1), dim3(64), 0, st, num, den, out);
    return hipGetLastError();
}

static int vec_blocks(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

hipError_t launch_axpy(const double *alpha, float sign, const float *x, float *yv, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(axpy_kernel, dim3(vec_blocks(n)), dim3(256), 0, st, alpha, sign, x, yv, n);
    return hipGetLastError();
}

hipError_t launch_xpay(const double *beta, const float *x, float *yv, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(xpay_kernel, dim3(vec_blocks(n)), dim3(256), 0, st, beta, x, yv, n);
    return hipGetLastError();
}

}  // namespace ss
