// ss_kernels.hip -- gfx950 kernels of the spline x-ray transform.
//
//   pad_volume_kernel + project_kernel
//                       forward model, one line per lane (quadrature form)
//   backproject_cells_kernel + cells_to_coeffs_kernel
//                       transpose: knot-cell gather, then coefficient gather (atomic-free)
//   footprint_kernel    P phi(w, x) for arbitrary pairs (diagnostics)
//   dot / axpy / xpay / ratio kernels for the least-squares loop
//
// The network form lives in ss_mlp.hip and shares the line set-up, block
// order and detector mapping of ss_math.hpp and ss_traverse.hpp.
#include "ss_kernels.hpp"

#include <algorithm>
#include <mutex>

namespace ss {

// Zero-padded copy of the coefficients for the forward walk: FWD_PAD(n)
// zero layers on every side, so that the (n+1)^3 block of every knot cell of
// the support-padded box (and of one cell beyond) is inside the copy.
__global__ void __launch_bounds__(256) pad_volume_kernel(const float *__restrict__ c, int N0, int N1, int N2, int P,
                                                         float *__restrict__ out) {
    const int S0 = N0 + 2 * P, S1 = N1 + 2 * P, S2 = N2 + 2 * P;
    const int64_t total = (int64_t)S0 * S1 * S2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int x = (int)(i % S0) - P;
        const int64_t r = i / S0;
        const int yy = (int)(r % S1) - P, z = (int)(r / S1) - P;
        const bool in = x >= 0 && x < N0 && yy >= 0 && yy < N1 && z >= 0 && z < N2;
        out[i] = in ? c[((int64_t)z * N1 + yy) * N0 + x] : 0.0f;
    }
}

// The same copy with x and y exchanged (y fastest: element (x, y, z) at
// ((z + P) (N0 + 2P) + x + P) (N1 + 2P) + y + P), for the views the forward
// walks in that order; each block transposes a 32 x 32 (x, y) tile of one
// z layer through LDS.
constexpr int PAD_T = 32;
__global__ void __launch_bounds__(256) pad_volume_yfast_kernel(const float *__restrict__ c, int N0, int N1, int N2,
                                                               int P, float *__restrict__ out) {
    __shared__ float tile[PAD_T][PAD_T + 1];  // [y][x] of the tile
    const int Sx = N0 + 2 * P, Sy = N1 + 2 * P;
    const int tiles_x = (Sx + PAD_T - 1) / PAD_T, tiles_y = (Sy + PAD_T - 1) / PAD_T;
    const int bx = blockIdx.x % tiles_x, by = (blockIdx.x / tiles_x) % tiles_y;
    const int zp = blockIdx.x / (tiles_x * tiles_y);  // padded z layer
    const int z = zp - P;
    const int tx = threadIdx.x % PAD_T, ty = threadIdx.x / PAD_T;  // 32 x 8
#pragma unroll
    for (int k = 0; k < PAD_T; k += 8) {
        const int x = bx * PAD_T + tx - P, yy = by * PAD_T + ty + k - P;
        const bool in = x >= 0 && x < N0 && yy >= 0 && yy < N1 && z >= 0 && z < N2;
        tile[ty + k][tx] = in ? c[((int64_t)z * N1 + yy) * N0 + x] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PAD_T; k += 8) {
        const int xp = bx * PAD_T + ty + k, yp = by * PAD_T + tx;
        if (xp < Sx && yp < Sy) out[((int64_t)zp * Sx + xp) * Sy + yp] = tile[tx][ty + k];
    }
}

// Whether the forward (degrees 1 to 3) walks view e in the y-fastest copy.
// Measured per 5-degree range of circular cone trajectories (256^3 and
// 512^3, degree 3; degrees 2 and 1 gain as much from it): with
// phi the angle between the view's central ray and its dominant horizontal
// axis, rows along the minor horizontal axis are faster for phi < 15
// degrees and rows along the dominant axis for 15 <= phi < 35; beyond, and
// for views whose central ray is mostly along z, the x-fastest copy.  Both
// copies hold the same values, so the choice changes only the FP32
// rounding order of the contraction, not what is computed.
__device__ __forceinline__ bool view_walks_yfast(const float *__restrict__ e, int kind) {
    float d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = kind != 0 ? e[3 + k] - e[k] : e[k];  // cone: source -> detector centre
    const float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
    const float hi = fmaxf(ax, ay), lo = fminf(ax, ay);
    if (!(az < hi)) return false;
    const float s = lo / hi;                        // tan(phi)
    constexpr float T15 = 0.26794919f, T35 = 0.70020754f;
    return ax >= ay ? s < T15 : (s >= T15 && s < T35);
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
// Launched once per copy: with yfast = 0 on the x-fastest copy for the views
// that walk it, with yfast = 1 on the y-fastest copy for the others (blocks
// of the other views return at once); the walk then runs with x and y
// exchanged.
template <int n>
__global__ void __launch_bounds__(256, 4) project_kernel(const float *__restrict__ cp, int N0, int N1, int N2,
                                                      const float *__restrict__ geom, int kind, int V, int R,
                                                      int C, float *__restrict__ y, int yfast) {
    using Rule = GLRule<Degree<n>::m>;
    constexpr int NB = n + 1;
    constexpr double h = (double)Degree<n>::h;
    constexpr double kap = (double)Degree<n>::kap;
    constexpr int qoff = CellBasis<n>::qoff;
    const int tR = (R + 15) / 16, tC = (C + 15) / 16;
    int v, tr, tc;
    if (!fwd_block_tile(V, tR, tC, v, tr, tc)) return;  // padding slot
    if (v < V && (n >= 1 && view_walks_yfast(geom + 12 * v, kind)) != (yfast != 0)) return;  // the other copy's view
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = tr * 16 + (wave >> 1) * 8 + (lane >> 3);
    const int i = tc * 16 + (wave & 1) * 8 + (lane & 7);
    if (v >= V || j >= R || i >= C) return;
    // the walk runs in the copy's axis order: (x, y, z), or (y, x, z)
    const int N[3] = {yfast ? N1 : N0, yfast ? N0 : N1, N2};
    const double centre[3] = {0.0, 0.0, 0.0};
    LineD L = make_line(geom + 12 * v, kind, R, C, j, i, centre);
    if (yfast) {
        const double a0 = L.a[0], w0 = L.w[0];
        L.a[0] = L.a[1]; L.a[1] = a0;
        L.w[0] = L.w[1]; L.w[1] = w0;
    }
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
            // zero-padded copy of the coefficients (FWD_PAD(n) layers per side)
            constexpr int P = FWD_PAD(n);
            const int64_t s1 = N[0] + 2 * P, s2 = (int64_t)(N[0] + 2 * P) * (N[1] + 2 * P);
            const int hi0 = N[0] - 1 + P - n, hi1 = N[1] - 1 + P - n, hi2 = N[2] - 1 + P - n;
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
                    // coefficient block from the padded copy: every cell of the
                    // walk lies in the support-padded box, so its block is inside
                    // the copy (the clamp only guards a cell index rounded past
                    // the box edge, whose segment has no length)
                    float cb[NB][NB][NB];
                    {
                        const int x0 = min(max(q0[0], -P), hi0) + P, x1 = min(max(q0[1], -P), hi1) + P,
                                  x2 = min(max(q0[2], -P), hi2) + P;
                        const float *base = cp + (int64_t)x2 * s2 + (int64_t)x1 * s1 + x0;
#pragma unroll
                        for (int a3 = 0; a3 < NB; ++a3)
#pragma unroll
                            for (int a2 = 0; a2 < NB; ++a2)
#pragma unroll
                                for (int a1 = 0; a1 < NB; ++a1) cb[a3][a2][a1] = base[a3 * s2 + a2 * s1 + a1];
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
// Adjoint, quadrature form: cell gather, two passes, no atomics.
//
// The transpose of the forward cell walk: line m adds y_m times the
// Gauss-Legendre integral, over its chord through knot cell K, of the
// restriction of basis q to the line, for each of the (n+1)^3 bases q whose
// support covers K.  Pass 1 gives every knot cell to one thread, which
// gathers, over all views, the lines of the pixels whose centres fall in the
// detector shadow of its cell, accumulates the centred moments of their
// chords (integrate_hit) and at the end maps them to the (n+1)^3 per-basis
// integrals (T[K][a] below, a = q - K - qoff per axis).  Pass 2 gives every
// coefficient to one thread, which adds its (n+1)^3 entries T[q - qoff - a][a]
// of the cells its support covers.  Every (line, basis) pair of eq. (4)
// is evaluated through the same per-cell Gauss-Legendre terms as the
// forward, each output has a single writer, and the summation order is
// fixed.
//
// Pass 1 blocks own GX x GY x GZ bricks of cells.  Per view a block projects
// the brick's lattice corners once into LDS (FP32 offsets from the brick
// centre, every term involving the centre or the source formed in FP64),
// appends the lines of the brick's pixel rectangle to an LDS table (FP64
// set-up, anchor re-based at the brick centre), and every thread takes the
// bounding rectangle of its own cell's eight projected corners as its
// candidate pixels (about 95 % of them hit the cell).  A thread queues its
// candidates without reading their lines in a ring, oldest first, and the
// integration drops the few whose chord through the cell is empty.  The
// table has two halves filled in turn (up to a few views each):
// before a half is refilled, each wave runs as many integration rounds as
// its lane with the most entries in that half needs, and lanes with fewer
// take entries of the other half in the same rounds, so that the lanes of a
// wave, whose candidate counts differ view by view, stay busy.
//
// The cell table T holds (n+1)^3 FP32 entries per cell, entry-major
// (T[a * cells + K], K x-fastest over the cells of a z-chunk), so that both
// passes access it coalesced.  Volumes whose table would exceed the
// context's scratch are processed in overlapping z-chunks of cell layers:
// a chunk of L layers finalises L - n coefficient layers.
// ---------------------------------------------------------------------------
constexpr int GX = 8, GY = 8, GZ = 4;
constexpr int NCORNER = (GX + 1) * (GY + 1) * (GZ + 1);
constexpr int HITQ_CAP = 32;                    // queued candidates per thread (a ring)
// Line table (two halves) and occupancy per degree: the cubic kernel's
// registers allow three waves per SIMD, so its table takes what LDS leaves
// for three blocks per CU beside the candidate queues and two corner tables,
// counting 160 KiB in 2 KiB units (three blocks of 54,232 bytes did not fit
// on a CU); lower degrees fit four waves and a smaller table.
template <int n> struct CellGather {
    static constexpr int waves = n == 3 ? 3 : 4;          // waves per SIMD: blocks per CU
    static constexpr int lds = (160 * 1024 / waves) / 2048 * 2048;
    static constexpr int fixed = HITQ_CAP * 256 * 2 + 2 * NCORNER * 8 + 16;
    static constexpr int cap = (lds - fixed) / 40 / 16 * 16;  // lines in the LDS table (40 bytes each)
    static constexpr int half = cap / 2;
    static constexpr int views_per_half = n == 3 ? 5 : 3;
    // wave priority while a block sets up a view (0: the default throughout)
    static constexpr int setup_prio = n == 0 ? 0 : 2;
};
constexpr float PIX_MARGIN = 1.0e-3f;           // pixels; covers FP32 rounding of the corner table

struct __attribute__((aligned(8))) CellRay {  // 40 bytes
    float a[3];      // point of the line nearest the brick centre, relative to it
    float iw[3];     // 1 / w_k; 0 marks an axis the line is parallel to
    float w[3];      // unit direction
    float y;         // sinogram value
};

__device__ __forceinline__ void fill_cellray(CellRay &rec, const float *__restrict__ e, int kind, int R, int C, int j,
                                             int i, const double centre[3], float yval) {
    const LineD L = make_line(e, kind, R, C, j, i, centre);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // a degenerate line is put far outside every cell, parallel to all axes
        const float wk = L.ok ? (float)L.w[k] : 0.0f;
        rec.a[k] = L.ok ? (float)(L.a[k] - centre[k]) : 1.0e30f;
        rec.w[k] = wk;
        rec.iw[k] = wk != 0.0f ? __builtin_amdgcn_rcpf(wk) : 0.0f;
    }
    rec.y = L.ok ? yval : 0.0f;
}

// Chord [t0, t1] of a line through the cell [lo, lo + 1]^3 (coordinates
// relative to the brick centre).  A line parallel to a knot plane belongs to
// the cell above it when it lies in the plane (the forward walk's choice);
// for degree 0 the support is open and such a line meets neither cell.
// Written without branches (selects only), so that the record is read in
// one go and the lanes of a wave never split on the rare parallel axis.
template <int n>
__device__ __forceinline__ bool cell_chord(const CellRay &r, const float lo[3], float &t0, float &t1) {
    bool in = true;
    t0 = -3.0e38f;
    t1 = 3.0e38f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const bool par = r.iw[k] == 0.0f;
        const bool inside = (n == 0 ? lo[k] < r.a[k] : lo[k] <= r.a[k]) & (r.a[k] < lo[k] + 1.0f);
        const float ta = (lo[k] - r.a[k]) * r.iw[k], tb = (lo[k] + 1.0f - r.a[k]) * r.iw[k];
        in = in & (inside | !par);
        t0 = par ? t0 : fmaxf(t0, fminf(ta, tb));
        t1 = par ? t1 : fminf(t1, fmaxf(ta, tb));
    }
    return in & (t0 < t1);
}

// Add one line's chord through the cell to the cell's moments: at the m
// Gauss-Legendre nodes of the chord, y * weight * u1^p1 u2^p2 u3^p3 for the
// centred cell coordinates u = t - 1/2.
template <int n>
__device__ __forceinline__ void integrate_hit(const CellRay &r, const float lo[3], float acc[]) {
    using Rule = GLRule<Degree<n>::m>;
    constexpr int NB = n + 1;
    float t0, t1;
    if (!cell_chord<n>(r, lo, t0, t1)) return;  // a candidate whose line misses the cell
    const float mid = 0.5f * (t0 + t1), half = 0.5f * (t1 - t0);
    float uc[3], du[3];  // centred cell coordinate at mid, and its step
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        uc[q] = fmaf(mid, r.w[q], r.a[q]) - (lo[q] + 0.5f);
        du[q] = half * r.w[q];
    }
    const float sc = half * r.y;
#pragma unroll
    for (int l = 0; l < Rule::m; ++l) {
        const float xi = Rule::x(l);
        // powers u^p of the three centred coordinates (p >= 1)
        float P1[NB], P2[NB], P3[NB];
        P1[0] = Rule::w(l) * sc;  // axis 1 carries the quadrature weight
        P2[0] = 1.0f;
        P3[0] = 1.0f;
        const float u1 = fmaf(du[0], xi, uc[0]), u2 = fmaf(du[1], xi, uc[1]), u3 = fmaf(du[2], xi, uc[2]);
#pragma unroll
        for (int p = 1; p <= n; ++p) {
            P1[p] = P1[p - 1] * u1;
            P2[p] = p == 1 ? u2 : P2[p - 1] * u2;
            P3[p] = p == 1 ? u3 : P3[p - 1] * u3;
        }
#pragma unroll
        for (int p3 = 0; p3 < NB; ++p3)
#pragma unroll
            for (int p2 = 0; p2 < NB; ++p2) {
                // z = u2^p2 u3^p3 (no product where either power is zero)
                const float z = p3 == 0 ? P2[p2] : (p2 == 0 ? P3[p3] : P3[p3] * P2[p2]);
#pragma unroll
                for (int p1 = 0; p1 < NB; ++p1) {
                    float &a = acc[(p3 * NB + p2) * NB + p1];
                    a = (p2 == 0 && p3 == 0) ? a + P1[p1] : fmaf(z, P1[p1], a);
                }
            }
    }
}

// Pixels whose centre lies in the continuous detector rectangle
// [cmin, cmax] x [rmin, rmax] (pixel units), clamped to the detector;
// PIX_MARGIN absorbs the FP32 rounding of the corner table.
__device__ __forceinline__ void pixel_rect(float cmin, float cmax, float rmin, float rmax, int R, int C, int &i0,
                                           int &i1, int &j0, int &j1) {
    // clamped in FP32 before converting
    const float fi0 = fmaxf(ceilf(cmin - PIX_MARGIN), 0.0f), fi1 = fminf(floorf(cmax + PIX_MARGIN), (float)(C - 1));
    const float fj0 = fmaxf(ceilf(rmin - PIX_MARGIN), 0.0f), fj1 = fminf(floorf(rmax + PIX_MARGIN), (float)(R - 1));
    if (fi0 <= fi1 && fj0 <= fj1) {
        i0 = (int)fi0; i1 = (int)fi1; j0 = (int)fj0; j1 = (int)fj1;
    } else {
        i0 = 0; i1 = -1; j0 = 0; j1 = -1;
    }
}

// Bounding rectangle of the projected corners of the lattice box
// [x0, x0 + sx] x [y0, y0 + sy] x [z0, z0 + sz] (corner table of the brick).
// The projection of the box is the convex hull of its corners' projections,
// so every pixel whose line meets the box is in the rectangle.
__device__ __forceinline__ void corner_bounds(const float2 *corner, int sx, int sy, int sz, int x0, int y0, int z0,
                                              float &cmin, float &cmax, float &rmin, float &rmax) {
    cmin = 3.0e38f; cmax = -3.0e38f; rmin = 3.0e38f; rmax = -3.0e38f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int cx = x0 + ((k & 1) ? sx : 0), cy = y0 + ((k & 2) ? sy : 0), cz = z0 + ((k & 4) ? sz : 0);
        const float2 p = corner[(cz * (GY + 1) + cy) * (GX + 1) + cx];
        cmin = fminf(cmin, p.x); cmax = fmaxf(cmax, p.x);
        rmin = fminf(rmin, p.y); rmax = fmaxf(rmax, p.y);
    }
}

// Three (degree 3, at most 168 VGPRs) or four (lower degrees, 128) waves per
// SIMD keep as many blocks on a CU, to hide the per-view set-up between
// barriers behind other blocks' integration.
template <int n>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CellGather<n>::waves)))
backproject_cells_kernel(const float *__restrict__ y, int N0, int N1, int N2, const float *__restrict__ geom,
                         const ViewProj *__restrict__ vps, int kind, int V, int R, int C, int mz0, int L,
                         float *__restrict__ T) {
    constexpr int NB = n + 1;
    constexpr int qoff = CellBasis<n>::qoff;
    constexpr double kap = (double)Degree<n>::kap;
    constexpr int CRAY_HALF = CellGather<n>::half, VIEWS_PER_HALF = CellGather<n>::views_per_half;
    // A view's set-up (corner table, rectangles, line table, queueing) is
    // short dependent chains ending in a barrier; the integration is long
    // runs of independent FMAs.  Raising a wave's priority for the set-up
    // lets each block reach its barrier sooner while the other blocks on the
    // CU keep the FMA pipes busy (degrees 1-3; the degree-0 kernel, whose
    // integration is short, runs faster without).
    constexpr int PRIO = CellGather<n>::setup_prio;
    const auto prio_setup = [] {
        if constexpr (PRIO > 0) __builtin_amdgcn_s_setprio(PRIO);
    };
    const auto prio_integrate = [] {
        if constexpr (PRIO > 0) __builtin_amdgcn_s_setprio(0);
    };
    static_assert(sizeof(CellRay) == 40, "line record size assumed by the LDS budget");
    __shared__ CellRay rays[CellGather<n>::cap];
    __shared__ unsigned short hitq[HITQ_CAP * 256];  // per-thread queue of candidate table indices
    __shared__ float2 corner[2][NCORNER];            // view v's corner table in [v & 1]
    __shared__ int badview[2];  // v + 1 in [v & 1] when a corner of view v is on or behind the source plane
    const int M0 = N0 + n, M1 = N1 + n;  // cells per row / column
    const int nbx = (M0 + GX - 1) / GX, nby = (M1 + GY - 1) / GY, nbz = (L + GZ - 1) / GZ;
    const int b = xcd_remap(blockIdx.x, nbx * nby * nbz);
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int tid = threadIdx.x;
    const int tx = tid % GX, ty = (tid / GX) % GY, tz = tid / (GX * GY);
    const int c0 = bx * GX + tx, c1 = by * GY + ty, c2 = bz * GZ + tz;  // cell, chunk-relative
    const bool mine = c0 < M0 && c1 < M1 && c2 < L;
    // first cell of the brick in index units (cell K spans [K + kap, K + kap + 1]
    // in coordinates x + (N - 1)/2), and the brick centre in world coordinates
    const int mlo = -qoff - n;
    const double centre[3] = {(double)(mlo + bx * GX) + kap - 0.5 * (N0 - 1) + 0.5 * GX,
                              (double)(mlo + by * GY) + kap - 0.5 * (N1 - 1) + 0.5 * GY,
                              (double)(mz0 + bz * GZ) + kap - 0.5 * (N2 - 1) + 0.5 * GZ};
    // this cell's low corner relative to the brick centre (exact)
    const float lo[3] = {(float)tx - 0.5f * GX, (float)ty - 0.5f * GY, (float)tz - 0.5f * GZ};
    const float oc = 0.5f * (float)(C - 1), orow = 0.5f * (float)(R - 1);
    float acc[NB * NB * NB];
#pragma unroll
    for (int e = 0; e < NB * NB * NB; ++e) acc[e] = 0.0f;
    // block-uniform: the half being filled, its entries and views, and
    // whether the other half has been filled before
    int half = 0, used = 0, nviews = 0;
    bool other_filled = false;
    // this thread's queue: a ring of table indices, oldest first, in slots
    // qhead + 256 k (mod the ring); the first `nolder` entries belong to the
    // other half
    constexpr int QMASK = HITQ_CAP * 256 - 1;
    int qhead = tid, count = 0, nolder = 0;

    // Detector position (pixel units) of every lattice corner of the brick
    // for view v, into corner[v & 1]; a corner on or behind the source plane
    // (no bounded shadow) stores v + 1 into badview[v & 1] (every writer the
    // same value, so no reset is needed).  View v + 1's table is written
    // while view v's lines are set up, so that one barrier per view orders
    // both: each view's phase ends with at least one barrier, table [v & 1]
    // and flag [v & 1] are read in phase v and rewritten in phase v + 1.
    auto project_corners = [&](int v) {
        LocalProj lp;  // the same in every thread
        make_localproj(vps[v], centre, lp);
        bool bad = false;
#pragma unroll
        for (int it = 0; it < (NCORNER + 255) / 256; ++it) {  // independent iterations
            const int t = tid + 256 * it;
            if (t < NCORNER) {
                const int cx = t % (GX + 1), cy = (t / (GX + 1)) % (GY + 1), cz = t / ((GX + 1) * (GY + 1));
                const float d[3] = {(float)cx - 0.5f * GX, (float)cy - 0.5f * GY, (float)cz - 0.5f * GZ};
                float cc = 0.0f, rr = 0.0f;
                const bool ok = local_to_detector(lp, d, cc, rr);
                bad = bad || !ok;
                corner[v & 1][t] = make_float2(cc + oc, rr + orow);
            }
        }
        if (bad) badview[v & 1] = v + 1;
    };
    if (tid < 2) badview[tid] = -1;
    __syncthreads();
    if (V > 0) project_corners(0);
    __syncthreads();

    for (int v = 0; v < V; ++v) {
        prio_setup();
        const float *e = geom + 12 * v;
        const float2 *cornerv = corner[v & 1];
        const bool anybad = badview[v & 1] == v + 1;
        // the brick's pixel rectangle (from its eight corners, the same for
        // every thread) and this cell's candidate pixels (from its own)
        int bi0, bi1, bj0, bj1;
        int mi0 = 0, mi1 = -1, mj0 = 0, mj1 = -1;
        if (anybad) {
            bi0 = 0; bi1 = C - 1; bj0 = 0; bj1 = R - 1;
            if (mine) { mi0 = 0; mi1 = C - 1; mj0 = 0; mj1 = R - 1; }
        } else {
            float bc0, bc1, br0, br1;
            corner_bounds(cornerv, GX, GY, GZ, 0, 0, 0, bc0, bc1, br0, br1);
            pixel_rect(bc0, bc1, br0, br1, R, C, bi0, bi1, bj0, bj1);
            if (mine) {
                float c0, c1, r0, r1;
                corner_bounds(cornerv, 1, 1, 1, tx, ty, tz, c0, c1, r0, r1);
                pixel_rect(c0, c1, r0, r1, R, C, mi0, mi1, mj0, mj1);
            }
        }
        if (v + 1 < V) project_corners(v + 1);
        bool barrier = false;  // block-uniform: a barrier has passed in this view's phase
        // the view's lines go into the current half of the table in segments
        // of whole rows (of columns, for a row wider than a half); this cell's
        // candidates are queued, and integrated before their half is refilled
        const int W = bi1 - bi0 + 1;
        if (W > 0 && bj1 >= bj0) {
            // integer quotients by a float reciprocal: (a + 1/2) / b is at
            // least 1/(2b) away from an integer, far more than its rounding
            const int rows_per_seg = max(1, (int)(((float)CRAY_HALF + 0.5f) * __builtin_amdgcn_rcpf((float)W)));
            const int cols = min(W, CRAY_HALF);
            for (int cj0 = bj0; cj0 <= bj1; cj0 += rows_per_seg) {
                const int cj1 = min(bj1, cj0 + rows_per_seg - 1);
                for (int ci0 = bi0; ci0 <= bi1; ci0 += cols) {
                    const int ci1 = min(bi1, ci0 + cols - 1);
                    const int cw = ci1 - ci0 + 1;
                    const int cn = (cj1 - cj0 + 1) * cw;
                    if (used + cn > CRAY_HALF || nviews == VIEWS_PER_HALF) {
                        // switch halves.  Before the other half is refilled,
                        // every lane retires its entries there; lanes with
                        // fewer of them integrate entries of this half in the
                        // same rounds (the wave runs as many rounds as its
                        // lane with the most entries in the other half)
                        if (other_filled) {
                            prio_integrate();
                            int K = nolder;
#pragma unroll
                            for (int m = 32; m >= 1; m >>= 1) K = max(K, __shfl_xor(K, m));
                            const int npop = min(K, count);
                            int idx = hitq[qhead];  // the next entry's index is read a round ahead
                            for (int k = 0; k < npop; ++k) {
                                qhead = (qhead + 256) & QMASK;
                                const int cur = idx;
                                idx = hitq[qhead];
                                integrate_hit<n>(rays[cur], lo, acc);
                            }
                            count -= npop;
                            __syncthreads();  // no wave reads the other half any more
                            prio_setup();
                        }
                        nolder = count;  // every queued entry is now in the older half
                        half ^= 1;
                        used = 0;
                        nviews = 0;
                        other_filled = true;
                    }
                    // new entries go past every queued one: no barrier needed
                    const int tb = half * CRAY_HALF + used;  // first table entry of the segment
                    const float rcw = __builtin_amdgcn_rcpf((float)cw);
                    for (int t = tid; t < cn; t += blockDim.x) {
                        const int q = (int)(((float)t + 0.5f) * rcw);
                        const int jj = cj0 + q, ii = ci0 + (t - q * cw);
                        fill_cellray(rays[tb + t], e, kind, R, C, jj, ii, centre,
                                     y[((int64_t)v * R + jj) * C + ii]);
                    }
                    __syncthreads();
                    barrier = true;
                    const int j0 = max(mj0, cj0), j1 = min(mj1, cj1);
                    const int i0 = max(mi0, ci0), i1 = min(mi1, ci1);
                    const int ni = i1 - i0 + 1, nc = (j1 >= j0 && ni > 0) ? (j1 - j0 + 1) * ni : 0;
                    if (count + nc <= HITQ_CAP) {
                        // room for every candidate: one flat loop in the same
                        // (row, column) order, no overflow test per entry
                        int e = tb + (j0 - cj0) * cw + (i0 - ci0);  // table entry of the first candidate
                        int slot = qhead + 256 * count;
                        for (int k = 0, ii = 0; k < nc; ++k) {
                            hitq[slot & QMASK] = (unsigned short)e;
                            slot += 256;
                            ++ii;
                            const bool wrap = ii == ni;
                            e += wrap ? cw - ni + 1 : 1;
                            ii = wrap ? 0 : ii;
                        }
                        count += nc;
                    } else {
                        for (int jj = j0; jj <= j1; ++jj)
                            for (int ii = i0; ii <= i1; ++ii) {
                                if (count == HITQ_CAP) {  // queue full: integrate its oldest entry now
                                    integrate_hit<n>(rays[hitq[qhead]], lo, acc);
                                    qhead = (qhead + 256) & QMASK;
                                    --count;
                                    nolder = max(nolder - 1, 0);
                                }
                                hitq[(qhead + 256 * count) & QMASK] =
                                    (unsigned short)(tb + (jj - cj0) * cw + (ii - ci0));
                                ++count;
                            }
                    }
                    used += cn;
                }
            }
            ++nviews;
        }
        if (!barrier) __syncthreads();
    }
    prio_integrate();
    int idx = hitq[qhead];
    for (int k = 0; k < count; ++k) {
        qhead = (qhead + 256) & QMASK;
        const int cur = idx;
        idx = hitq[qhead];
        integrate_hit<n>(rays[cur], lo, acc);
    }
    // moments -> per-basis integrals: apply the blending map along each axis
    if constexpr (n > 0) {
#pragma unroll
        for (int i = 0; i < NB * NB; ++i) {  // axis 1: index (i, p1)
            float t[NB];
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                t[a] = 0.0f;
#pragma unroll
                for (int p = 0; p < NB; ++p) t[a] = fmaf(blend_u<n>(a, p), acc[i * NB + p], t[a]);
            }
#pragma unroll
            for (int a = 0; a < NB; ++a) acc[i * NB + a] = t[a];
        }
#pragma unroll
        for (int i3 = 0; i3 < NB; ++i3)  // axis 2: index (i3, p2, a1)
#pragma unroll
            for (int i1 = 0; i1 < NB; ++i1) {
                float t[NB];
#pragma unroll
                for (int a = 0; a < NB; ++a) {
                    t[a] = 0.0f;
#pragma unroll
                    for (int p = 0; p < NB; ++p) t[a] = fmaf(blend_u<n>(a, p), acc[(i3 * NB + p) * NB + i1], t[a]);
                }
#pragma unroll
                for (int a = 0; a < NB; ++a) acc[(i3 * NB + a) * NB + i1] = t[a];
            }
#pragma unroll
        for (int i = 0; i < NB * NB; ++i) {  // axis 3: index (p3, i)
            float t[NB];
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                t[a] = 0.0f;
#pragma unroll
                for (int p = 0; p < NB; ++p) t[a] = fmaf(blend_u<n>(a, p), acc[p * NB * NB + i], t[a]);
            }
#pragma unroll
            for (int a = 0; a < NB; ++a) acc[a * NB * NB + i] = t[a];
        }
    }
    if (mine) {
        const int64_t cells = (int64_t)M0 * M1 * L;
        const int64_t K = ((int64_t)c2 * M1 + c1) * M0 + c0;
#pragma unroll
        for (int a = 0; a < NB * NB * NB; ++a) T[a * cells + K] = acc[a];
    }
}

// Pass 2: coefficient q (layer q2 in [qz0, qz1]) adds T[K][a] over the cells
// K = q - qoff - a of its support (FP64 sum of the (n+1)^3 FP32 entries).
template <int n>
__global__ void __launch_bounds__(256) cells_to_coeffs_kernel(const float *__restrict__ T, int N0, int N1,
                                                              int mz0, int L, int qz0, int qz1,
                                                              float *__restrict__ c) {
    constexpr int NB = n + 1;
    constexpr int qoff = CellBasis<n>::qoff;
    const int64_t per = (int64_t)N0 * N1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per * (qz1 - qz0 + 1)) return;
    const int k2 = qz0 + (int)(idx / per);
    const int rem = (int)(idx % per);
    const int k1 = rem / N0, k0 = rem % N0;
    const int M0 = N0 + n, M1 = N1 + n;
    const int mlo = -qoff - n;
    const int64_t cells = (int64_t)M0 * M1 * L;
    double s = 0.0;
#pragma unroll
    for (int a3 = 0; a3 < NB; ++a3) {
        const int z = k2 - qoff - a3 - mz0;  // in [0, L) for qz0 <= k2 <= qz1
#pragma unroll
        for (int a2 = 0; a2 < NB; ++a2) {
            const int yy = k1 - qoff - a2 - mlo;
#pragma unroll
            for (int a1 = 0; a1 < NB; ++a1) {
                const int xx = k0 - qoff - a1 - mlo;
                const int64_t K = ((int64_t)z * M1 + yy) * M0 + xx;
                s += (double)T[((a3 * NB + a2) * NB + a1) * cells + K];
            }
        }
    }
    c[(int64_t)k2 * per + rem] = (float)s;
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
    const int nb = (int)fwd_blocks(tR, tC, a.V);
    constexpr int P = FWD_PAD(n);
    const int64_t padded = (int64_t)(a.N[0] + 2 * P) * (a.N[1] + 2 * P) * (a.N[2] + 2 * P);
    if (!a.scratch || a.scratch_floats < padded) return hipErrorInvalidValue;
    const int pb = (int)std::min<int64_t>((padded + 255) / 256, 65536);
    hipLaunchKernelGGL(pad_volume_kernel, dim3(pb), dim3(256), 0, st, a.coeffs, a.N[0], a.N[1], a.N[2], P,
                       a.scratch);
    // Occupancy of the walk: for degrees 1..3 a block reserves LDS it does
    // not use (FWD_IDLE_LDS), so that at most three blocks, three waves per
    // SIMD, share a CU.  Fewer concurrent walks then share the CU's L1
    // cache, which keeps more of each wave's coefficient rows; the degree-0
    // walk (one coefficient per cell) runs best at full occupancy.
    constexpr int FWD_IDLE_LDS = n == 0 ? 0 : 50 * 1024;  // 3 x 50 KiB of the CU's 160 KiB
    hipLaunchKernelGGL(project_kernel<n>, dim3(nb), dim3(256), FWD_IDLE_LDS, st, a.scratch, a.N[0], a.N[1],
                       a.N[2], a.geom, a.kind, a.V, a.R, a.C, a.sino, 0);
    if constexpr (n >= 1) {
        // the views that walk the y-fastest copy: the same scratch, rewritten
        // after the first launch (stream order); the degree-0 walk, bound by
        // L2 refills rather than by its arithmetic, keeps one copy
        const int64_t yb = (int64_t)((a.N[0] + 2 * P + PAD_T - 1) / PAD_T) * ((a.N[1] + 2 * P + PAD_T - 1) / PAD_T) *
                           (a.N[2] + 2 * P);
        if (yb > INT32_MAX) return hipErrorInvalidValue;
        hipLaunchKernelGGL(pad_volume_yfast_kernel, dim3((unsigned)yb), dim3(256), 0, st, a.coeffs, a.N[0], a.N[1],
                           a.N[2], P, a.scratch);
        hipLaunchKernelGGL(project_kernel<n>, dim3(nb), dim3(256), FWD_IDLE_LDS, st, a.scratch, a.N[0], a.N[1],
                           a.N[2], a.geom, a.kind, a.V, a.R, a.C, a.sino, 1);
    }
    return hipGetLastError();
}

int64_t project_quad_scratch_floats(int degree, const int N[3]) {
    const int64_t P = degree + 1;
    return (N[0] + 2 * P) * (N[1] + 2 * P) * (N[2] + 2 * P);
}

int64_t backproject_quad_scratch_floats(int degree, const int N[3], int64_t limit) {
    const int64_t nb = degree + 1;
    const int64_t layer = nb * nb * nb * (int64_t)(N[0] + degree) * (N[1] + degree);
    const int64_t full = layer * (N[2] + degree);
    // at least 4 (n + 1) layers per chunk, so that chunking re-does at most
    // a quarter of the cell layers
    const int64_t floor_layers = std::min<int64_t>(N[2] + degree, 4 * nb);
    return std::min(full, std::max(limit, layer * floor_layers));
}

template <int n>
static hipError_t launch_backproject_n(const LaunchArgs &a, hipStream_t st) {
    constexpr int qoff = CellBasis<n>::qoff;
    constexpr int64_t NB3 = (int64_t)(n + 1) * (n + 1) * (n + 1);
    const int M0 = a.N[0] + n, M1 = a.N[1] + n, M2 = a.N[2] + n;
    const int64_t layer = NB3 * M0 * M1;
    const int Lmax = (int)std::min<int64_t>(M2, a.scratch_floats / layer);
    if (!a.scratch || Lmax <= n) return hipErrorInvalidValue;
    const int mlo = -qoff - n;
    const int64_t plane = (int64_t)a.N[0] * a.N[1];
    for (int s = mlo;;) {
        const int L = std::min(Lmax, mlo + M2 - s);
        const int nb = ((M0 + GX - 1) / GX) * ((M1 + GY - 1) / GY) * ((L + GZ - 1) / GZ);
        hipLaunchKernelGGL(backproject_cells_kernel<n>, dim3(nb), dim3(256), 0, st, a.sino_in, a.N[0], a.N[1],
                           a.N[2], a.geom, a.vproj, a.kind, a.V, a.R, a.C, s, L, a.scratch);
        const int qz0 = s + qoff + n, qz1 = std::min(s + L - 1 + qoff, a.N[2] - 1);
        if (qz1 >= qz0) {
            const int64_t cnt = plane * (qz1 - qz0 + 1);
            hipLaunchKernelGGL(cells_to_coeffs_kernel<n>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
                               a.scratch, a.N[0], a.N[1], s, L, qz0, qz1, a.coeffs_out);
        }
        if (s + L >= mlo + M2) break;
        s += L - n;
    }
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

// ---------------------------------------------------------------------------
// Allocation-free forward: a file-scope device array holds the view vectors
// and the zero-padded coefficients.  Host code never passes `scratch` itself
// to a kernel (in host code the name is a host-side stand-in); it asks the
// runtime, once per device with that device current, for the array's device
// address and passes that.
// ---------------------------------------------------------------------------
static __device__ __align__(256) float scratch[STATIC_SCRATCH_FLOATS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t static_scratch_address(int device, float **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<float *>(p);
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
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
