// ss_traverse.hpp -- launch-order and detector-mapping helpers shared by the
// quadrature and network kernels.
#pragma once

#include "ss_math.hpp"

namespace ss {

// ---------------------------------------------------------------------------
// XCD-aware block order: consecutive hardware block ids go round-robin over
// the 8 XCDs, each with its own L2.  Give every XCD a contiguous run of
// logical tiles so neighbouring tiles (which read overlapping coefficient
// regions) share an L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    constexpr int NX = 8;
    const int per = (nblocks + NX - 1) / NX;
    const int xcd = b % NX, local = b / NX;
    const int full = nblocks % NX == 0 ? NX : nblocks % NX;  // XCDs that get `per` blocks
    int t;
    if (xcd < full) t = xcd * per + local;
    else t = full * per + (xcd - full) * (per - 1) + local;
    return t;
}

// Forward launches: one 256-thread block per 16x16-pixel tile and view.
// Tiles form FT_GH x FT_GW groups; the groups go round-robin to the 8 XCDs
// (hardware block h runs on XCD h % 8), and within a group the views are
// innermost.  An XCD thus takes groups x, x + 8, x + 16, ... spread over the
// detector (the XCDs get equal work), and the blocks it runs at one time walk
// neighbouring lines of consecutive views, which share coefficient lines in
// its L2.
constexpr int FT_GH = 2, FT_GW = 2;
__host__ __device__ inline int fwd_groups(int tR, int tC) {
    return ((tR + FT_GH - 1) / FT_GH) * ((tC + FT_GW - 1) / FT_GW);
}
__host__ __device__ inline int64_t fwd_blocks(int tR, int tC, int V) {
    return (int64_t)((fwd_groups(tR, tC) + 7) / 8 * 8) * FT_GH * FT_GW * V;
}
// View and tile of this block; false for a padding slot (a whole block).
__device__ __forceinline__ bool fwd_block_tile(int V, int tR, int tC, int &v, int &tr, int &tc) {
    const int per = FT_GH * FT_GW * V;
    const int x = blockIdx.x % 8, l = blockIdx.x / 8;
    const int G = (l / per) * 8 + x, inner = l % per;
    v = inner % V;
    const int q = inner / V;
    if (G >= fwd_groups(tR, tC)) return false;
    const int gC = (tC + FT_GW - 1) / FT_GW;
    tr = (G / gC) * FT_GH + q / FT_GW;
    tc = (G % gC) * FT_GW + q % FT_GW;
    return tr < tR && tc < tC;
}

struct ViewProj {    // detector coordinates of a world point (FP64 set-up)
    double d0[3], s[3], du_s[3], dv_s[3], nrm[3];
    double plane;    // (d0 - s) . nrm  (cone)
    // for make_localproj: o . du_s, o . dv_s, o . nrm with o = s (cone) or d0
    // (parallel), and the FP32 values that do not depend on the centre
    double odu, odv, onm;
    float du_f[3], dv_f[3], nm_f[3];
    float ac_f, ar_f, plane_f;  // (s - d0) . du_s, (s - d0) . dv_s, plane
    int kind;
};

// Continuous pixel coordinates (column, row) of world point X.
// parallel: X = d0 + alpha du + beta dv + t w ;  cone: the detector point
// of the line through the source and X.  Returns false when undefined.
__device__ __forceinline__ bool to_detector(const ViewProj &P, const double X[3], double &col, double &row) {
    double q[3];
    if (P.kind == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] = X[k] - P.d0[k];
    } else {
        double dx[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) dx[k] = X[k] - P.s[k];
        const double den = dx[0] * P.nrm[0] + dx[1] * P.nrm[1] + dx[2] * P.nrm[2];
        if (!(den * P.plane > 0.0)) return false;  // X on or behind the source plane
        const double lam = P.plane / den;
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] = P.s[k] + lam * dx[k] - P.d0[k];
    }
    col = q[0] * P.du_s[0] + q[1] * P.du_s[1] + q[2] * P.du_s[2];
    row = q[0] * P.dv_s[0] + q[1] * P.dv_s[1] + q[2] * P.dv_s[2];
    return true;
}

// Dual basis: du_s . du = 1, du_s . dv = 0, du_s . m = 0 (m = w or the
// detector normal), likewise dv_s.
__host__ __device__ inline void make_viewproj(const float *__restrict__ e, int kind, ViewProj &P) {
    double du[3], dv[3], m[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        P.s[k] = e[k];
        P.d0[k] = e[3 + k];
        du[k] = e[6 + k];
        dv[k] = e[9 + k];
    }
    P.kind = kind;
    P.nrm[0] = du[1] * dv[2] - du[2] * dv[1];
    P.nrm[1] = du[2] * dv[0] - du[0] * dv[2];
    P.nrm[2] = du[0] * dv[1] - du[1] * dv[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) m[k] = kind == 0 ? P.s[k] : P.nrm[k];
    P.plane = (P.d0[0] - P.s[0]) * P.nrm[0] + (P.d0[1] - P.s[1]) * P.nrm[1] + (P.d0[2] - P.s[2]) * P.nrm[2];
    // rows of inverse([du dv m]) via cross products
    double c0[3] = {dv[1] * m[2] - dv[2] * m[1], dv[2] * m[0] - dv[0] * m[2], dv[0] * m[1] - dv[1] * m[0]};
    double c1[3] = {m[1] * du[2] - m[2] * du[1], m[2] * du[0] - m[0] * du[2], m[0] * du[1] - m[1] * du[0]};
    const double det = du[0] * c0[0] + du[1] * c0[1] + du[2] * c0[2];
    const double id = det != 0.0 ? 1.0 / det : 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        P.du_s[k] = c0[k] * id;
        P.dv_s[k] = c1[k] * id;
    }
    double o[3], sd[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        o[k] = kind == 0 ? P.d0[k] : P.s[k];
        sd[k] = P.s[k] - P.d0[k];
        P.du_f[k] = (float)P.du_s[k];
        P.dv_f[k] = (float)P.dv_s[k];
        P.nm_f[k] = (float)P.nrm[k];
    }
    P.odu = o[0] * P.du_s[0] + o[1] * P.du_s[1] + o[2] * P.du_s[2];
    P.odv = o[0] * P.dv_s[0] + o[1] * P.dv_s[1] + o[2] * P.dv_s[2];
    P.onm = o[0] * P.nrm[0] + o[1] * P.nrm[1] + o[2] * P.nrm[2];
    P.ac_f = (float)(sd[0] * P.du_s[0] + sd[1] * P.du_s[1] + sd[2] * P.du_s[2]);
    P.ar_f = (float)(sd[0] * P.dv_s[0] + sd[1] * P.dv_s[1] + sd[2] * P.dv_s[2]);
    P.plane_f = (float)P.plane;
}

// Detector coordinates of points X = c + delta near a centre c, evaluated in
// FP32 for small delta; every term that involves c or the source is formed
// in FP64 once.  With D = c - s (cone) or c - d0 (parallel):
//   parallel: col = D . du_s + delta . du_s
//   cone:     col = (s - d0) . du_s + plane (D . du_s + delta . du_s) / (D . nrm + delta . nrm)
// and likewise for rows with dv_s.
struct LocalProj {
    float du[3], dv[3], nm[3];
    float nc, nr, dn;   // D . du_s, D . dv_s, D . nrm
    float ac, ar;       // (s - d0) . du_s, (s - d0) . dv_s  (cone)
    float plane;
    int kind;
};

// D . du_s = c . du_s - o . du_s in FP64 (three FMA and a difference per
// term); everything else comes from the view's set-up.
__device__ __forceinline__ void make_localproj(const ViewProj &P, const double c[3], LocalProj &L) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        L.du[k] = P.du_f[k];
        L.dv[k] = P.dv_f[k];
        L.nm[k] = P.nm_f[k];
    }
    L.nc = (float)(fma(c[2], P.du_s[2], fma(c[1], P.du_s[1], c[0] * P.du_s[0])) - P.odu);
    L.nr = (float)(fma(c[2], P.dv_s[2], fma(c[1], P.dv_s[1], c[0] * P.dv_s[0])) - P.odv);
    L.dn = (float)(fma(c[2], P.nrm[2], fma(c[1], P.nrm[1], c[0] * P.nrm[0])) - P.onm);
    L.ac = P.ac_f;
    L.ar = P.ar_f;
    L.plane = P.plane_f;
    L.kind = P.kind;
}

// false when X is on or behind the source plane (cone)
__device__ __forceinline__ bool local_to_detector(const LocalProj &L, const float d[3], float &col, float &row) {
    const float nu = fmaf(d[2], L.du[2], fmaf(d[1], L.du[1], fmaf(d[0], L.du[0], L.nc)));
    const float nv = fmaf(d[2], L.dv[2], fmaf(d[1], L.dv[1], fmaf(d[0], L.dv[0], L.nr)));
    if (L.kind == 0) {
        col = nu;
        row = nv;
        return true;
    }
    const float den = fmaf(d[2], L.nm[2], fmaf(d[1], L.nm[1], fmaf(d[0], L.nm[0], L.dn)));
    if (!(den * L.plane > 0.0f)) return false;
    const float lam = L.plane * __builtin_amdgcn_rcpf(den);
    col = fmaf(lam, nu, L.ac);
    row = fmaf(lam, nv, L.ar);
    return true;
}

// Pixel rectangle [i0, i1] x [j0, j1] covering every line that meets the
// box [lo, hi] (whole detector if the projection is undefined).
__device__ __forceinline__ void box_to_pixels(const ViewProj &P, const double lo[3], const double hi[3], int R,
                                              int C, int &i0, int &i1, int &j0, int &j1) {
    double cmin = 1e300, cmax = -1e300, rmin = 1e300, rmax = -1e300;
    bool ok = true;
#pragma unroll
    for (int corner = 0; corner < 8; ++corner) {
        double X[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) X[k] = ((corner >> k) & 1) ? hi[k] : lo[k];
        double cc, rr;
        if (!to_detector(P, X, cc, rr)) ok = false;
        cmin = fmin(cmin, cc); cmax = fmax(cmax, cc);
        rmin = fmin(rmin, rr); rmax = fmax(rmax, rr);
    }
    if (!ok) { i0 = 0; i1 = C - 1; j0 = 0; j1 = R - 1; return; }
    const double oc = 0.5 * (C - 1), orow = 0.5 * (R - 1);
    const double fi0 = floor(cmin + oc) - 1.0, fi1 = ceil(cmax + oc) + 1.0;
    const double fj0 = floor(rmin + orow) - 1.0, fj1 = ceil(rmax + orow) + 1.0;
    if (!(fi1 >= 0.0 && fj1 >= 0.0 && fi0 <= (double)(C - 1) && fj0 <= (double)(R - 1))) {
        i0 = 0; i1 = -1; j0 = 0; j1 = -1;  // empty (also catches NaN)
        return;
    }
    // clamped in FP64 before converting
    i0 = (int)fmax(fi0, 0.0); i1 = (int)fmin(fi1, (double)(C - 1));
    j0 = (int)fmax(fj0, 0.0); j1 = (int)fmin(fj1, (double)(R - 1));
}

}  // namespace ss
