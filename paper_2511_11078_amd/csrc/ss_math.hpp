// ss_math.hpp -- device arithmetic of the spline x-ray transform (gfx950).
//
// Everything here is shared by the forward and the adjoint kernels so that
// both evaluate the same footprint for the same (line, basis) pair:
//
//  * the centred B-spline beta^n, evaluated piece by piece (the piece of each
//    factor is fixed on a quadrature piece, so a node costs one Horner
//    evaluation per factor);
//  * the footprint of one basis in "slab form".  For a line whose dominant
//    axis is d (Definition 2.1: |w_d| maximal) let s = x_d - x_{q,d} be the
//    coordinate along d relative to the basis centre, and u1, u2 the
//    transverse offsets of the line from the centre where it crosses the
//    plane s = 0.  With slopes r_i = w_i / w_d (|r_i| <= 1),
//        P phi(w, x) = (1/|w_d|) * F(r1, r2, u1, u2),
//        F = int_{-h}^{h} beta(s) beta(u1 + r1 s) beta(u2 + r2 s) ds.
//    The integrand is a polynomial of degree 3n between knot crossings, so
//    m-point Gauss-Legendre with 2m - 1 >= 3n is exact on each piece.  On a
//    unit interval of s (one piece of the dominant factor) each transverse
//    factor has at most one knot, because its knots are 1/|r_i| >= 1 apart;
//    every unit interval is therefore cut into at most three pieces.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ss {

// ---------------------------------------------------------------------------
// Gauss-Legendre rules on [-1, 1] (closed forms: m = 2 nodes +-1/sqrt(3);
// m = 4 nodes +-sqrt(3/7 -+ (2/7) sqrt(6/5)); m = 5 nodes 0,
// +-(1/3) sqrt(5 -+ 2 sqrt(10/7)), with their textbook weights).
// ---------------------------------------------------------------------------
template <int M> struct GLRule;
template <> struct GLRule<1> {
    static constexpr int m = 1;
    __device__ static constexpr float x(int) { return 0.0f; }
    __device__ static constexpr float w(int) { return 2.0f; }
};
template <> struct GLRule<2> {
    static constexpr int m = 2;
    __device__ static constexpr float x(int l) { return l == 0 ? -0.57735026918962576f : 0.57735026918962576f; }
    __device__ static constexpr float w(int) { return 1.0f; }
};
template <> struct GLRule<4> {
    static constexpr int m = 4;
    __device__ static constexpr float x(int l) {
        return l == 0 ? -0.86113631159405258f : l == 1 ? -0.33998104358485626f
             : l == 2 ? 0.33998104358485626f : 0.86113631159405258f;
    }
    __device__ static constexpr float w(int l) {
        return (l == 0 || l == 3) ? 0.34785484513745386f : 0.65214515486254614f;
    }
};
template <> struct GLRule<5> {
    static constexpr int m = 5;
    __device__ static constexpr float x(int l) {
        return l == 0 ? -0.90617984593866399f : l == 1 ? -0.53846931010568309f : l == 2 ? 0.0f
             : l == 3 ? 0.53846931010568309f : 0.90617984593866399f;
    }
    __device__ static constexpr float w(int l) {
        return (l == 0 || l == 4) ? 0.23692688505618909f
             : (l == 1 || l == 3) ? 0.47862867049936647f : 0.56888888888888889f;
    }
};

// quadrature order that is exact for the degree-3n integrand
template <int n> struct Degree {
    static constexpr float h = 0.5f * (n + 1);      // support half-width
    static constexpr float kap = (n & 1) ? 0.0f : 0.5f;  // knots at kap + integer
    static constexpr int m = n == 0 ? 1 : n == 1 ? 2 : n == 2 ? 4 : 5;
};

// ---------------------------------------------------------------------------
// One polynomial piece of beta^n written in a shifted variable
// t = sg * z - k, value c0 + t (c1 + t (c2 + t c3)).  The piece is chosen
// from a point z strictly inside it (by symmetry only the pieces at z >= 0
// are tabulated; for even n the central piece is even in z).
// ---------------------------------------------------------------------------
struct Piece {
    float sg, k, c0, c1, c2, c3;
};

template <int n>
__device__ __forceinline__ Piece piece_at(float z) {
    Piece p;
    const float az = fabsf(z);
    const float sgn = z < 0.0f ? -1.0f : 1.0f;
    if constexpr (n == 3) {
        const bool inner = az < 1.0f;
        p.sg = sgn;
        p.k = inner ? 0.0f : 1.0f;
        p.c0 = inner ? (2.0f / 3.0f) : (1.0f / 6.0f);
        p.c1 = inner ? 0.0f : -0.5f;
        p.c2 = inner ? -1.0f : 0.5f;
        p.c3 = inner ? 0.5f : (-1.0f / 6.0f);
    } else if constexpr (n == 2) {
        const bool inner = az < 0.5f;
        p.sg = inner ? 1.0f : sgn;
        p.k = inner ? 0.0f : 0.5f;
        p.c0 = inner ? 0.75f : 0.5f;
        p.c1 = inner ? 0.0f : -1.0f;
        p.c2 = inner ? -1.0f : 0.5f;
        p.c3 = 0.0f;
    } else if constexpr (n == 1) {
        p.sg = sgn; p.k = 0.0f; p.c0 = 1.0f; p.c1 = -1.0f; p.c2 = 0.0f; p.c3 = 0.0f;
    } else {
        p.sg = 0.0f; p.k = -1.0f; p.c0 = 1.0f; p.c1 = 0.0f; p.c2 = 0.0f; p.c3 = 0.0f;
    }
    return p;
}

template <int n>
__device__ __forceinline__ float piece_eval(const Piece &p, float t) {
    if constexpr (n == 3) return fmaf(t, fmaf(t, fmaf(t, p.c3, p.c2), p.c1), p.c0);
    else if constexpr (n == 2) return fmaf(t, fmaf(t, p.c2, p.c1), p.c0);
    else if constexpr (n == 1) return fmaf(t, p.c1, p.c0);
    else return 1.0f;
}

// Full beta^n (used only by diagnostics and tests of the piece tables).
template <int n>
__device__ __forceinline__ float bspline(float z) {
    const float az = fabsf(z);
    if (!(az < Degree<n>::h)) return 0.0f;
    Piece p = piece_at<n>(z);
    return piece_eval<n>(p, fmaf(p.sg, z, -p.k));
}

// ---------------------------------------------------------------------------
// B-spline weights inside one knot cell.  Along an axis the knot planes sit
// at kap + m (index units); inside the cell [kap + m, kap + m + 1] exactly
// n + 1 bases are non-zero, q = m + qoff .. m + qoff + n, and with the local
// coordinate t in [0, 1) their values are the uniform B-spline blending
// polynomials below (wt[a] is the weight of basis m + qoff + a).
// ---------------------------------------------------------------------------
template <int n> struct CellBasis;
template <> struct CellBasis<0> { static constexpr int qoff = 1; };
template <> struct CellBasis<1> { static constexpr int qoff = 0; };
template <> struct CellBasis<2> { static constexpr int qoff = 0; };
template <> struct CellBasis<3> { static constexpr int qoff = -1; };

template <int n>
__device__ __forceinline__ void cell_weights(float t, float wt[n + 1]) {
    if constexpr (n == 0) {
        wt[0] = 1.0f;
    } else if constexpr (n == 1) {
        wt[0] = 1.0f - t;
        wt[1] = t;
    } else if constexpr (n == 2) {
        const float s = 1.0f - t;
        wt[0] = 0.5f * s * s;
        wt[1] = fmaf(t, s, 0.5f);            // 1/2 + t - t^2
        wt[2] = 0.5f * t * t;
    } else {
        const float s = 1.0f - t, t2 = t * t, s2 = s * s;
        const float k6 = 1.0f / 6.0f;
        wt[0] = k6 * s2 * s;                               // (1-t)^3 / 6
        wt[3] = k6 * t2 * t;                               // t^3 / 6
        wt[1] = fmaf(t2, fmaf(0.5f, t, -1.0f), 2.0f / 3.0f);  // 2/3 - t^2 + t^3/2
        wt[2] = fmaf(s2, fmaf(0.5f, s, -1.0f), 2.0f / 3.0f);  // same in 1 - t
    }
}

// The same blending polynomials in the centred coordinate u = t - 1/2
// (|u| <= 1/2 inside the cell): wt[a] = sum_p blend_u<n>(a, p) u^p.  Sums of
// products of powers of u (moments) accumulated over many lines convert to
// sums of products of weights by one linear map per axis; centring keeps
// that map well conditioned (the powers are at most 2^-p).
template <int n>
__host__ __device__ constexpr float blend_u(int a, int p) {
    if constexpr (n == 0) {
        return 1.0f;
    } else if constexpr (n == 1) {
        constexpr float B[2][2] = {{0.5f, -1.0f}, {0.5f, 1.0f}};
        return B[a][p];
    } else if constexpr (n == 2) {
        constexpr float B[3][3] = {{0.125f, -0.5f, 0.5f}, {0.75f, 0.0f, -1.0f}, {0.125f, 0.5f, 0.5f}};
        return B[a][p];
    } else {
        constexpr float B[4][4] = {{1.0f / 48.0f, -0.125f, 0.25f, -1.0f / 6.0f},
                                   {23.0f / 48.0f, -0.625f, -0.25f, 0.5f},
                                   {23.0f / 48.0f, 0.625f, -0.25f, -0.5f},
                                   {1.0f / 48.0f, 0.125f, 0.25f, 1.0f / 6.0f}};
        return B[a][p];
    }
}

// ---------------------------------------------------------------------------
// Per-line data of the slab form.  ir_i = 1 / r_i, or 0 when r_i == 0.
// ---------------------------------------------------------------------------
struct Slopes {
    float r1, r2, ir1, ir2;
};

// Restrict [lo, hi] to the s where |u + r s| < h.
template <int n>
__device__ __forceinline__ void chord_clip(float u, float r, float ir, float &lo, float &hi) {
    constexpr float h = Degree<n>::h;
    if (r == 0.0f) {
        if (!(fabsf(u) < h)) hi = lo;  // empty
    } else {
        const float ta = (-h - u) * ir, tb = (h - u) * ir;
        lo = fmaxf(lo, fminf(ta, tb));
        hi = fminf(hi, fmaxf(ta, tb));
    }
}

// The transverse knot strictly inside (A, B), as a value of s, or B.
template <int n>
__device__ __forceinline__ float knot_split(float u, float r, float ir, float A, float B) {
    constexpr float kap = Degree<n>::kap;
    const float zA = fmaf(r, A, u), zB = fmaf(r, B, u);
    const float zlo = fminf(zA, zB), zhi = fmaxf(zA, zB);
    const float kn = ceilf(zhi - kap) - 1.0f + kap;  // largest knot below zhi
    float s = (kn - u) * ir;
    s = fminf(fmaxf(s, A), B);
    return kn > zlo ? s : B;
}

// Gauss-Legendre integral of the triple product over [a, b] (a piece on
// which no factor crosses a knot).  Dominant piece chosen by its index kd.
template <int n>
__device__ __forceinline__ float gl_piece(float a, float b, const Piece &pd, float u1, float r1,
                                          float u2, float r2) {
    using R = GLRule<Degree<n>::m>;
    const float mid = 0.5f * (a + b), half = 0.5f * (b - a);
    const Piece p1 = piece_at<n>(fmaf(r1, mid, u1));
    const Piece p2 = piece_at<n>(fmaf(r2, mid, u2));
    // t_f(xi) = A_f + B_f xi for each factor, s = mid + half xi
    const float Ad = fmaf(pd.sg, mid, -pd.k), Bd = pd.sg * half;
    const float A1 = fmaf(p1.sg, fmaf(r1, mid, u1), -p1.k), B1 = p1.sg * r1 * half;
    const float A2 = fmaf(p2.sg, fmaf(r2, mid, u2), -p2.k), B2 = p2.sg * r2 * half;
    float acc = 0.0f;
#pragma unroll
    for (int l = 0; l < R::m; ++l) {
        const float xi = R::x(l);
        const float fd = piece_eval<n>(pd, fmaf(Bd, xi, Ad));
        const float f1 = piece_eval<n>(p1, fmaf(B1, xi, A1));
        const float f2 = piece_eval<n>(p2, fmaf(B2, xi, A2));
        acc = fmaf(R::w(l), fd * f1 * f2, acc);
    }
    return acc * half;
}

// Does the line (slab form) meet the open support of the basis?
template <int n>
__device__ __forceinline__ bool chord_nonempty(const Slopes &S, float u1, float u2) {
    float lo = -Degree<n>::h, hi = Degree<n>::h;
    chord_clip<n>(u1, S.r1, S.ir1, lo, hi);
    chord_clip<n>(u2, S.r2, S.ir2, lo, hi);
    return lo < hi;
}

// F(r1, r2, u1, u2) = int beta(s) beta(u1 + r1 s) beta(u2 + r2 s) ds, exact
// up to FP32 rounding.  Multiply by 1/|w_d| for the footprint.
template <int n>
__device__ __forceinline__ float footprint_slab(const Slopes &S, float u1, float u2) {
    constexpr float h = Degree<n>::h;
    float lo = -h, hi = h;
    chord_clip<n>(u1, S.r1, S.ir1, lo, hi);
    chord_clip<n>(u2, S.r2, S.ir2, lo, hi);
    if (!(lo < hi)) return 0.0f;
    if constexpr (n == 0) {
        return hi - lo;
    } else {
        float acc = 0.0f;
#pragma unroll
        for (int kd = 0; kd <= n; ++kd) {
            const float A0 = -h + (float)kd;
            const float A = fmaxf(lo, A0), B = fminf(hi, A0 + 1.0f);
            if (A < B) {
                const Piece pd = piece_at<n>(A0 + 0.5f);
                const float s1 = knot_split<n>(u1, S.r1, S.ir1, A, B);
                const float s2 = knot_split<n>(u2, S.r2, S.ir2, A, B);
                const float sa = fminf(s1, s2), sb = fmaxf(s1, s2);
                acc += gl_piece<n>(A, sa, pd, u1, S.r1, u2, S.r2);
                if (sa < B) acc += gl_piece<n>(sa, sb, pd, u1, S.r1, u2, S.r2);
                if (sb < B) acc += gl_piece<n>(sb, B, pd, u1, S.r1, u2, S.r2);
            }
        }
        return acc;
    }
}

// ---------------------------------------------------------------------------
// Lines.  A view is 12 floats: parallel (w, d0, du, dv) or cone
// (src, d0, du, dv).  Pixel (j, i) passes through
// p = d0 + (i - (C-1)/2) du + (j - (R-1)/2) dv.  The set-up runs in FP64 so
// that the FP32 quantities derived from it (slopes, offsets relative to a
// nearby point) carry only their own rounding.
// ---------------------------------------------------------------------------
struct LineD {
    double a[3];  // point of the line nearest to `centre`
    double w[3];  // unit direction
    bool ok;
};

__device__ __forceinline__ LineD make_line(const float *__restrict__ e, int kind, int R, int C, int j,
                                           int i, const double centre[3]) {
    LineD L;
    const double ci = (double)i - 0.5 * (double)(C - 1), cj = (double)j - 0.5 * (double)(R - 1);
    double p[3], d[3], a[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k] = fma(cj, (double)e[9 + k], fma(ci, (double)e[6 + k], (double)e[3 + k]));
    if (kind == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) { d[k] = (double)e[k]; a[k] = p[k]; }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) { d[k] = p[k] - (double)e[k]; a[k] = (double)e[k]; }
    }
    const double nn = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    L.ok = nn > 0.0;
    // 1/|d|: the FP32 reciprocal square root refined by one Newton step in
    // FP64 (relative error ~1e-14, a short dependency chain), exact division
    // outside the FP32 range
    double inv;
    if (nn > 1.0e-30 && nn < 1.0e30) {
        const double r0 = (double)__builtin_amdgcn_rsqf((float)nn);
        inv = r0 * fma(-0.5 * nn, r0 * r0, 1.5);
    } else {
        inv = L.ok ? 1.0 / sqrt(nn) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) L.w[k] = d[k] * inv;
    double rel[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) rel[k] = a[k] - centre[k];
    const double t = rel[0] * L.w[0] + rel[1] * L.w[1] + rel[2] * L.w[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) L.a[k] = fma(-t, L.w[k], rel[k]) + centre[k];
    return L;
}

// v[k] for a run-time k without dynamic register indexing (which would
// spill the array to scratch memory).
template <class T>
__device__ __forceinline__ T pick3(const T v[3], int k) {
    return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]);
}

// Dominant axis (Definition 2.1), lowest index among ties; i1 < i2 the others.
__device__ __forceinline__ void dominant_axis(const double w[3], int &d, int &i1, int &i2) {
    const double a0 = fabs(w[0]), a1 = fabs(w[1]), a2 = fabs(w[2]);
    if (a0 >= a1 && a0 >= a2) { d = 0; i1 = 1; i2 = 2; }
    else if (a1 >= a2) { d = 1; i1 = 0; i2 = 2; }
    else { d = 2; i1 = 0; i2 = 1; }
}

__device__ __forceinline__ Slopes make_slopes(float r1, float r2) {
    Slopes S;
    S.r1 = r1;
    S.r2 = r2;
    S.ir1 = r1 == 0.0f ? 0.0f : 1.0f / r1;
    S.ir2 = r2 == 0.0f ? 0.0f : 1.0f / r2;
    return S;
}

}  // namespace ss
