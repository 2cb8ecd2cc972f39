/*
 * oracle.c -- plain FP64 reference for the spline x-ray transform.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product:
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header, table or constant generator
 * with the HIP path.  It favours obviously-correct over fast: plain loops,
 * double precision, compensated sums, OpenMP over rays.
 *
 * What it computes (paper: "SplineSplat: 3D Ray Tracing for Higher-Quality
 * Tomography", arXiv 2511.11078):
 *   - lines {a + t w} (Sec. 1.2, eq. (1)); the x-ray transform integrates a
 *     function over the whole line (eq. (2));
 *   - the volume f(x) = sum_k c_k phi(x - x_k) (eq. (3)) with phi the
 *     tensor-product centred B-spline of degree n (Sec. 2.2 uses n = 2; the
 *     benchmark workloads use n = 3; n = 0 is the voxel baseline of Sec. 3),
 *     coefficient k sitting at x_k = k - (N - 1)/2 per axis (lattice of unit
 *     step, Sec. 2.1), zero outside the index box;
 *   - the single-basis footprint P phi(w, x) = int phi(x + t w) dt (the
 *     "contribution" of eq. (4));
 *   - the forward model [P]_{m,l} = P phi(w_m, s_m - Proj k_l) (eq. (7)) and
 *     its transpose.
 *
 * Exactness: on a line, phi(x(t) - x_k) is a polynomial of degree <= 3n
 * between two consecutive crossings of knot planes, so m-point
 * Gauss-Legendre with 2m - 1 >= 3n is exact on every such segment.
 *
 * Parts:  O1 or_bspline / or_bspline_tp    centred B-spline, two formulas
 *         O2 or_gauss_legendre             GL rule by Newton on P_m
 *         O3 or_project                    direct integral of f along rays
 *         O4 or_footprint                  single-basis footprint
 *         O5 or_project_basis_sum          sum_k c_k * O4 (eq. (4))
 *         O6 or_backproject_subset         voxel-driven transpose of eq. (7)
 *         O7 or_dense_matrix               eq. (7) as a dense matrix
 *         O9 or_counts, or_direct_counts   pairs / segments per ray
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* O1: centred B-spline of degree n (textbook piecewise form).              */
/* beta^0 = 1 on (-1/2, 1/2); beta^n = beta^0 * beta^(n-1); support (-h, h) */
/* with h = (n + 1)/2.                                                      */
/* ------------------------------------------------------------------------ */
double or_bspline(int n, double x)
{
    double a = fabs(x);
    switch (n) {
    case 0:
        return a < 0.5 ? 1.0 : 0.0;
    case 1:
        return a < 1.0 ? 1.0 - a : 0.0;
    case 2:
        if (a < 0.5) return 0.75 - a * a;
        if (a < 1.5) { double t = 1.5 - a; return 0.5 * t * t; }
        return 0.0;
    case 3:
        if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
        if (a < 2.0) { double t = 2.0 - a; return t * t * t / 6.0; }
        return 0.0;
    default:
        return NAN;
    }
}

/* Truncated-power form (1/n!) sum_j (-1)^j C(n+1, j) (x + h - j)_+^n, used
 * only to cross-check the piecewise form.  (z)_+^0 is 1 for z > 0. */
double or_bspline_tp(int n, double x)
{
    if (n < 0 || n > 7) return NAN;
    double h = 0.5 * (n + 1), s = 0.0, fact = 1.0, binom = 1.0;
    for (int i = 2; i <= n; ++i) fact *= i;
    for (int j = 0; j <= n + 1; ++j) {
        double z = x + h - j;
        if (z > 0.0) s += ((j & 1) ? -1.0 : 1.0) * binom * (n == 0 ? 1.0 : pow(z, n));
        binom = binom * (n + 1 - j) / (j + 1);
    }
    return s / fact;
}

/* ------------------------------------------------------------------------ */
/* O2: m-point Gauss-Legendre rule on [-1, 1].  Nodes are the roots of the  */
/* Legendre polynomial P_m found by Newton's method from Chebyshev-like     */
/* starting points; weights 2 / ((1 - x^2) P_m'(x)^2).                      */
/* ------------------------------------------------------------------------ */
int or_gauss_legendre(int m, double *nodes, double *weights)
{
    if (m < 1 || m > 64) return 1;
    for (int i = 0; i < m; ++i) {
        double x = cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;            /* P_0, P_1 */
            if (m == 1) { p1 = x; p0 = 1.0; }
            for (int k = 2; k <= m; ++k) {      /* Bonnet recurrence */
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            /* p1 = P_m(x), p0 = P_{m-1}(x) */
            dp = m * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        {   /* recompute the derivative at the converged node */
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= m; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = m * (x * p1 - p0) / (x * x - 1.0);
        }
        nodes[m - 1 - i] = x;                   /* ascending order */
        weights[m - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    if (m == 1) { nodes[0] = 0.0; weights[0] = 2.0; }
    return 0;
}

/* GL order that integrates a degree-3n polynomial exactly: 2m - 1 >= 3n. */
static int gl_order(int n) { return (3 * n + 2) / 2 > 0 ? (3 * n + 2) / 2 : 1; }

static double GLX[8][8], GLW[8][8];
__attribute__((constructor)) static void init_gl(void)
{
    for (int m = 1; m < 8; ++m) or_gauss_legendre(m, GLX[m], GLW[m]);
}

/* ------------------------------------------------------------------------ */
/* Neumaier compensated summation.                                          */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } ksum;
static inline void ks_add(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static inline double ks_val(const ksum *k) { return k->s + k->c; }

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* O4: footprint of one basis, P phi(w, x) = int phi(x + t w) dt.           */
/* The chord of the open support cube (-h, h)^3 comes from a slab test; the */
/* interior knot planes x_i + t w_i = kappa (kappa = -h+1, ..., h-1) split  */
/* it into <= 3n + 1 polynomial segments, each integrated by GL.            */
/* nseg (may be NULL) receives the number of non-empty segments.            */
/* ------------------------------------------------------------------------ */
static double footprint_impl(int n, const double w[3], const double x[3], int *nseg)
{
    double h = 0.5 * (n + 1);
    double t0 = -INFINITY, t1 = INFINITY;
    if (nseg) *nseg = 0;
    if (w[0] == 0.0 && w[1] == 0.0 && w[2] == 0.0) return NAN;
    for (int i = 0; i < 3; ++i) {
        if (w[i] == 0.0) {
            if (!(fabs(x[i]) < h)) return 0.0;
        } else {
            double ta = (-h - x[i]) / w[i], tb = (h - x[i]) / w[i];
            t0 = fmax(t0, fmin(ta, tb));
            t1 = fmin(t1, fmax(ta, tb));
        }
    }
    if (!(t0 < t1)) return 0.0;
    double T[3 * 8 + 2];
    int nt = 0;
    T[nt++] = t0;
    T[nt++] = t1;
    for (int i = 0; i < 3; ++i) {
        if (w[i] == 0.0) continue;
        for (int j = 1; j <= n; ++j) {
            double t = (-h + j - x[i]) / w[i];
            if (t > t0 && t < t1) T[nt++] = t;
        }
    }
    qsort(T, nt, sizeof(double), cmp_double);
    int m = gl_order(n);
    ksum acc = {0.0, 0.0};
    for (int k = 0; k + 1 < nt; ++k) {
        double a = T[k], b = T[k + 1];
        if (!(b > a)) continue;
        double mid = 0.5 * (a + b), half = 0.5 * (b - a), s = 0.0;
        for (int l = 0; l < m; ++l) {
            double t = mid + half * GLX[m][l];
            s += GLW[m][l] * or_bspline(n, x[0] + t * w[0]) * or_bspline(n, x[1] + t * w[1])
                 * or_bspline(n, x[2] + t * w[2]);
        }
        ks_add(&acc, half * s);
        if (nseg) ++*nseg;
    }
    return ks_val(&acc);
}

double or_footprint(int n, const double w[3], const double x[3])
{
    return footprint_impl(n, w, x, NULL);
}

/* Vectorised form: cnt (w, x) pairs laid out as w[cnt][3], x[cnt][3]. */
int or_footprint_many(int n, int64_t cnt, const double *w, const double *x, double *out)
{
    if (n < 0 || n > 3) return 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < cnt; ++i) out[i] = footprint_impl(n, w + 3 * i, x + 3 * i, NULL);
    return 0;
}

int or_bspline_many(int n, int64_t cnt, const double *x, double *out, int tp)
{
    for (int64_t i = 0; i < cnt; ++i) out[i] = tp ? or_bspline_tp(n, x[i]) : or_bspline(n, x[i]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Rays from the 12-float view vectors.  Ray index r = (v * R + j) * C + i  */
/* (view, detector row, detector column).  Pixel centre offset from d0 is   */
/* (i - (C-1)/2) du + (j - (R-1)/2) dv.                                     */
/*   parallel (kind 0): vec = (w, d0, du, dv); anchor = pixel centre,       */
/*                      direction = w / |w|;                                */
/*   cone     (kind 1): vec = (src, d0, du, dv); anchor = src, direction =  */
/*                      (pixel centre - src) / |...|.                       */
/* The whole line is integrated in both cases.                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind, V, R, C;
    const float *vecs;
} geom_t;

static int make_ray(const geom_t *g, int64_t r, double a[3], double w[3])
{
    int64_t i = r % g->C, j = (r / g->C) % g->R, v = r / ((int64_t)g->C * g->R);
    const float *e = g->vecs + 12 * v;
    double ci = (double)i - 0.5 * (g->C - 1), cj = (double)j - 0.5 * (g->R - 1);
    double p[3];
    for (int k = 0; k < 3; ++k) p[k] = (double)e[3 + k] + ci * (double)e[6 + k] + cj * (double)e[9 + k];
    double d[3];
    if (g->kind == 0) {
        for (int k = 0; k < 3; ++k) { d[k] = e[k]; a[k] = p[k]; }
    } else {
        for (int k = 0; k < 3; ++k) { d[k] = p[k] - (double)e[k]; a[k] = e[k]; }
    }
    double nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(nrm > 0.0)) return 1;
    for (int k = 0; k < 3; ++k) w[k] = d[k] / nrm;
    return 0;
}

int or_make_rays(int kind, int V, int R, int C, const float *vecs, const int64_t *rays,
                 int64_t nrays, double *a_out, double *w_out)
{
    geom_t g = {kind, V, R, C, vecs};
    for (int64_t k = 0; k < nrays; ++k) {
        int64_t r = rays ? rays[k] : k;
        if (make_ray(&g, r, a_out + 3 * k, w_out + 3 * k)) return 1;
    }
    return 0;
}

/* Clip the line a + t w to the open box prod (lo_i, hi_i).  Returns 0 if
 * the intersection is empty. */
static int clip_box(const double a[3], const double w[3], const double lo[3], const double hi[3],
                    double *t0, double *t1)
{
    double s0 = -INFINITY, s1 = INFINITY;
    for (int i = 0; i < 3; ++i) {
        if (w[i] == 0.0) {
            if (!(a[i] > lo[i] && a[i] < hi[i])) return 0;
        } else {
            double ta = (lo[i] - a[i]) / w[i], tb = (hi[i] - a[i]) / w[i];
            s0 = fmax(s0, fmin(ta, tb));
            s1 = fmin(s1, fmax(ta, tb));
        }
    }
    *t0 = s0;
    *t1 = s1;
    return s0 < s1;
}

/* ------------------------------------------------------------------------ */
/* O3: direct integral of f = sum_k c_k phi(. - x_k) along one ray.         */
/* Clip to the support-padded box, cut at every knot plane the ray crosses, */
/* integrate f exactly on each segment with GL.                             */
/* ------------------------------------------------------------------------ */
static double ray_direct(int n, const float *c, const int64_t N[3], const double a[3],
                         const double w[3], double *T /* workspace */)
{
    double h = 0.5 * (n + 1), o[3], lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
        o[i] = -0.5 * (double)(N[i] - 1);
        lo[i] = o[i] - h;
        hi[i] = o[i] + (double)(N[i] - 1) + h;
    }
    double t0, t1;
    if (!clip_box(a, w, lo, hi, &t0, &t1)) return 0.0;
    double kap = (n & 1) ? 0.0 : 0.5;   /* knot planes sit at o + kap + integer */
    int64_t nt = 0;
    T[nt++] = t0;
    T[nt++] = t1;
    for (int i = 0; i < 3; ++i) {
        if (w[i] == 0.0) continue;
        double xa = a[i] + t0 * w[i], xb = a[i] + t1 * w[i];
        double xl = fmin(xa, xb), xh = fmax(xa, xb);
        int64_t m0 = (int64_t)floor(xl - o[i] - kap) - 1, m1 = (int64_t)ceil(xh - o[i] - kap) + 1;
        for (int64_t mm = m0; mm <= m1; ++mm) {
            double t = (o[i] + kap + (double)mm - a[i]) / w[i];
            if (t > t0 && t < t1) T[nt++] = t;
        }
    }
    qsort(T, nt, sizeof(double), cmp_double);
    int m = gl_order(n);
    ksum acc = {0.0, 0.0};
    double bw[3][8];
    for (int64_t s = 0; s + 1 < nt; ++s) {
        double ta = T[s], tb = T[s + 1];
        if (!(tb > ta)) continue;
        double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
        int64_t klo[3], khi[3];
        int empty = 0;
        for (int i = 0; i < 3; ++i) {
            double xm = a[i] + mid * w[i];
            klo[i] = (int64_t)floor(xm - o[i] - h) + 1;
            khi[i] = (int64_t)ceil(xm - o[i] + h) - 1;
            if (klo[i] < 0) klo[i] = 0;
            if (khi[i] > N[i] - 1) khi[i] = N[i] - 1;
            if (klo[i] > khi[i]) empty = 1;
        }
        if (empty) continue;
        double seg = 0.0;
        for (int l = 0; l < m; ++l) {
            double t = mid + half * GLX[m][l];
            for (int i = 0; i < 3; ++i) {
                double xi = a[i] + t * w[i];
                for (int64_t k = klo[i]; k <= khi[i]; ++k)
                    bw[i][k - klo[i]] = or_bspline(n, xi - (o[i] + (double)k));
            }
            double f = 0.0;
            for (int64_t k3 = klo[2]; k3 <= khi[2]; ++k3)
                for (int64_t k2 = klo[1]; k2 <= khi[1]; ++k2)
                    for (int64_t k1 = klo[0]; k1 <= khi[0]; ++k1)
                        f += (double)c[(k3 * N[1] + k2) * N[0] + k1] * bw[0][k1 - klo[0]]
                             * bw[1][k2 - klo[1]] * bw[2][k3 - klo[2]];
            seg += GLW[m][l] * f;
        }
        ks_add(&acc, half * seg);
    }
    return ks_val(&acc);
}

/* Number of non-empty polynomial segments of the direct integral: the
 * knot cells of the padded box the line passes through. */
static int64_t ray_direct_segments(int n, const int64_t N[3], const double a[3], const double w[3],
                                   double *T)
{
    double h = 0.5 * (n + 1), o[3], lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
        o[i] = -0.5 * (double)(N[i] - 1);
        lo[i] = o[i] - h;
        hi[i] = o[i] + (double)(N[i] - 1) + h;
    }
    double t0, t1;
    if (!clip_box(a, w, lo, hi, &t0, &t1)) return 0;
    double kap = (n & 1) ? 0.0 : 0.5;
    int64_t nt = 0;
    T[nt++] = t0;
    T[nt++] = t1;
    for (int i = 0; i < 3; ++i) {
        if (w[i] == 0.0) continue;
        double xa = a[i] + t0 * w[i], xb = a[i] + t1 * w[i];
        double xl = fmin(xa, xb), xh = fmax(xa, xb);
        int64_t m0 = (int64_t)floor(xl - o[i] - kap) - 1, m1 = (int64_t)ceil(xh - o[i] - kap) + 1;
        for (int64_t mm = m0; mm <= m1; ++mm) {
            double t = (o[i] + kap + (double)mm - a[i]) / w[i];
            if (t > t0 && t < t1) T[nt++] = t;
        }
    }
    qsort(T, nt, sizeof(double), cmp_double);
    int64_t segs = 0;
    for (int64_t s = 0; s + 1 < nt; ++s)
        if (T[s + 1] > T[s]) ++segs;
    return segs;
}

static int check_args(int n, const int64_t N[3], int kind, int V, int R, int C)
{
    if (n < 0 || n > 3) return 1;
    if (kind != 0 && kind != 1) return 1;
    if (V < 1 || R < 1 || C < 1) return 1;
    for (int i = 0; i < 3; ++i)
        if (N[i] < 1) return 1;
    return 0;
}

int or_project(int n, const float *c, const int64_t N[3], int kind, int V, int R, int C,
               const float *vecs, const int64_t *rays, int64_t nrays, double *out)
{
    if (check_args(n, N, kind, V, R, C)) return 1;
    geom_t g = {kind, V, R, C, vecs};
    int64_t cap = 2 + 3 * (N[0] + N[1] + N[2]) + 32;
    int bad = 0;
#pragma omp parallel
    {
        double *T = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < nrays; ++k) {
            double a[3], w[3];
            int64_t r = rays ? rays[k] : k;
            if (make_ray(&g, r, a, w)) { out[k] = NAN; bad = 1; continue; }
            out[k] = ray_direct(n, c, N, a, w, T);
        }
        free(T);
    }
    return bad;
}

/* O3 on explicitly given lines a_k + t w_k (w_k unit): the same direct     */
/* integral as or_project, for lines that do not come from a geometry.      */
int or_project_lines(int n, const float *c, const int64_t N[3], int64_t nlines, const double *a,
                     const double *w, double *out)
{
    if (n < 0 || n > 3) return 1;
    for (int i = 0; i < 3; ++i)
        if (N[i] < 1) return 1;
    int64_t cap = 2 + 3 * (N[0] + N[1] + N[2]) + 32;
#pragma omp parallel
    {
        double *T = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < nlines; ++k) out[k] = ray_direct(n, c, N, a + 3 * k, w + 3 * k, T);
        free(T);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Enumerate every basis q in the index box whose open support meets the    */
/* ray, by nested clipping of the ray's parameter interval axis by axis     */
/* (axis 3, then 2, then 1).  Calls visit(q, xloc) with xloc = a - x_q.     */
/* ------------------------------------------------------------------------ */
typedef void (*visit_fn)(void *ctx, int64_t q, const double xloc[3]);

static void clip_axis(double ai, double wi, double xk, double h, double t0, double t1, double *s0,
                      double *s1)
{
    if (wi == 0.0) {
        if (fabs(ai - xk) < h) { *s0 = t0; *s1 = t1; }
        else { *s0 = 1.0; *s1 = 0.0; }
        return;
    }
    double ta = (xk - h - ai) / wi, tb = (xk + h - ai) / wi;
    *s0 = fmax(t0, fmin(ta, tb));
    *s1 = fmin(t1, fmax(ta, tb));
}

static void axis_range(double ai, double wi, double o, double h, int64_t Nn, double t0, double t1,
                       int64_t *k0, int64_t *k1)
{
    double xa = ai + t0 * wi, xb = ai + t1 * wi;
    double xl = fmin(xa, xb), xh = fmax(xa, xb);
    *k0 = (int64_t)floor(xl - o - h) - 1;
    *k1 = (int64_t)ceil(xh - o + h) + 1;
    if (*k0 < 0) *k0 = 0;
    if (*k1 > Nn - 1) *k1 = Nn - 1;
}

static void enumerate_pairs(int n, const int64_t N[3], const double a[3], const double w[3],
                            visit_fn visit, void *ctx)
{
    double h = 0.5 * (n + 1), o[3], lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
        o[i] = -0.5 * (double)(N[i] - 1);
        lo[i] = o[i] - h;
        hi[i] = o[i] + (double)(N[i] - 1) + h;
    }
    double t0, t1;
    if (!clip_box(a, w, lo, hi, &t0, &t1)) return;
    int64_t a0, a1;
    axis_range(a[2], w[2], o[2], h, N[2], t0, t1, &a0, &a1);
    for (int64_t q3 = a0; q3 <= a1; ++q3) {
        double s0, s1;
        clip_axis(a[2], w[2], o[2] + (double)q3, h, t0, t1, &s0, &s1);
        if (!(s0 < s1)) continue;
        int64_t b0, b1;
        axis_range(a[1], w[1], o[1], h, N[1], s0, s1, &b0, &b1);
        for (int64_t q2 = b0; q2 <= b1; ++q2) {
            double u0, u1;
            clip_axis(a[1], w[1], o[1] + (double)q2, h, s0, s1, &u0, &u1);
            if (!(u0 < u1)) continue;
            int64_t c0, c1;
            axis_range(a[0], w[0], o[0], h, N[0], u0, u1, &c0, &c1);
            for (int64_t q1 = c0; q1 <= c1; ++q1) {
                double v0, v1;
                clip_axis(a[0], w[0], o[0] + (double)q1, h, u0, u1, &v0, &v1);
                if (!(v0 < v1)) continue;
                double xl[3] = {a[0] - (o[0] + (double)q1), a[1] - (o[1] + (double)q2),
                                a[2] - (o[2] + (double)q3)};
                visit(ctx, (q3 * N[1] + q2) * N[0] + q1, xl);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* O5: the same transform as the sum over bases of c_q * footprint (eq. 4). */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    const double *w;
    const float *c;
    ksum acc;
    int64_t pairs, segs;
} bsum_ctx;

static void bsum_visit(void *vctx, int64_t q, const double xl[3])
{
    bsum_ctx *b = (bsum_ctx *)vctx;
    int ns = 0;
    double fp = footprint_impl(b->n, b->w, xl, &ns);
    if (b->c) ks_add(&b->acc, (double)b->c[q] * fp);
    b->pairs += 1;
    b->segs += ns;
}

int or_project_basis_sum(int n, const float *c, const int64_t N[3], int kind, int V, int R, int C,
                         const float *vecs, const int64_t *rays, int64_t nrays, double *out)
{
    if (check_args(n, N, kind, V, R, C)) return 1;
    geom_t g = {kind, V, R, C, vecs};
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrays; ++k) {
        double a[3], w[3];
        int64_t r = rays ? rays[k] : k;
        if (make_ray(&g, r, a, w)) { out[k] = NAN; bad = 1; continue; }
        bsum_ctx b = {n, w, c, {0.0, 0.0}, 0, 0};
        enumerate_pairs(n, N, a, w, bsum_visit, &b);
        out[k] = ks_val(&b.acc);
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* O9: per-ray count of (ray, basis) pairs with a non-empty chord, and of   */
/* the polynomial segments their footprints split into.                     */
/* ------------------------------------------------------------------------ */
int or_counts(int n, const int64_t N[3], int kind, int V, int R, int C, const float *vecs,
              const int64_t *rays, int64_t nrays, int64_t *pairs, int64_t *segs)
{
    if (check_args(n, N, kind, V, R, C)) return 1;
    geom_t g = {kind, V, R, C, vecs};
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrays; ++k) {
        double a[3], w[3];
        int64_t r = rays ? rays[k] : k;
        pairs[k] = 0;
        segs[k] = 0;
        if (make_ray(&g, r, a, w)) { bad = 1; continue; }
        bsum_ctx b = {n, w, NULL, {0.0, 0.0}, 0, 0};
        enumerate_pairs(n, N, a, w, bsum_visit, &b);
        pairs[k] = b.pairs;
        segs[k] = b.segs;
    }
    return bad;
}

int or_direct_counts(int n, const int64_t N[3], int kind, int V, int R, int C, const float *vecs,
                     const int64_t *rays, int64_t nrays, int64_t *segs)
{
    if (check_args(n, N, kind, V, R, C)) return 1;
    geom_t g = {kind, V, R, C, vecs};
    int64_t cap = 2 + 3 * (N[0] + N[1] + N[2]) + 32;
    int bad = 0;
#pragma omp parallel
    {
        double *T = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nrays; ++k) {
            double a[3], w[3];
            int64_t r = rays ? rays[k] : k;
            segs[k] = 0;
            if (make_ray(&g, r, a, w)) { bad = 1; continue; }
            segs[k] = ray_direct_segments(n, N, a, w, T);
        }
        free(T);
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* O6: transpose of eq. (7), voxel-driven, for a subset of coefficients.    */
/* (A^T y)_q = sum_r y_r P phi(w_r, a_r - x_q).  For each view the 8        */
/* corners of q's support cube are mapped to continuous detector            */
/* coordinates; every pixel of the integer box around them (widened by one) */
/* is visited, footprints of rays that miss the support are exactly zero.   */
/* ------------------------------------------------------------------------ */
static double det3(const double m[3][3])
{
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
           - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
           + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

/* Solve [c0 c1 c2] z = rhs (columns c0, c1, c2) by Cramer's rule. */
static int solve3(const double c0[3], const double c1[3], const double c2[3], const double rhs[3],
                  double z[3])
{
    double M[3][3];
    for (int i = 0; i < 3; ++i) { M[i][0] = c0[i]; M[i][1] = c1[i]; M[i][2] = c2[i]; }
    double D = det3(M);
    if (!(fabs(D) > 1e-300)) return 1;
    for (int col = 0; col < 3; ++col) {
        double Mc[3][3];
        memcpy(Mc, M, sizeof(M));
        for (int i = 0; i < 3; ++i) Mc[i][col] = rhs[i];
        z[col] = det3(Mc) / D;
    }
    return 0;
}

/* Pixel box [i0, i1] x [j0, j1] that holds every ray meeting the open cube
 * centred at xc with half-side h; falls back to the whole detector when the
 * projection is degenerate. */
static void shadow_box(const geom_t *g, int v, const double xc[3], double h, int64_t *i0,
                       int64_t *i1, int64_t *j0, int64_t *j1)
{
    const float *e = g->vecs + 12 * v;
    double d0[3], du[3], dv[3], s[3];
    for (int k = 0; k < 3; ++k) {
        s[k] = e[k];
        d0[k] = e[3 + k];
        du[k] = e[6 + k];
        dv[k] = e[9 + k];
    }
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    int full = 0, sign = 0;
    for (int corner = 0; corner < 8 && !full; ++corner) {
        double X[3];
        for (int k = 0; k < 3; ++k) X[k] = xc[k] + (((corner >> k) & 1) ? h : -h);
        double z[3];
        if (g->kind == 0) {
            /* X = d0 + alpha du + beta dv + t w */
            double rhs[3] = {X[0] - d0[0], X[1] - d0[1], X[2] - d0[2]};
            if (solve3(du, dv, s, rhs, z)) { full = 1; break; }
        } else {
            /* d0 + alpha du + beta dv = s + lambda (X - s) */
            double mx[3] = {-(X[0] - s[0]), -(X[1] - s[1]), -(X[2] - s[2])};
            double rhs[3] = {s[0] - d0[0], s[1] - d0[1], s[2] - d0[2]};
            if (solve3(du, dv, mx, rhs, z)) { full = 1; break; }
            int sg = z[2] > 0.0 ? 1 : (z[2] < 0.0 ? -1 : 0);
            if (sg == 0 || (sign != 0 && sg != sign)) { full = 1; break; }
            sign = sg;
        }
        umin = fmin(umin, z[0]);
        umax = fmax(umax, z[0]);
        vmin = fmin(vmin, z[1]);
        vmax = fmax(vmax, z[1]);
    }
    if (full) {
        *i0 = 0; *i1 = g->C - 1; *j0 = 0; *j1 = g->R - 1;
        return;
    }
    double ci = 0.5 * (g->C - 1), cj = 0.5 * (g->R - 1);
    *i0 = (int64_t)floor(umin + ci) - 1;
    *i1 = (int64_t)ceil(umax + ci) + 1;
    *j0 = (int64_t)floor(vmin + cj) - 1;
    *j1 = (int64_t)ceil(vmax + cj) + 1;
    if (*i0 < 0) *i0 = 0;
    if (*j0 < 0) *j0 = 0;
    if (*i1 > g->C - 1) *i1 = g->C - 1;
    if (*j1 > g->R - 1) *j1 = g->R - 1;
}

int or_backproject_subset(int n, const float *y, const int64_t N[3], int kind, int V, int R, int C,
                          const float *vecs, const int64_t *coefs, int64_t ncoef, double *out)
{
    if (check_args(n, N, kind, V, R, C)) return 1;
    geom_t g = {kind, V, R, C, vecs};
    double h = 0.5 * (n + 1);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < ncoef; ++k) {
        int64_t q = coefs ? coefs[k] : k;
        int64_t q1 = q % N[0], q2 = (q / N[0]) % N[1], q3 = q / (N[0] * N[1]);
        double xc[3] = {(double)q1 - 0.5 * (double)(N[0] - 1), (double)q2 - 0.5 * (double)(N[1] - 1),
                        (double)q3 - 0.5 * (double)(N[2] - 1)};
        ksum acc = {0.0, 0.0};
        for (int v = 0; v < V; ++v) {
            int64_t i0, i1, j0, j1;
            shadow_box(&g, v, xc, h, &i0, &i1, &j0, &j1);
            for (int64_t j = j0; j <= j1; ++j)
                for (int64_t i = i0; i <= i1; ++i) {
                    int64_t r = ((int64_t)v * R + j) * C + i;
                    double a[3], w[3];
                    if (make_ray(&g, r, a, w)) { bad = 1; continue; }
                    double xl[3] = {a[0] - xc[0], a[1] - xc[1], a[2] - xc[2]};
                    double fp = footprint_impl(n, w, xl, NULL);
                    if (fp != 0.0) ks_add(&acc, (double)y[r] * fp);
                }
        }
        out[k] = ks_val(&acc);
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* O7: dense forward matrix A[k][q] = P phi(w_r, a_r - x_q) for the rays     */
/* r = rays[k] (all rays if NULL) and every coefficient q.                  */
/* ------------------------------------------------------------------------ */
int or_dense_matrix(int n, const int64_t N[3], int kind, int V, int R, int C, const float *vecs,
                    const int64_t *rays, int64_t nrays, double *A)
{
    if (check_args(n, N, kind, V, R, C)) return 1;
    geom_t g = {kind, V, R, C, vecs};
    int64_t nq = N[0] * N[1] * N[2];
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nrays; ++k) {
        double a[3], w[3];
        int64_t r = rays ? rays[k] : k;
        if (make_ray(&g, r, a, w)) { bad = 1; continue; }
        for (int64_t q = 0; q < nq; ++q) {
            int64_t q1 = q % N[0], q2 = (q / N[0]) % N[1], q3 = q / (N[0] * N[1]);
            double xl[3] = {a[0] - ((double)q1 - 0.5 * (double)(N[0] - 1)),
                            a[1] - ((double)q2 - 0.5 * (double)(N[1] - 1)),
                            a[2] - ((double)q3 - 0.5 * (double)(N[2] - 1))};
            A[k * nq + q] = footprint_impl(n, w, xl, NULL);
        }
    }
    return bad;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Number of OpenMP threads of the following calls (timing of the oracle on
 * one core and on all of them); k < 1 restores the default. */
void or_set_num_threads(int k)
{
#ifdef _OPENMP
    static int deflt = 0;
    if (deflt == 0) deflt = omp_get_max_threads();
    omp_set_num_threads(k >= 1 ? k : deflt);
#else
    (void)k;
#endif
}
