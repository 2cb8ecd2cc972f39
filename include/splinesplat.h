/*
 * splinesplat.h -- C ABI of the MI355X (gfx950) spline x-ray transform.
 *
 * The library computes the forward model of "SplineSplat: 3D Ray Tracing for
 * Higher-Quality Tomography" (arXiv 2511.11078) and its transpose:
 *
 *   forward   y_m = P f(w_m, s_m) = sum_k c_k P phi(w_m, s_m - Proj k)     (eq. (2), (4), (7))
 *   adjoint   (A^T y)_k = sum_m y_m P phi(w_m, s_m - Proj k)               (transpose of eq. (7))
 *
 * for a volume f = sum_k c_k phi(. - x_k) (eq. (3)) on the unit lattice,
 * phi the tensor-product centred B-spline of degree n (Sec. 2.2 uses n = 2;
 * n = 3 is the default of the benchmark workloads; n = 0 is the voxel basis
 * of the baseline in Sec. 3).  The forward walks every line through the
 * lattice slab by slab along its dominant axis (Definition 2.1) and sums
 * coefficient x footprint over every basis whose support the line crosses
 * (projection algorithm and neighbour search of Sec. 2.3).  The footprint
 * P phi(w, x) = int phi(x + t w) dt is evaluated either
 *   - exactly, by piecewise Gauss-Legendre quadrature in FP32
 *     (SS_FORM_QUAD_FP32: integrated knot cell by knot cell along each line,
 *     the nodes of a cell shared by the bases covering it; or
 *     SS_FORM_QUAD_PAIR_FP32: per (line, basis) pair on the network's walk), or
 *   - by the learned network f_theta of Sec. 2.2 (SS_FORM_MLP_BF16):
 *     5 -> 4 x 64 (SiLU) -> 1, hidden layers on BF16 matrix cores with FP32
 *     accumulation, gated by the exact line/support intersection test.
 * The adjoint (Sec. 2.3 states that the projection algorithm with minor
 * changes gives a matched adjoint) is a gather: each coefficient sums over
 * the detector pixels of its own shadow and has a single writer (no atomic
 * operations in device memory; results are deterministic).
 *
 * Conventions shared by every entry point
 *   - Coefficient k = (k1, k2, k3) sits at world position
 *     x_k = k - (N - 1)/2 per axis; c is FP32, laid out [N3][N2][N1]
 *     (k1 fastest).  Coefficients outside the index box are zero.
 *   - Sinograms are FP32 [n_views][det_rows][det_cols] (column fastest).
 *     Pixel (view v, row j, column i) is one line: the line through
 *     d0 + (i - (C-1)/2) du + (j - (R-1)/2) dv, with direction w
 *     (parallel beam) or through the source (cone beam).  The whole line
 *     is integrated (eq. (2) integrates over all t).
 *   - Pointers named d_* are DEVICE pointers on the context's GPU, owned by
 *     the caller.  Outputs are always overwritten, never accumulated into.
 *   - Every call enqueues work on `hip_stream` (a hipStream_t; NULL = the
 *     default stream) and returns without waiting.  Argument errors are
 *     detected on the host before anything is enqueued and return a
 *     non-zero ss_status with nothing launched; launch failures return
 *     SS_EDEVICE.  Faults inside kernels surface at the caller's next
 *     synchronisation.
 *   - A context may be used from one host thread at a time, and its calls
 *     must be ordered on one stream (the geometry it uploads is shared by
 *     consecutive calls).
 *   - ss_last_error() returns a thread-local description of the last
 *     failure on the calling thread.
 */
#ifndef SPLINESPLAT_H
#define SPLINESPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 1: first release; 2: adds SS_FORM_QUAD_PAIR_FP32, ss_project_noalloc and
 * ss_set_scratch_limit (calls and arguments of version 1 unchanged). */
#define SS_ABI_VERSION 2

typedef enum {
    SS_OK = 0,
    SS_EINVAL = 1,         /* bad argument (null pointer, size, non-finite geometry, ...) */
    SS_ENOMEM = 2,         /* device or host allocation of library-internal memory failed */
    SS_EDEVICE = 3,        /* HIP runtime / launch error                                  */
    SS_EUNSUPPORTED = 4,   /* degree or form not built into this library                   */
    SS_EBLOB = 5           /* network weight blob malformed or not matching the context    */
} ss_status;

typedef enum {
    SS_FORM_QUAD_FP32 = 0,      /* exact piecewise Gauss-Legendre footprint, FP32 */
    SS_FORM_MLP_BF16 = 1,       /* learned footprint, BF16 MFMA + FP32 accumulate */
    SS_FORM_QUAD_PAIR_FP32 = 2  /* the exact FP32 footprint evaluated per (line, basis)
                                   pair on the traversal of SS_FORM_MLP_BF16: the same
                                   slab windows (forward) and coefficient-brick gather
                                   (adjoint), only the footprint differs -- the
                                   reference point for the network's speed (Sec. 2.2) */
} ss_form;

typedef enum {
    SS_GEOM_PARALLEL = 0,
    SS_GEOM_CONE = 1
} ss_geom_kind;

/* Acquisition geometry (host memory; copied to the device by the calls that
 * take it).  vecs holds n_views x 12 floats per view:
 *   parallel: (w[3], d0[3], du[3], dv[3])   w need not be normalised
 *   cone:     (src[3], d0[3], du[3], dv[3])
 * in world units (coefficient spacing).  This is the line parameterisation
 * of eq. (1): one (w_m, s_m) per detector pixel. */
typedef struct {
    int32_t kind;          /* ss_geom_kind */
    int32_t n_views;       /* >= 1 */
    int32_t det_rows;      /* >= 1 */
    int32_t det_cols;      /* >= 1 */
    const float *vecs;     /* host pointer, n_views * 12 floats */
} ss_geometry;

typedef struct ss_ctx ss_ctx;

/* Create a context on HIP device `device` for basis degree `degree`
 * (0..3) and footprint form `form`.  For SS_FORM_MLP_BF16, `mlp_blob` /
 * `blob_bytes` is a host copy of the trained network (layout below); the
 * weights are uploaded once and owned by the context.  For
 * SS_FORM_QUAD_FP32 and SS_FORM_QUAD_PAIR_FP32 pass NULL, 0.
 * Blob layout (little endian): char magic[8] = "SSMLP\0\0\1"; uint32
 * version (1), degree, in (5), hidden (64), depth (4), activation (1 = SiLU),
 * fold convention (1), training seed; float rel_l2_fp32, rel_l2_bf16; then
 * W1[64][5] f32, b1[64] f32, 3 x (W[64][64] bf16 row-major [out][in],
 * b[64] f32), Wout[64] f32, bout f32.
 * Errors: SS_EINVAL (out == NULL, bad degree/form, a blob given to an exact
 * form), SS_EUNSUPPORTED (MLP form with degree 0), SS_EBLOB, SS_EDEVICE,
 * SS_ENOMEM. */
ss_status ss_create(ss_ctx **out, int device, int degree, ss_form form,
                    const void *mlp_blob, size_t blob_bytes);

/* Release a context and its device memory (waits for nothing: the caller
 * must make sure no enqueued call still uses it).  NULL is accepted. */
ss_status ss_destroy(ss_ctx *ctx);

/* Forward transform, eq. (7): d_sino[v][j][i] = sum_k c_k P phi(w, s - Proj k)
 * for every pixel line.  d_coeffs: FP32 [dims[2]][dims[1]][dims[0]];
 * d_sino: FP32 [n_views][det_rows][det_cols], overwritten.
 * With SS_FORM_QUAD_FP32 the context's device scratch (the one described
 * at ss_backproject) first receives a zero-padded copy of d_coeffs,
 * (dims + 2 degree + 2) floats per axis.
 * Errors: SS_EINVAL (null pointers, dims < 1 or > 4096, non-finite vecs,
 * zero-length ray direction, more than 2^31 rays per call), SS_ENOMEM. */
ss_status ss_project(ss_ctx *ctx, const float *d_coeffs, const int64_t dims[3],
                     const ss_geometry *geom, float *d_sino, void *hip_stream);

/* Adjoint (exact transpose of ss_project up to FP32 rounding):
 * d_coeffs[k] = sum over lines m of d_sino[m] * P phi(w_m, s_m - Proj k),
 * overwritten.  Same layouts and errors as ss_project.
 * With SS_FORM_QUAD_FP32 the context keeps a device table of (degree+1)^3
 * floats per knot cell of the support-padded volume (4.45 GB for 256^3,
 * 35.6 GB for 512^3, degree 3), allocated on the first call that needs it
 * and at most the context's scratch limit (64 GiB unless set with
 * ss_set_scratch_limit; a larger table is processed in z-chunks of cell
 * layers, recomputing `degree` layers at each chunk boundary; the result
 * equals one pass up to FP32 rounding, as the cell bricks align to each
 * chunk's first layer); growing it waits for the device.  Calls on one
 * context must not overlap in time (they share the table).  Additional
 * error: SS_ENOMEM when the table cannot be allocated. */
ss_status ss_backproject(ss_ctx *ctx, const float *d_sino, const ss_geometry *geom,
                         const int64_t dims[3], float *d_coeffs, void *hip_stream);

/* Allocation-free forward, for callers that cannot allocate device memory
 * (code under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Computes what ss_project computes with a SS_FORM_QUAD_FP32
 * context of degree `degree` (0..3) on HIP device `device`, with the same
 * kernels and bit-identical results, but needs no context and calls no
 * allocating routine: the view vectors and the zero-padded coefficients go
 * into a static device array of the library, SS_STATIC_SCRATCH_BYTES per GPU,
 * held until the process ends.  It must hold 12 n_views floats (rounded up
 * to 64) plus (dims[k] + 2 degree + 2) floats per axis of padded volume
 * (256^3 fits at every degree); larger problems return SS_EINVAL before
 * anything is enqueued.  The view vectors are copied from the caller's host
 * memory with hipMemcpyAsync on hip_stream.  Every call on one GPU uses that
 * GPU's array, which keeps the last call's contents: calls that overlap in
 * time on one GPU race (order them on one stream).  Other errors as
 * ss_project. */
#define SS_STATIC_SCRATCH_BYTES ((size_t)96 << 20)
ss_status ss_project_noalloc(int device, int degree, const float *d_coeffs, const int64_t dims[3],
                             const ss_geometry *geom, float *d_sino, void *hip_stream);

/* Largest knot-cell table (bytes) the quadrature adjoint of this context
 * may allocate; 0 restores the default of 64 GiB.  Tables that would be
 * larger are processed in z-chunks (never fewer than 4 (degree+1) cell
 * layers per chunk, whatever the limit).  For callers that share the GPU's
 * memory with other work: they trade memory for recomputed layers.  A
 * scratch buffer already above the new limit is released (after waiting for
 * the device).  Errors: SS_EINVAL (ctx NULL), SS_EDEVICE. */
ss_status ss_set_scratch_limit(ss_ctx *ctx, size_t bytes);

/* Evaluate the context's footprint P phi(w, x) = int phi(x + t w) dt (the
 * contribution of eq. (4)) for `count` pairs: d_dirs FP32 [count][3] (unit
 * directions), d_offsets FP32 [count][3] (any point of the line relative to
 * the basis centre), d_out FP32 [count].  Diagnostic entry point.
 * Errors: SS_EINVAL (null pointers, count < 0 or >= 2^31). */
ss_status ss_footprint(ss_ctx *ctx, const float *d_dirs, const float *d_offsets, int64_t count,
                       float *d_out, void *hip_stream);

/* Inner product of two FP32 vectors accumulated in FP64 (deterministic
 * two-pass reduction): *d_out = sum_i a_i b_i.  n >= 0 (n = 0 writes 0).
 * Used for the scalars of the least-squares loop of Sec. 3 (eq. (6)). */
ss_status ss_dot_f64(ss_ctx *ctx, const float *d_a, const float *d_b, int64_t n, double *d_out,
                     void *hip_stream);

/* *d_out = *d_num / *d_den in FP64 on the device (0 when *d_den == 0): the
 * CGLS step length alpha = gamma / ||q||^2 and ratio beta = gamma' / gamma. */
ss_status ss_cgls_scalars(ss_ctx *ctx, const double *d_num, const double *d_den, double *d_out,
                          void *hip_stream);

/* d_y[i] += sign * (*d_alpha) * d_x[i] for i < n; sign is +1 or -1; the
 * scalar is read on the device and rounded to FP32 once. */
ss_status ss_axpy(ss_ctx *ctx, const double *d_alpha, int sign, const float *d_x, float *d_y,
                  int64_t n, void *hip_stream);

/* d_y[i] = d_x[i] + (*d_beta) * d_y[i] for i < n (CGLS direction update). */
ss_status ss_xpay(ss_ctx *ctx, const double *d_beta, const float *d_x, float *d_y, int64_t n,
                  void *hip_stream);

/* Host-only check of a problem description, the same one ss_project and
 * ss_backproject run before enqueuing anything: SS_OK, or SS_EINVAL with
 * ss_last_error() set (dims outside [1, 4096] or over 2^31 - 1
 * coefficients; geometry kind, sizes, NULL or non-finite vecs, zero
 * direction, a parallel direction inside the detector plane, a degenerate
 * detector or a cone source inside the detector plane; over 2^31 - 1 rays).
 * Needs no GPU. */
ss_status ss_validate_problem(const int64_t dims[3], const ss_geometry *geom);

/* Thread-local message describing the last failing call on this thread
 * ("" if none).  The string stays valid until the next failing call. */
const char *ss_last_error(void);

/* Degree, form and device of a context (any output pointer may be NULL). */
ss_status ss_query(const ss_ctx *ctx, int *degree, int *form, int *device);

/* SS_ABI_VERSION of the built library. */
int ss_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPLINESPLAT_H */
