// ss_abi.cpp -- the C ABI declared in include/splinesplat.h.
//
// Host-side only: argument validation (all of it before anything is
// enqueued), the context (device geometry buffer, reduction scratch, network
// weights), geometry upload on the caller's stream, and kernel dispatch per
// (degree, form).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "splinesplat.h"
#include "ss_geom_upload.hpp"
#include "ss_kernels.hpp"

struct ss_ctx {
    int device = 0;
    int degree = 3;
    int form = SS_FORM_QUAD_FP32;
    ss::GeomBuffer geom;            // device copy of the last geometry, pinned staging, upload cache
    hipEvent_t staged = nullptr;    // marks the end of the last upload's read of the staging buffer
    double *d_partials = nullptr;   // dot-product partial sums
    void *d_mlp = nullptr;          // network weights in kernel layout
    float *d_cells = nullptr;       // quadrature scratch: padded coefficients (forward), knot-cell table (adjoint)
    int64_t cells_cap = 0;          // floats
    int64_t cell_limit = ss::CELL_SCRATCH_DEFAULT_FLOATS;  // largest knot-cell table (floats)
};

namespace ss {
thread_local std::string g_err;

ss_status fail(ss_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}
}  // namespace ss

namespace {
using ss::fail;
using ss::g_err;

ss_status hip_fail(hipError_t e, const char *what) {
    return fail(SS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Switch to the context's device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

constexpr int64_t MAX_DIM = 4096;
constexpr int64_t MAX_ELEMS = (int64_t(1) << 31) - 1;

ss_status check_dims(const int64_t dims[3]) {
    if (!dims) return fail(SS_EINVAL, "dims is NULL");
    int64_t tot = 1;
    for (int k = 0; k < 3; ++k) {
        if (dims[k] < 1 || dims[k] > MAX_DIM)
            return fail(SS_EINVAL, "dims[%d] = %lld outside [1, %lld]", k, (long long)dims[k], (long long)MAX_DIM);
        tot *= dims[k];
    }
    if (tot > MAX_ELEMS) return fail(SS_EINVAL, "volume has more than 2^31 - 1 coefficients");
    return SS_OK;
}

inline double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

ss_status check_geom(const ss_geometry *g) {
    if (!g) return fail(SS_EINVAL, "geometry is NULL");
    if (g->kind != SS_GEOM_PARALLEL && g->kind != SS_GEOM_CONE)
        return fail(SS_EINVAL, "geometry kind %d is neither parallel (0) nor cone (1)", g->kind);
    if (g->n_views < 1 || g->det_rows < 1 || g->det_cols < 1)
        return fail(SS_EINVAL, "geometry sizes must be >= 1 (views %d, rows %d, cols %d)", g->n_views, g->det_rows,
                    g->det_cols);
    if (!g->vecs) return fail(SS_EINVAL, "geometry vecs is NULL");
    const int64_t rays = (int64_t)g->n_views * g->det_rows * g->det_cols;
    if (rays > MAX_ELEMS) return fail(SS_EINVAL, "more than 2^31 - 1 rays in one call");
    for (int64_t v = 0; v < g->n_views; ++v) {
        const float *e = g->vecs + 12 * v;
        double a[3], d0[3], du[3], dv[3], nrm[3];
        for (int k = 0; k < 12; ++k)
            if (!std::isfinite(e[k])) return fail(SS_EINVAL, "view %lld: non-finite geometry value", (long long)v);
        for (int k = 0; k < 3; ++k) {
            a[k] = e[k];
            d0[k] = e[3 + k];
            du[k] = e[6 + k];
            dv[k] = e[9 + k];
        }
        cross3(du, dv, nrm);
        if (g->kind == SS_GEOM_PARALLEL) {
            // w, du, dv must span space (the adjoint maps points to pixels)
            if (!(dot3(a, a) > 0.0)) return fail(SS_EINVAL, "view %lld: zero ray direction", (long long)v);
            if (!(std::fabs(dot3(nrm, a)) > 1e-12 * std::sqrt(dot3(a, a)) * std::sqrt(dot3(nrm, nrm)) &&
                  dot3(nrm, nrm) > 0.0))
                return fail(SS_EINVAL, "view %lld: direction lies in the detector plane", (long long)v);
        } else {
            if (!(dot3(nrm, nrm) > 0.0)) return fail(SS_EINVAL, "view %lld: degenerate detector", (long long)v);
            double sd[3] = {d0[0] - a[0], d0[1] - a[1], d0[2] - a[2]};
            if (!(std::fabs(dot3(sd, nrm)) > 0.0))
                return fail(SS_EINVAL, "view %lld: source lies in the detector plane", (long long)v);
        }
    }
    return SS_OK;
}

// Float offset of the per-view projections behind the view vectors.
size_t vproj_offset(size_t n_views) { return (n_views * 12 + 3) / 4 * 4; }

// HIP device operations of the geometry upload (ss_geom_upload.hpp).
struct HipUploadOps {
    hipStream_t st;
    hipEvent_t ev;
    int dev_alloc(void **p, size_t bytes) { return (int)hipMalloc(p, bytes); }
    void dev_free(void *p) { (void)hipFree(p); }
    int host_alloc(void **p, size_t bytes) { return (int)hipHostMalloc(p, bytes, hipHostMallocDefault); }
    void host_free(void *p) { (void)hipHostFree(p); }
    int device_sync() { return (int)hipDeviceSynchronize(); }
    int event_sync() { return (int)hipEventSynchronize(ev); }
    int copy_async(void *dst, const void *src, size_t bytes) {
        return (int)hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    }
    int event_record() { return (int)hipEventRecord(ev, st); }
};

// Upload the geometry if it differs from what the device buffer holds: the
// view vectors, followed by each view's detector projection (FP64, computed
// here once instead of by every block of the adjoint at every view).
ss_status upload_geom(ss_ctx *ctx, const ss_geometry *g, hipStream_t st) {
    const size_t nv = (size_t)g->n_views;
    const size_t nf = nv * 12;
    const size_t vp_off = vproj_offset(nv);
    const size_t total = vp_off + nv * (sizeof(ss::ViewProj) / sizeof(float));
    HipUploadOps ops{st, ctx->staged};
    auto fill = [&](float *stage) {
        ss::ViewProj *vp = reinterpret_cast<ss::ViewProj *>(stage + vp_off);
        for (size_t v = 0; v < nv; ++v) ss::make_viewproj(g->vecs + 12 * v, (int)g->kind, vp[v]);
    };
    int code = 0;
    const ss::UploadError r = ctx->geom.upload(ops, g->vecs, nf, (int)g->kind, total, fill, &code);
    const char *msg = hipGetErrorString((hipError_t)code);
    switch (r) {
    case ss::UPLOAD_OK: return SS_OK;
    case ss::UPLOAD_SYNC: return fail(SS_EDEVICE, "geometry upload: synchronisation: %s", msg);
    case ss::UPLOAD_DEV_ALLOC: return fail(SS_ENOMEM, "geometry buffer: %s", msg);
    case ss::UPLOAD_HOST_ALLOC: return fail(SS_ENOMEM, "geometry staging: %s", msg);
    case ss::UPLOAD_COPY: return fail(SS_EDEVICE, "geometry upload: %s", msg);
    case ss::UPLOAD_EVENT: return fail(SS_EDEVICE, "geometry upload: hipEventRecord: %s", msg);
    }
    return fail(SS_EDEVICE, "geometry upload failed");
}

// Make the quadrature scratch (padded coefficients for the forward, the
// knot-cell table for the adjoint) hold at least `need` floats.
ss_status ensure_cells(ss_ctx *ctx, int64_t need) {
    if (need <= ctx->cells_cap) return SS_OK;
    hipError_t e;
    if (ctx->d_cells) {
        // the old table may still be in use by enqueued work: wait for it
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        (void)hipFree(ctx->d_cells);
        ctx->d_cells = nullptr;
        ctx->cells_cap = 0;
    }
    if ((e = hipMalloc(&ctx->d_cells, (size_t)need * sizeof(float))) != hipSuccess) {
        ctx->d_cells = nullptr;
        return fail(SS_ENOMEM, "quadrature scratch (%lld bytes): %s", (long long)need * 4, hipGetErrorString(e));
    }
    ctx->cells_cap = need;
    return SS_OK;
}

ss_status check_ctx(const ss_ctx *ctx) {
    if (!ctx) return fail(SS_EINVAL, "context is NULL");
    return SS_OK;
}

}  // namespace

extern "C" {

const char *ss_last_error(void) { return g_err.c_str(); }

ss_status ss_validate_problem(const int64_t dims[3], const ss_geometry *geom) {
    if (ss_status s = check_dims(dims)) return s;
    return check_geom(geom);
}

int ss_abi_version(void) { return SS_ABI_VERSION; }

ss_status ss_query(const ss_ctx *ctx, int *degree, int *form, int *device) {
    if (ss_status s = check_ctx(ctx)) return s;
    if (degree) *degree = ctx->degree;
    if (form) *form = ctx->form;
    if (device) *device = ctx->device;
    return SS_OK;
}

ss_status ss_create(ss_ctx **out, int device, int degree, ss_form form, const void *mlp_blob, size_t blob_bytes) {
    if (!out) return fail(SS_EINVAL, "out is NULL");
    *out = nullptr;
    if (degree < 0 || degree > 3) return fail(SS_EINVAL, "degree %d outside 0..3", degree);
    if (form != SS_FORM_QUAD_FP32 && form != SS_FORM_MLP_BF16 && form != SS_FORM_QUAD_PAIR_FP32)
        return fail(SS_EINVAL, "unknown form %d", (int)form);
    if (form == SS_FORM_MLP_BF16 && degree == 0)
        return fail(SS_EUNSUPPORTED, "the network form is built for degrees 1..3");
    if (form != SS_FORM_MLP_BF16 && (mlp_blob || blob_bytes))
        return fail(SS_EINVAL, "the exact footprint forms take no weight blob");
    std::vector<unsigned char> image;
    if (form == SS_FORM_MLP_BF16) {
        if (!mlp_blob) return fail(SS_EBLOB, "the network form needs a weight blob");
        if (ss_status s = ss::mlp_blob_to_image(mlp_blob, blob_bytes, degree, image)) return s;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(SS_EINVAL, "device %d not in [0, %d)", device, ndev);
    DeviceGuard guard(device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
    ss_ctx *ctx = new (std::nothrow) ss_ctx;
    if (!ctx) return fail(SS_ENOMEM, "context allocation");
    ctx->device = device;
    ctx->degree = degree;
    ctx->form = form;
    if ((e = hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming)) != hipSuccess) {
        delete ctx;
        return hip_fail(e, "hipEventCreate");
    }
    if ((e = hipMalloc(&ctx->d_partials, sizeof(double) * ss::dot_partials_needed())) != hipSuccess) {
        ss_destroy(ctx);
        return fail(SS_ENOMEM, "reduction scratch: %s", hipGetErrorString(e));
    }
    if (!image.empty()) {
        if ((e = hipMalloc(&ctx->d_mlp, image.size())) != hipSuccess) {
            ss_destroy(ctx);
            return fail(SS_ENOMEM, "network weights: %s", hipGetErrorString(e));
        }
        if ((e = hipMemcpy(ctx->d_mlp, image.data(), image.size(), hipMemcpyHostToDevice)) != hipSuccess) {
            ss_destroy(ctx);
            return hip_fail(e, "network weight upload");
        }
    }
    *out = ctx;
    return SS_OK;
}

ss_status ss_destroy(ss_ctx *ctx) {
    if (!ctx) return SS_OK;
    DeviceGuard guard(ctx->device);
    if (ctx->geom.staged_pending) (void)hipEventSynchronize(ctx->staged);
    {
        HipUploadOps ops{nullptr, ctx->staged};
        ctx->geom.release(ops);
    }
    if (ctx->staged) (void)hipEventDestroy(ctx->staged);
    if (ctx->d_partials) (void)hipFree(ctx->d_partials);
    if (ctx->d_mlp) (void)hipFree(ctx->d_mlp);
    if (ctx->d_cells) (void)hipFree(ctx->d_cells);
    delete ctx;
    return SS_OK;
}

static ss_status run_transform(ss_ctx *ctx, bool forward, const float *in, const int64_t dims[3],
                               const ss_geometry *geom, float *out, void *hip_stream) {
    if (ss_status s = check_ctx(ctx)) return s;
    if (!in) return fail(SS_EINVAL, forward ? "d_coeffs is NULL" : "d_sino is NULL");
    if (!out) return fail(SS_EINVAL, forward ? "d_sino is NULL" : "d_coeffs is NULL");
    if (ss_status s = check_dims(dims)) return s;
    if (ss_status s = check_geom(geom)) return s;
    DeviceGuard guard(ctx->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    if (ss_status s = upload_geom(ctx, geom, st)) return s;
    ss::LaunchArgs a{};
    a.geom = ctx->geom.d_geom;
    a.vproj = reinterpret_cast<const ss::ViewProj *>(ctx->geom.d_geom + vproj_offset((size_t)geom->n_views));
    a.N[0] = (int)dims[0];
    a.N[1] = (int)dims[1];
    a.N[2] = (int)dims[2];
    a.kind = geom->kind;
    a.V = geom->n_views;
    a.R = geom->det_rows;
    a.C = geom->det_cols;
    a.mlp = ctx->d_mlp;
    hipError_t e;
    if (forward) {
        a.coeffs = in;
        a.sino = out;
        if (ctx->form == SS_FORM_QUAD_FP32) {
            if (ss_status s = ensure_cells(ctx, ss::project_quad_scratch_floats(ctx->degree, a.N))) return s;
            a.scratch = ctx->d_cells;
            a.scratch_floats = ctx->cells_cap;
        }
        e = ctx->form == SS_FORM_QUAD_FP32   ? ss::launch_project_quad(ctx->degree, a, st)
            : ctx->form == SS_FORM_MLP_BF16  ? ss::launch_project_mlp(ctx->degree, a, st)
                                             : ss::launch_project_pair(ctx->degree, a, st);
    } else {
        a.sino_in = in;
        a.coeffs_out = out;
        if (ctx->form == SS_FORM_QUAD_FP32) {
            const int64_t need = ss::backproject_quad_scratch_floats(ctx->degree, a.N, ctx->cell_limit);
            if (ss_status s = ensure_cells(ctx, need)) return s;
            a.scratch = ctx->d_cells;
            a.scratch_floats = need;  // the chunking follows the limit, not the buffer's size
        }
        e = ctx->form == SS_FORM_QUAD_FP32   ? ss::launch_backproject_quad(ctx->degree, a, st)
            : ctx->form == SS_FORM_MLP_BF16  ? ss::launch_backproject_mlp(ctx->degree, a, st)
                                             : ss::launch_backproject_pair(ctx->degree, a, st);
    }
    if (e != hipSuccess) return hip_fail(e, forward ? "project launch" : "backproject launch");
    return SS_OK;
}

ss_status ss_project(ss_ctx *ctx, const float *d_coeffs, const int64_t dims[3], const ss_geometry *geom,
                     float *d_sino, void *hip_stream) {
    return run_transform(ctx, true, d_coeffs, dims, geom, d_sino, hip_stream);
}

ss_status ss_backproject(ss_ctx *ctx, const float *d_sino, const ss_geometry *geom, const int64_t dims[3],
                         float *d_coeffs, void *hip_stream) {
    return run_transform(ctx, false, d_sino, dims, geom, d_coeffs, hip_stream);
}

ss_status ss_project_noalloc(int device, int degree, const float *d_coeffs, const int64_t dims[3],
                             const ss_geometry *geom, float *d_sino, void *hip_stream) {
    if (degree < 0 || degree > 3) return fail(SS_EINVAL, "degree %d outside 0..3", degree);
    if (!d_coeffs) return fail(SS_EINVAL, "d_coeffs is NULL");
    if (!d_sino) return fail(SS_EINVAL, "d_sino is NULL");
    if (ss_status s = check_dims(dims)) return s;
    if (ss_status s = check_geom(geom)) return s;
    const int N[3] = {(int)dims[0], (int)dims[1], (int)dims[2]};
    // view vectors first (rounded up to 256 bytes), then the padded volume
    const int64_t geom_floats = ((int64_t)geom->n_views * 12 + 63) / 64 * 64;
    const int64_t padded = ss::project_quad_scratch_floats(degree, N);
    if (geom_floats + padded > ss::STATIC_SCRATCH_FLOATS)
        return fail(SS_EINVAL, "ss_project_noalloc: %lld view floats + %lld padded coefficients exceed the %lld-float "
                    "static scratch", (long long)geom_floats, (long long)padded, (long long)ss::STATIC_SCRATCH_FLOATS);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(SS_EINVAL, "device %d not in [0, %d)", device, ndev);
    DeviceGuard guard(device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
    float *base = nullptr;
    if ((e = ss::static_scratch_address(device, &base)) != hipSuccess) return hip_fail(e, "hipGetSymbolAddress");
    hipStream_t st = (hipStream_t)hip_stream;
    if ((e = hipMemcpyAsync(base, geom->vecs, (size_t)geom->n_views * 12 * sizeof(float), hipMemcpyHostToDevice,
                            st)) != hipSuccess)
        return hip_fail(e, "geometry copy");
    ss::LaunchArgs a{};
    a.coeffs = d_coeffs;
    a.sino = d_sino;
    a.geom = base;
    a.N[0] = N[0];
    a.N[1] = N[1];
    a.N[2] = N[2];
    a.kind = geom->kind;
    a.V = geom->n_views;
    a.R = geom->det_rows;
    a.C = geom->det_cols;
    a.scratch = base + geom_floats;
    a.scratch_floats = ss::STATIC_SCRATCH_FLOATS - geom_floats;
    if ((e = ss::launch_project_quad(degree, a, st)) != hipSuccess) return hip_fail(e, "project launch");
    return SS_OK;
}

ss_status ss_set_scratch_limit(ss_ctx *ctx, size_t bytes) {
    if (ss_status s = check_ctx(ctx)) return s;
    const int64_t floats = bytes == 0 ? ss::CELL_SCRATCH_DEFAULT_FLOATS
                                      : (int64_t)std::min<size_t>(bytes / sizeof(float), (size_t)1 << 40);
    ctx->cell_limit = floats;
    if (ctx->d_cells && ctx->cells_cap > floats) {
        // release a buffer above the new limit (enqueued work may still use it)
        DeviceGuard guard(ctx->device);
        if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
        hipError_t e;
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        (void)hipFree(ctx->d_cells);
        ctx->d_cells = nullptr;
        ctx->cells_cap = 0;
    }
    return SS_OK;
}

ss_status ss_footprint(ss_ctx *ctx, const float *d_dirs, const float *d_offsets, int64_t count, float *d_out,
                       void *hip_stream) {
    if (ss_status s = check_ctx(ctx)) return s;
    if (count < 0 || count > MAX_ELEMS) return fail(SS_EINVAL, "count %lld out of range", (long long)count);
    if (count > 0 && (!d_dirs || !d_offsets || !d_out)) return fail(SS_EINVAL, "NULL buffer");
    if (count == 0) return SS_OK;
    DeviceGuard guard(ctx->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = ctx->form == SS_FORM_MLP_BF16
                       ? ss::launch_footprint_mlp(ctx->degree, ctx->d_mlp, d_dirs, d_offsets, (int)count, d_out, st)
                       : ss::launch_footprint_quad(ctx->degree, d_dirs, d_offsets, (int)count, d_out, st);
    if (e != hipSuccess) return hip_fail(e, "footprint launch");
    return SS_OK;
}

ss_status ss_dot_f64(ss_ctx *ctx, const float *d_a, const float *d_b, int64_t n, double *d_out, void *hip_stream) {
    if (ss_status s = check_ctx(ctx)) return s;
    if (n < 0) return fail(SS_EINVAL, "n < 0");
    if (!d_out || (n > 0 && (!d_a || !d_b))) return fail(SS_EINVAL, "NULL buffer");
    DeviceGuard guard(ctx->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
    hipError_t e = ss::launch_dot(d_a, d_b, n, ctx->d_partials, d_out, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "dot launch");
    return SS_OK;
}

ss_status ss_cgls_scalars(ss_ctx *ctx, const double *d_num, const double *d_den, double *d_out, void *hip_stream) {
    if (ss_status s = check_ctx(ctx)) return s;
    if (!d_num || !d_den || !d_out) return fail(SS_EINVAL, "NULL scalar");
    DeviceGuard guard(ctx->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
    hipError_t e = ss::launch_ratio(d_num, d_den, d_out, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "ratio launch");
    return SS_OK;
}

ss_status ss_axpy(ss_ctx *ctx, const double *d_alpha, int sign, const float *d_x, float *d_y, int64_t n,
                  void *hip_stream) {
    if (ss_status s = check_ctx(ctx)) return s;
    if (sign != 1 && sign != -1) return fail(SS_EINVAL, "sign must be +1 or -1");
    if (n < 0) return fail(SS_EINVAL, "n < 0");
    if (!d_alpha || (n > 0 && (!d_x || !d_y))) return fail(SS_EINVAL, "NULL buffer");
    DeviceGuard guard(ctx->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
    hipError_t e = ss::launch_axpy(d_alpha, (float)sign, d_x, d_y, n, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "axpy launch");
    return SS_OK;
}

ss_status ss_xpay(ss_ctx *ctx, const double *d_beta, const float *d_x, float *d_y, int64_t n, void *hip_stream) {
    if (ss_status s = check_ctx(ctx)) return s;
    if (n < 0) return fail(SS_EINVAL, "n < 0");
    if (!d_beta || (n > 0 && (!d_x || !d_y))) return fail(SS_EINVAL, "NULL buffer");
    DeviceGuard guard(ctx->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
    hipError_t e = ss::launch_xpay(d_beta, d_x, d_y, n, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "xpay launch");
    return SS_OK;
}

}  // extern "C"
