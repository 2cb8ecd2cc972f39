// ss_kernels.hpp -- launch interface between the C ABI (ss_abi.cpp) and the
// gfx950 kernels.
//
// Window of the slab walk.  A line with dominant axis d (|w_d| maximal)
// crosses the plane x_d = x_j of slab j at P(j).  A basis q with q_d = j can
// meet the line only where |x_d - x_j| < h, and there the transverse
// coordinate moves by at most h |r_i| (r_i = w_i / w_d, |r_i| <= 1) from
// P_i(j); so |q_i - P_i(j)| < h (1 + |r_i|) is necessary.  This per-line
// bound replaces the fixed l_inf window of the paper's neighbour search (the
// union of the windows of the <= 3 cells crossed in one slab) and, being one
// window per slab, needs no history of the two previous steps: every basis
// belongs to exactly one slab, so it is visited exactly once.  The exact
// chord test then drops the candidates the line misses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "splinesplat.h"
#include "ss_math.hpp"
#include "ss_traverse.hpp"

namespace ss {

struct LaunchArgs {
    const float *coeffs;   // forward input
    float *sino;           // forward output
    const float *sino_in;  // adjoint input
    float *coeffs_out;     // adjoint output
    const float *geom;     // device, V x 12
    const ViewProj *vproj; // device, V detector projections (FP64)
    int N[3];
    int kind, V, R, C;
    const void *mlp;       // device weights (network form)
    float *scratch;        // quadrature forward: padded coefficients; adjoint: knot-cell table
    int64_t scratch_floats;
};

// Default largest knot-cell table of the quadrature adjoint: 2^34 floats
// (64 GiB; 256^3 needs 4.45 GB, 512^3 35.6 GB); larger tables are processed
// in z-chunks of cell layers.  A context may set another limit.
constexpr int64_t CELL_SCRATCH_DEFAULT_FLOATS = (int64_t)1 << 34;
// Table size the quadrature adjoint uses for a volume of N[0] x N[1] x N[2]
// under a limit of `limit` floats (never below 4 (n+1) cell layers).
int64_t backproject_quad_scratch_floats(int degree, const int N[3], int64_t limit);
// Zero-padded copy of the coefficients the quadrature forward walks.
#define FWD_PAD(n) ((n) + 1)
int64_t project_quad_scratch_floats(int degree, const int N[3]);

hipError_t launch_project_quad(int degree, const LaunchArgs &a, hipStream_t st);

// Static scratch of the allocation-free forward (ss_project_noalloc): view
// vectors, then the zero-padded coefficients, in one file-scope device array
// of STATIC_SCRATCH_FLOATS floats per GPU.  static_scratch_address returns
// its device address on `device`, which must be the current device (looked
// up once per device, then cached).
constexpr int64_t STATIC_SCRATCH_FLOATS = (int64_t)24 << 20;  // 96 MiB
hipError_t static_scratch_address(int device, float **ptr);
hipError_t launch_backproject_quad(int degree, const LaunchArgs &a, hipStream_t st);
hipError_t launch_footprint_quad(int degree, const float *dirs, const float *offs, int count, float *out,
                                 hipStream_t st);

hipError_t launch_project_mlp(int degree, const LaunchArgs &a, hipStream_t st);
hipError_t launch_backproject_mlp(int degree, const LaunchArgs &a, hipStream_t st);
// Exact footprint per (line, basis) pair on the network form's walk and gather.
hipError_t launch_project_pair(int degree, const LaunchArgs &a, hipStream_t st);
hipError_t launch_backproject_pair(int degree, const LaunchArgs &a, hipStream_t st);
hipError_t launch_footprint_mlp(int degree, const void *mlp, const float *dirs, const float *offs, int count,
                                float *out, hipStream_t st);
// Record a thread-local error message (printf format) and return s.
ss_status fail(ss_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Validate a weight blob against the context's degree and build the device
// image of the weights (kernel layout).  Sets the thread's error message.
ss_status mlp_blob_to_image(const void *blob, size_t bytes, int degree, std::vector<unsigned char> &image);

hipError_t launch_dot(const float *a, const float *b, int64_t n, double *partials, double *out, hipStream_t st);
int dot_partials_needed();
hipError_t launch_ratio(const double *num, const double *den, double *out, hipStream_t st);
hipError_t launch_axpy(const double *alpha, float sign, const float *x, float *y, int64_t n, hipStream_t st);
hipError_t launch_xpay(const double *beta, const float *x, float *y, int64_t n, hipStream_t st);

}  // namespace ss
