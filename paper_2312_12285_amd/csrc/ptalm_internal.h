// Internal declarations of the ptalm HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace ptalm {

// Every per-m segment of the step-coefficient table is padded by this many
// entries so that an l-block may run past lmax without reading out of bounds.
constexpr int kCoefPad = 64;

// Neumaier's compensated addition: sum + c carries the exact running total to
// within one rounding of the final result, whatever the order of magnitudes.
__device__ inline void neumaier_add(double &sum, double &c, double v) {
    const double t = sum + v;
    c += (fabs(sum) >= fabs(v)) ? (sum - t) + v : (v - t) + sum;
    sum = t;
}

__host__ __device__ inline int64_t tri_size(int lmax) { return (int64_t)(lmax + 1) * (lmax + 2) / 2; }

// healpy index of (l, m)
__host__ __device__ inline int64_t hp_index(int lmax, int l, int m) {
    return (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
}

// start of order m's column in healpy order: index(m, m)
__host__ __device__ inline int64_t column_start(int lmax, int m) { return hp_index(lmax, m, m); }

// start of order m's padded segment in the step-coefficient table
__host__ __device__ inline int64_t coef_segment(int lmax, int m) {
    return column_start(lmax, m) + (int64_t)m * kCoefPad;
}

__host__ __device__ inline int64_t coef_table_size(int lmax) {
    return tri_size(lmax) + (int64_t)(lmax + 1) * kCoefPad;
}

// Device tables for one lmax (built once per device, immutable afterwards).
struct Tables {
    int lmax = -1;
    double *coef = nullptr;   // step coefficients, coef_table_size(lmax)
    double *sigma = nullptr;  // output scale per (l, m), healpy order, tri_size(lmax)
    float *coef32 = nullptr;  // FP32 copy of coef for the mixed-precision kernel
};

// Work decomposition of one transform.
struct Plan {
    int points_per_lane = 0;  // KP
    int l_block = 0;          // LB
    int n_slices = 0;         // S
    int n_ranges = 0;         // R
    int64_t groups = 0;       // ceil(n / (64*KP))
    std::vector<int> range_m; // R+1 boundaries of the m ranges
};

// Arguments of the transform kernels (passed by value).
struct AlmArgs {
    const double *theta;
    const double *phi;
    const double *w;
    int64_t n;
    int lmax;
    int n_ranges;
    int n_slices;
    int64_t groups;
    const int *range_m;       // device, n_ranges+1
    const double *coef;       // device step coefficients
    const float *coef32;
    double *partial;          // device, n_slices * 2T doubles
    int64_t w_stride;         // multi-weight: distance between weight rows
    int n_weights;
    // when set, the number of points is read here on the device (n and groups
    // above are then upper bounds used only by the plan)
    const int64_t *n_dev = nullptr;
    // slices [slice_base, slice_base + slice_count) of the n_slices of the plan are
    // launched (slice_count 0: all of them); the request server runs a call this way
    // in chunks, each computing exactly the partials the whole launch computes
    int slice_base = 0;
    int slice_count = 0;
};

// One transform planned as ptalm_alm_from_points_ex would run it (same kernel
// variant, slices and ranges, tables built), for launching in chunks of point
// slices followed by the second pass.
struct SlicedCall {
    AlmArgs a;
    int precision = 0, kp = 0, lb = 0, mode = 0;
    const double *sigma = nullptr;
};

// Arguments of the multi-weight MFMA kernels.
struct MultiArgs {
    const double *theta;
    const double *phi;
    const double *w;          // device, n_weights rows of n
    float *w32;               // device scratch, FP32 copy of w
    int64_t n;
    int lmax;
    int n_weights;            // 16 or 32
    int n_slices;
    int64_t groups;           // ceil(n / kMultiGroup)
    const double *coef;       // device step coefficients
    float *partial32;         // device, [n_slices][multi_rows(lmax)][2 n_weights] floats
};

// Rows of the multi-weight partial buffer: order m's segment starts at
// column_start(m) + kMultiPad*m and holds L(m) rows plus kMultiPad rows of
// padding, so whole 32-row tiles can be read and written without bounds tests.
constexpr int kMultiPad = 32;
constexpr int kMultiGroup = 512;   // points per group = threads per workgroup
__host__ __device__ inline int64_t multi_row_start(int lmax, int m) {
    return column_start(lmax, m) + (int64_t)m * kMultiPad;
}
__host__ __device__ inline int64_t multi_rows(int lmax) {
    return tri_size(lmax) + (int64_t)(lmax + 1) * kMultiPad;
}

// --- launchers (defined in the .hip files) ----------------------------------
hipError_t build_tables(int lmax, Tables *t, hipStream_t stream);
hipError_t launch_alm_fp64(const AlmArgs &a, int kp, int lb, int mode, hipStream_t stream, bool *supported);
hipError_t launch_alm_mixed(const AlmArgs &a, int kp, int lb, int mode, hipStream_t stream, bool *supported);
hipError_t launch_alm_fp32(const AlmArgs &a, int kp, int lb, int mode, hipStream_t stream, bool *supported);
hipError_t noalloc_scratch(void **out);   // device address of the static scratch (alm_direct.hip)

// request server support (api.hip): the slice count the call would use, the
// plan itself (tables built on first use; `partial` is its scratch), one chunk
// of slices, and the second pass into alm
int sliced_slice_count(int64_t n, int lmax, int precision);
int plan_sliced(const double *theta, const double *phi, const double *w, int64_t n, int lmax, int precision,
                double *partial, SlicedCall *c);
hipError_t launch_sliced(const SlicedCall &c, int s0, int s1, hipStream_t stream);
hipError_t launch_sliced_finish(const SlicedCall &c, double *alm, hipStream_t stream);
hipError_t launch_reduce_partials(const double *partial, int n_slices, const double *sigma, int lmax,
                                  double *alm, hipStream_t stream);
hipError_t launch_cl(const double *alm1, const double *alm2, int lmax, double *cl, hipStream_t stream);
hipError_t launch_axpy(double alpha, const double *x, double *y, int64_t count, hipStream_t stream);
hipError_t launch_zero(double *p, int64_t count, hipStream_t stream);
hipError_t launch_fkp(const double *ad, const double *ar, int lmax, double *delta, double *window,
                      double *alpha_out, hipStream_t stream);

// Kernel variants compiled into the library, as (points_per_lane, l_block, mode)
// with mode = register butterfly stage (bit 0) | pipelined reduction (bit 1).
bool fp64_variant_exists(int kp, int lb, int mode);
// (points_per_lane, l_block, mode) of every compiled variant of a precision
// (0 FP64, 1 mixed, 2 FP32): writes min(count, max) entries, returns count
int list_variants(int precision, int (*out)[3], int max);
bool mixed_variant_exists(int kp, int lb, int mode);
bool fp32_variant_exists(int kp, int lb, int mode);

// mode coupling and bandpowers (coupling.hip)
int bandpower_count(int lmax, int lmin, int delta_l);
size_t bandpower_scratch_doubles(int lmax, int nb);
size_t coupling_scratch_doubles(int lmax);
// frees the lmax-only coupling tables kept per (device, lmax); the first hipFree error, else hipSuccess
hipError_t release_coupling_tables();
hipError_t launch_coupling(const double *Wl, int lmax_w, const double *shot, double *scratch, int lmax, double *M,
                           hipStream_t stream);
hipError_t launch_bandpowers(const double *cl_hat, const double *M, const double *Wl, int lmax_w, int lmax, int lmin,
                             int delta_l, int nb, int mode, double *cb, double *window, double *scratch,
                             hipStream_t stream);
size_t shot_noise_scratch_doubles();
hipError_t launch_shot_noise(const double *w, int64_t n, const double *alpha, double *out, double *partial,
                             hipStream_t stream);

// interpolated transform (spline.hip)
struct SplinePlan {
    int n_int = 0, n_pass = 0;
    int sort_chunks = 1;                // stable sort: chunks of the input (one wavefront each)
    int64_t sort_chunk = 1;             // points per chunk
    int ns_slices = 0, ns_ranges = 0;   // node sum: node slices x order ranges
    int64_t ns_groups = 0;              // node groups of 64 KP
    size_t v_doubles = 0, wn_doubles = 0, state_doubles = 0;
};
// Arguments of the node-sum kernel (passed by value).
struct NodeSumArgs {
    const double *xn, *thn;
    int n_nodes;
    int lmax;
    int n_ranges;
    int n_slices;
    int64_t groups;
    const int *range_m;       // device, n_ranges+1
    const double *coef;       // alpha table, coef_table_size(lmax)
    const double2 *wn;        // node weights (V, F, G) per (m, node)
    double *partial;          // n_slices * 4T doubles
};
SplinePlan spline_plan(int64_t n, int lmax, int n_nodes);
hipError_t launch_spline_sort(const double *theta, const double *phi, const double *w, int64_t n, double theta_cut,
                              double h, int n_nodes, const SplinePlan &p, double *xn, double *thn, unsigned *H,
                              unsigned *counts, int64_t *offsets, int64_t *n_polar, double *q, double *pth, double *pph,
                              double *pw, hipStream_t stream);
hipError_t launch_spline_transform(const SplinePlan &p, const double *q, int64_t n_spline, const int64_t *offsets,
                                   const double *xn, const double *thn, int n_nodes, int lmax, double2 *v,
                                   double2 *wn, double *state, const int *ranges, double *alm, hipStream_t stream,
                                   hipEvent_t bin_start = nullptr, hipEvent_t bin_stop = nullptr);

// Spin +-2 transform for shear: device tables per lmax, kernel arguments.
struct SpinTables {
    int lmax = -1;
    double2 *coef = nullptr;  // (alpha, beta) step pairs, coef_table_size(lmax)
    double *sigma = nullptr;  // output scale per (l, m), healpy order; 0 for l < 2
};
struct SpinArgs {
    const double *theta, *phi, *w, *g1, *g2;
    int64_t n;
    int lmax;
    int n_ranges;
    int n_slices;
    int64_t groups;           // ceil(n / (64 KP))
    const int *range_m;       // device, n_ranges+1
    const double2 *coef;
    double *partial;          // device, n_slices * 4T doubles
};
hipError_t build_spin_tables(int lmax, SpinTables *t, hipStream_t stream);
bool spin_variant_exists(int kp, int lb, bool single);
hipError_t launch_spin(const SpinArgs &a, int kp, int lb, bool single, hipStream_t stream, bool *supported);
hipError_t launch_spin_finish(const double *partial, int n_slices, const double *sigma, int lmax, double *alm_e,
                              double *alm_b, hipStream_t stream);

bool multi_nw_supported(int nw);
hipError_t launch_alm_multi(const MultiArgs &a, hipStream_t stream);
hipError_t launch_multi_finish(const MultiArgs &a, const double *sigma, double *alm, hipStream_t stream);

}  // namespace ptalm
