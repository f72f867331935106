// Spectra and field combinations on a_lm (Sec. 2.1, Sec. 2.3).
#include "ptalm_internal.h"

namespace ptalm {

namespace {

// One wavefront per l: C_l = (2l+1)^-1 [ f(a_l0) + 2 sum_{m=1..l} f(a_lm) ] with
// f = |a|^2 (auto, eq. pseudoCl) or Re(a conj(b)) (cross).  Lane k sums
// m = k, k+64, ... in order; lanes are combined by a fixed butterfly, so the
// result is deterministic.
__global__ __launch_bounds__(64) void cl_kernel(const double *__restrict__ a, const double *__restrict__ b,
                                                int lmax, double *__restrict__ cl) {
    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    const double2 *A = reinterpret_cast<const double2 *>(a);
    const double2 *B = reinterpret_cast<const double2 *>(b ? b : a);
    double s = 0.0;
    for (int m = lane; m <= l; m += 64) {
        const int64_t k = hp_index(lmax, l, m);
        const double2 x = A[k], y = B[k];
        const double v = x.x * y.x + x.y * y.y;
        s += (m == 0) ? v : 2.0 * v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) cl[l] = s / (2.0 * l + 1.0);
}

// p[0, count) = 0 (a kernel rather than a memset, so that a captured graph holds no memset node)
__global__ void zero_kernel(double *__restrict__ p, int64_t count) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

__global__ void axpy_kernel(double alpha, const double *__restrict__ x, double *__restrict__ y, int64_t count) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
        y[k] = fma(alpha, x[k], y[k]);
}

// alpha = a_00(data) / a_00(randoms); delta = a_d - alpha a_r; window = alpha a_r.
__global__ void fkp_kernel(const double *__restrict__ ad, const double *__restrict__ ar, int64_t count,
                           double *__restrict__ delta, double *__restrict__ window, double *__restrict__ alpha_out) {
    const double alpha = ad[0] / ar[0];
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (first == 0 && alpha_out) *alpha_out = alpha;
    for (int64_t k = first; k < count; k += (int64_t)gridDim.x * blockDim.x) {
        const double wr = alpha * ar[k];
        if (delta) delta[k] = ad[k] - wr;
        if (window) window[k] = wr;
    }
}

unsigned grid_for(int64_t count, int threads) {
    int64_t blocks = (count + threads - 1) / threads;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    return (unsigned)blocks;
}

}  // namespace

hipError_t launch_cl(const double *alm1, const double *alm2, int lmax, double *cl, hipStream_t stream) {
    hipLaunchKernelGGL(cl_kernel, dim3(lmax + 1), dim3(64), 0, stream, alm1, alm2, lmax, cl);
    return hipGetLastError();
}

hipError_t launch_axpy(double alpha, const double *x, double *y, int64_t count, hipStream_t stream) {
    hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(count, 256)), dim3(256), 0, stream, alpha, x, y, count);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t count, hipStream_t stream) {
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(count, 256)), dim3(256), 0, stream, p, count);
    return hipGetLastError();
}

hipError_t launch_fkp(const double *ad, const double *ar, int lmax, double *delta, double *window,
                      double *alpha_out, hipStream_t stream) {
    const int64_t count = 2 * tri_size(lmax);
    hipLaunchKernelGGL(fkp_kernel, dim3(grid_for(count, 256)), dim3(256), 0, stream, ad, ar, count, delta, window,
                       alpha_out);
    return hipGetLastError();
}

}  // namespace ptalm
