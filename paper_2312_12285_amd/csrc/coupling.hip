// Mode coupling and bandpowers (Sec. 2.1 eq. chat, eq. mode_coupling; App. C).
//
// M[l][l'] = (2l'+1)/(4 pi) sum_lambda (2 lambda + 1) (l l' lambda; 0 0 0)^2 W_lambda.
// One thread per (l, l').  Only squares of 3j symbols enter, so the kernel
// carries g = (l l' lambda; 000)^2 and never takes a square root:
//   * start at the stretched triangle lambda = |l - l'|: with a = max, b = min,
//     (a, b, a - b; 000)^2 = 1/(2a+1) * prod_{k<b} (2k+1)(a-k) / ((k+1)(2a-2k-1)),
//     the paper's recurrence of App. C (l2 -> l2+1, l3 -> l3-1 at fixed l1 and L)
//     run outward from its terminal case (a, 0, a) = (-1)^a / sqrt(2a+1);
//   * step lambda -> lambda + 2 with the ratio of consecutive symbols at fixed
//     (l, l'), obtained from the same closed form,
//     g(lambda+2)/g(lambda) = (L-2l+1)(L-2l'+1)(L+2)(L-2 lambda)
//                            / ((L-2l+2)(L-2l'+2)(L+3)(L-2 lambda-1)),  L = l+l'+lambda.
// Every factor is positive, so the sums carry no cancellation.
//
// Bandpowers: theta_b^l = 1/delta_l on complete bins [lmin + b delta_l, lmin + (b+1) delta_l).
// Mode-decoupled (eq. mode_coupling): C~ = Mbb^-1 theta C^ with Mbb = theta M chi, and the
// window cal M = Mbb^-1 theta M (eq. expectation_value), by Gauss-Jordan elimination with
// partial pivoting in one workgroup.  Normalised: C~' = N theta C^, cal M' = N theta M,
// 1/N = sum_l (2l+1) W_l / (4 pi).
#include "ptalm_internal.h"

namespace ptalm {

namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;

__global__ __launch_bounds__(256) void coupling_kernel(const double *__restrict__ Wl, int lmax_w, int lmax,
                                                      double *__restrict__ M) {
    const int64_t n1 = lmax + 1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n1 * n1) return;
    const int l = (int)(idx / n1), lp = (int)(idx % n1);
    const int a = l > lp ? l : lp, b = l > lp ? lp : l;
    const int lam0 = a - b;
    double s = 0.0;
    if (lam0 <= lmax_w) {
        double g = 1.0 / (2.0 * a + 1.0);
        for (int k = 0; k < b; ++k)
            g *= ((2.0 * k + 1.0) * (double)(a - k)) / ((k + 1.0) * (2.0 * (a - k) - 1.0));
        const int lam_hi = (a + b) < lmax_w ? (a + b) : lmax_w;
        for (int lam = lam0; lam <= lam_hi; lam += 2) {
            s = fma((2.0 * lam + 1.0) * g, Wl[lam], s);
            const double L = (double)(l + lp + lam);
            g *= ((L - 2.0 * l + 1.0) * (L - 2.0 * lp + 1.0) * (L + 2.0) * (L - 2.0 * lam)) /
                 ((L - 2.0 * l + 2.0) * (L - 2.0 * lp + 2.0) * (L + 3.0) * (L - 2.0 * lam - 1.0));
        }
    }
    M[idx] = (2.0 * lp + 1.0) * kInv4Pi * s;
}

// rows[b][c] = (1/delta_l) sum_{l in b} src[l][c] for c < ncols (src row-major, ld = ncols)
__global__ void bin_rows_kernel(const double *__restrict__ src, int ncols, int lmin, int delta_l, int nb,
                                double *__restrict__ dst, int ld_dst) {
    const int64_t total = (int64_t)nb * ncols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / ncols), c = (int)(e % ncols);
        const int l0 = lmin + b * delta_l;
        double s = 0.0;
        for (int k = 0; k < delta_l; ++k) s += src[(int64_t)(l0 + k) * ncols + c];
        dst[(int64_t)b * ld_dst + c] = s / delta_l;
    }
}

// Augmented system for the decoupling, row b:
//   [ Mbb[b][0..nb) | C^_b | (theta M)[b][0..lmax] ]
// from R = theta M (nb x (lmax+1)) and C^ (lmax+1).
__global__ void build_system_kernel(const double *__restrict__ R, const double *__restrict__ cl_hat, int lmax,
                                    int lmin, int delta_l, int nb, double *__restrict__ A, int ld) {
    const int n1 = lmax + 1;
    const int64_t total = (int64_t)nb * ld;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / ld), c = (int)(e % ld);
        double v;
        if (c < nb) {                                   // Mbb[b][c] = sum_{l' in c} R[b][l']
            const int l0 = lmin + c * delta_l;
            double s = 0.0;
            for (int k = 0; k < delta_l; ++k) s += R[(int64_t)b * n1 + l0 + k];
            v = s;
        } else if (c == nb) {                           // C^_b
            const int l0 = lmin + b * delta_l;
            double s = 0.0;
            for (int k = 0; k < delta_l; ++k) s += cl_hat[l0 + k];
            v = s / delta_l;
        } else {
            v = R[(int64_t)b * n1 + (c - nb - 1)];
        }
        A[e] = v;
    }
}

// Gauss-Jordan elimination with partial pivoting of the nb x nb block of the
// augmented matrix A (nb rows, ld columns) in one workgroup of 1024 threads;
// afterwards columns nb.. hold Mbb^-1 applied to the right-hand sides.
__global__ __launch_bounds__(1024) void gauss_jordan_kernel(double *__restrict__ A, int nb, int ld) {
    __shared__ double red_v[1024];
    __shared__ int red_i[1024];
    __shared__ double pivot_col[1024];
    const int tid = threadIdx.x;
    for (int k = 0; k < nb; ++k) {
        // pivot: largest |A[i][k]| for i >= k, lowest index on ties
        double best = -1.0;
        int bi = k;
        for (int i = k + tid; i < nb; i += blockDim.x) {
            const double v = fabs(A[(int64_t)i * ld + k]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        red_v[tid] = best;
        red_i[tid] = bi;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (tid < w) {
                const double o = red_v[tid + w];
                const int oi = red_i[tid + w];
                if (o > red_v[tid] || (o == red_v[tid] && oi < red_i[tid])) {
                    red_v[tid] = o;
                    red_i[tid] = oi;
                }
            }
            __syncthreads();
        }
        const int p = red_i[0];
        // swap rows k and p
        if (p != k)
            for (int c = tid; c < ld; c += blockDim.x) {
                const double t = A[(int64_t)k * ld + c];
                A[(int64_t)k * ld + c] = A[(int64_t)p * ld + c];
                A[(int64_t)p * ld + c] = t;
            }
        __syncthreads();
        // scale the pivot row
        const double inv = 1.0 / A[(int64_t)k * ld + k];
        for (int c = tid; c < ld; c += blockDim.x) A[(int64_t)k * ld + c] *= inv;
        __syncthreads();
        // column k of every row (read once, before the rows change)
        for (int i = tid; i < nb; i += blockDim.x) pivot_col[i] = A[(int64_t)i * ld + k];
        __syncthreads();
        // eliminate column k from every other row
        const int64_t cells = (int64_t)nb * ld;
        for (int64_t e = tid; e < cells; e += blockDim.x) {
            const int i = (int)(e / ld), c = (int)(e % ld);
            if (i != k) A[e] = fma(-pivot_col[i], A[(int64_t)k * ld + c], A[e]);
        }
        __syncthreads();
    }
}

// out[b] = A[b][col0], window[b][c] = A[b][col0 + 1 + c]
__global__ void extract_kernel(const double *__restrict__ A, int nb, int ld, int col0, int n1,
                               double *__restrict__ cb, double *__restrict__ window) {
    const int64_t total = (int64_t)nb * (n1 + 1);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / (n1 + 1)), c = (int)(e % (n1 + 1));
        const double v = A[(int64_t)b * ld + col0 + c];
        if (c == 0) cb[b] = v;
        else if (window) window[(int64_t)b * n1 + c - 1] = v;
    }
}

// Normalised convention: N = 1 / sum_l (2l+1) W_l / (4 pi) (one workgroup, fixed-order
// tree), then cb[b] = N (theta C^)_b and window = N theta M.
__global__ __launch_bounds__(1024) void normalise_kernel(const double *__restrict__ Wl, int lmax_w,
                                                         const double *__restrict__ R, const double *__restrict__ cl_hat,
                                                         int lmax, int lmin, int delta_l, int nb,
                                                         double *__restrict__ cb, double *__restrict__ window) {
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int l = tid; l <= lmax_w; l += blockDim.x) s += (2.0 * l + 1.0) * Wl[l];
    red[tid] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double N = 1.0 / (red[0] * kInv4Pi);
    const int n1 = lmax + 1;
    for (int b = tid; b < nb; b += blockDim.x) {
        const int l0 = lmin + b * delta_l;
        double c = 0.0;
        for (int k = 0; k < delta_l; ++k) c += cl_hat[l0 + k];
        cb[b] = N * c / delta_l;
    }
    if (window)
        for (int64_t e = tid; e < (int64_t)nb * n1; e += blockDim.x) window[e] = N * R[e];
}

// out = scale^2 sum_i w_i^2 / (4 pi), scale = *alpha or 1 (one workgroup, fixed order)
__global__ __launch_bounds__(1024) void shot_noise_kernel(const double *__restrict__ w, int64_t n,
                                                          const double *__restrict__ alpha, double *__restrict__ out) {
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int64_t i = tid; i < n; i += blockDim.x) s = fma(w[i], w[i], s);
    red[tid] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if (tid < k) red[tid] += red[tid + k];
        __syncthreads();
    }
    if (tid == 0) {
        const double a = alpha ? *alpha : 1.0;
        out[0] = a * a * red[0] * kInv4Pi;
    }
}

// W_l - shot for l <= lmax_w (into dst)
__global__ void subtract_kernel(const double *__restrict__ src, int count, const double *__restrict__ shot,
                                double *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = src[i] - shot[0];
}

unsigned blocks_for(int64_t count, int threads) {
    int64_t b = (count + threads - 1) / threads;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

int bandpower_count(int lmax, int lmin, int delta_l) {
    if (lmax < 0 || lmin < 0 || delta_l < 1 || lmin > lmax) return 0;
    return (lmax + 1 - lmin) / delta_l;
}

hipError_t launch_coupling(const double *Wl, int lmax_w, const double *shot, double *wtmp, int lmax, double *M,
                           hipStream_t stream) {
    const double *W = Wl;
    if (shot) {
        hipLaunchKernelGGL(subtract_kernel, dim3((lmax_w + 256) / 256), dim3(256), 0, stream, Wl, lmax_w + 1, shot, wtmp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        W = wtmp;
    }
    const int64_t cells = (int64_t)(lmax + 1) * (lmax + 1);
    hipLaunchKernelGGL(coupling_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, stream, W, lmax_w, lmax, M);
    return hipGetLastError();
}

size_t bandpower_scratch_doubles(int lmax, int nb) {
    const size_t n1 = (size_t)lmax + 1;
    const size_t ld = (size_t)nb + 1 + n1;
    return (size_t)nb * n1 + (size_t)nb * ld;   // R = theta M, then the augmented system
}

hipError_t launch_bandpowers(const double *cl_hat, const double *M, const double *Wl, int lmax_w, int lmax, int lmin,
                             int delta_l, int nb, int mode, double *cb, double *window, double *scratch,
                             hipStream_t stream) {
    const int n1 = lmax + 1;
    double *R = scratch;
    hipLaunchKernelGGL(bin_rows_kernel, dim3(blocks_for((int64_t)nb * n1, 256)), dim3(256), 0, stream, M, n1, lmin,
                       delta_l, nb, R, n1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (mode == 1) {
        hipLaunchKernelGGL(normalise_kernel, dim3(1), dim3(1024), 0, stream, Wl, lmax_w, R, cl_hat, lmax, lmin, delta_l,
                           nb, cb, window);
        return hipGetLastError();
    }
    const int ld = nb + 1 + n1;
    double *A = scratch + (size_t)nb * n1;
    hipLaunchKernelGGL(build_system_kernel, dim3(blocks_for((int64_t)nb * ld, 256)), dim3(256), 0, stream, R, cl_hat,
                       lmax, lmin, delta_l, nb, A, ld);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(gauss_jordan_kernel, dim3(1), dim3(1024), 0, stream, A, nb, ld);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(extract_kernel, dim3(blocks_for((int64_t)nb * (n1 + 1), 256)), dim3(256), 0, stream, A, nb, ld,
                       nb, n1, cb, window);
    return hipGetLastError();
}

hipError_t launch_shot_noise(const double *w, int64_t n, const double *alpha, double *out, hipStream_t stream) {
    hipLaunchKernelGGL(shot_noise_kernel, dim3(1), dim3(1024), 0, stream, w, n, alpha, out);
    return hipGetLastError();
}

}  // namespace ptalm
