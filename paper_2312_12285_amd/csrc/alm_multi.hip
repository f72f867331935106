// Multi-weight transform on the matrix cores: NW weight vectors share one
// position set, a^(v)_lm = sum_i w_v[i] Y*_lm(theta_i, phi_i) (eq. alm_def for
// each v).  For a fixed order m the sum over points is a dense contraction
//     D[l][c] = sum_i A[l][i] B[i][c],
//     A[l][i] = Pbar_l^m(x_i) / (s_i^m e_j)       (the scaled recurrence value),
//     B[i][2v + part] = w_v[i] * (cos, -sin)(m phi_i) * s_i^m   (as a normalised
//                       mantissa; its exponent is folded into A),
// with M = l, K = points, N = 2 NW columns, which maps onto MFMA.  Operands are
// split into bf16 hi + lo parts and three products (hi.hi + hi.lo + lo.hi) are
// accumulated in FP32 on v_mfma_f32_16x16x32_bf16; the neglected lo.lo term and
// the residual of the two-term split leave ~2^-16 relative error per product.
//
// Work decomposition.  One workgroup (4 wavefronts, 256 threads) per (slice, m)
// item, dispatched in increasing m (largest work first).  It streams its slice
// in groups of 256 points, one point per thread:
//   1. each thread computes its point's x, s^m e^{-i m phi} (FP64, exponent
//      tracked) and writes its row of B (2 NW columns, bf16 hi/lo) to LDS;
//      each wavefront then keeps its B fragments in registers for all l;
//   2. per tile of 32 l: each thread advances the FP64 split recurrence of
//      tables.hip 32 steps and writes A (bf16 hi/lo) for its point to LDS;
//      wavefront w multiplies M-tile (w & 1) by its half of the N-tiles over the
//      256 points (8 K-steps x 3 products per D tile) and adds the FP32 D tile
//      into its slice's FP32 partial (the first group stores).
// A final pass sums the slices in FP64 in fixed order and applies the output
// scale sigma_lm.  Every order is fixed, so results are reproducible.
#include "ptalm_internal.h"

namespace ptalm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_bits;

template <typename T>
using const_ptr = const T __attribute__((address_space(4))) *;

constexpr int kG = 256;          // points per group = threads per workgroup
constexpr int kLT = 32;          // l values per tile
constexpr int kRow = kG + 8;     // padded LDS row (bf16 elements): rows land on different banks
constexpr double kChainAbove = 0x1p+64;

__device__ inline double ldexp_d(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
__device__ inline int frexp_exp_d(double x) { return __builtin_amdgcn_frexp_exp(x); }

__device__ inline void renorm(double &re, double &im, int &exponent) {
    const double mx = fmax(fabs(re), fabs(im));
    const int e = (mx != 0.0) ? frexp_exp_d(mx) : 0;
    re = ldexp_d(re, -e);
    im = ldexp_d(im, -e);
    exponent += e;
}

// f = hi + lo + O(2^-16 |f|), both rounded to nearest even (v_cvt_pk_bf16_f32)
__device__ inline void split_bf16(float f, bf16_bits &hi, bf16_bits &lo) {
    const __bf16 h = (__bf16)f;
    const __bf16 l = (__bf16)(f - (float)h);
    hi = __builtin_bit_cast(bf16_bits, h);
    lo = __builtin_bit_cast(bf16_bits, l);
}

__device__ inline bf16x8 load_frag(const bf16_bits *p) {
    // 8 consecutive bf16 (16 bytes, 16-byte aligned)
    const uint4 u = *reinterpret_cast<const uint4 *>(p);
    bf16x8 r;
    __builtin_memcpy(&r, &u, sizeof(r));
    return r;
}

template <int NW>
__global__ __launch_bounds__(256) void alm_multi_kernel(MultiArgs a) {
    constexpr int NC = 2 * NW;          // columns of B (re, im per weight vector)
    constexpr int NT = NC / 16;         // 16-column N-tiles
    constexpr int NTW = NT / 2;         // N-tiles per wavefront (two wavefronts per M-tile)
    static_assert(NW % 16 == 0 && NW <= 32, "NW must be 16 or 32");

    __shared__ __attribute__((aligned(16))) bf16_bits Bh[NC * kRow];
    __shared__ __attribute__((aligned(16))) bf16_bits Bl[NC * kRow];
    __shared__ __attribute__((aligned(16))) bf16_bits Ah[2][kLT * kRow];   // double-buffered A tile
    __shared__ __attribute__((aligned(16))) bf16_bits Al[2][kLT * kRow];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int lmax = a.lmax;
    const int s = blockIdx.x % a.n_slices;
    const int m = __builtin_amdgcn_readfirstlane(blockIdx.x / a.n_slices);
    const int L = lmax - m + 1;
    const int64_t T = tri_size(lmax);
    const int64_t g_a = (int64_t)s * a.groups / a.n_slices;
    const int64_t g_b = (int64_t)(s + 1) * a.groups / a.n_slices;
    const const_ptr<double> cm = (const_ptr<double>)a.coef + coef_segment(lmax, m);
    float *part = a.partial32 + (int64_t)s * NW * 2 * T;
    const int64_t col0 = column_start(lmax, m);

    const int mt = wave & 1;             // M-tile of this wavefront
    const int nt0 = (wave >> 1) * NTW;   // first N-tile of this wavefront
    const int frow = lane & 15;          // fragment row / column within a 16-tile
    const int fk = 8 * (lane >> 4);      // fragment k offset within a 32-step

    for (int64_t g = g_a; g < g_b; ++g) {
        const bool first = (g == g_a);
        // ---- 1. point data and this point's row of B ------------------------
        const int64_t i = g * kG + tid;
        double th = 1.5707963267948966, ph = 0.0;
        const bool valid = i < a.n;
        if (valid) {
            th = a.theta[i];
            ph = a.phi[i];
        }
        double st, ct, sp, cp;
        sincos(th, &st, &ct);
        sincos(ph, &sp, &cp);
        const double x = ct, y = ct * ct;
        // Z = (s e^{-i phi})^m, mantissa + exponent, by binary powering
        double br = st * cp, bi = -st * sp;
        int be = 0;
        renorm(br, bi, be);
        double zr = 1.0, zi = 0.0;
        int ze = 0;
        for (int k = m; k; k >>= 1) {
            if (k & 1) {
                const double tr = zr * br - zi * bi, ti = zr * bi + zi * br;
                zr = tr;
                zi = ti;
                ze += be;
                renorm(zr, zi, ze);
            }
            if (k > 1) {
                const double tr = br * br - bi * bi, ti = 2.0 * br * bi;
                br = tr;
                bi = ti;
                be *= 2;
                renorm(br, bi, be);
            }
        }
#pragma unroll 4
        for (int v = 0; v < NW; ++v) {
            const double wv = valid ? (double)a.w32[(int64_t)v * a.n + i] : 0.0;
            bf16_bits h, l;
            split_bf16((float)(wv * zr), h, l);
            Bh[(2 * v) * kRow + tid] = h;
            Bl[(2 * v) * kRow + tid] = l;
            split_bf16((float)(wv * zi), h, l);
            Bh[(2 * v + 1) * kRow + tid] = h;
            Bl[(2 * v + 1) * kRow + tid] = l;
        }
        __syncthreads();
        // B fragments of this wavefront, kept for every l-tile of this group
        bf16x8 bh[NTW][kG / 32], bl[NTW][kG / 32];
#pragma unroll
        for (int n = 0; n < NTW; ++n)
#pragma unroll
            for (int ks = 0; ks < kG / 32; ++ks) {
                const int off = ((nt0 + n) * 16 + frow) * kRow + ks * 32 + fk;
                bh[n][ks] = load_frag(Bh + off);
                bl[n][ks] = load_frag(Bl + off);
            }

        // ---- 2. l-tiles, software pipelined: the MFMAs of tile t read one A
        // buffer while the recurrence writes tile t+1 into the other ----------
        double E = -1.0, O = 0.0;
        // exponent turning the chain into A; a point exactly at a pole has
        // s^m = 0 for m > 0 and contributes nothing (its chain is not bounded by
        // a physical value there, so it must not reach A)
        int q = (zr == 0.0 && zi == 0.0) ? -100000 : ze;
        // A values of 32 steps starting at jb into buffer b (entries past lmax-m
        // read the zero padding of the coefficient table and are never flushed)
        auto recur_tile = [&](int jb, int b) {
#pragma unroll
            for (int k = 0; k < kLT; ++k) {
                const double c = cm[jb + k];
                double val;
                if ((k & 1) == 0) {
                    E = fma(c * y, O, -E);
                    val = E;
                } else {
                    O = fma(c, E, -O);
                    val = O * x;
                }
                bf16_bits h, l;
                split_bf16((float)ldexp_d(val, q), h, l);
                Ah[b][k * kRow + tid] = h;
                Al[b][k * kRow + tid] = l;
            }
        };
        recur_tile(0, 0);
        __syncthreads();
        const int ntiles = (L + kLT - 1) / kLT;
        for (int t = 0; t < ntiles; ++t) {
            const int jb = t * kLT;
            const int b = t & 1;
            // previous partials of this tile, fetched before the work that hides their latency
            float prev[NTW][4];
#pragma unroll
            for (int n = 0; n < NTW; ++n) {
                const int col = (nt0 + n) * 16 + frow;
                const float *pc = part + (int64_t)(col >> 1) * 2 * T + (col & 1);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = jb + mt * 16 + 4 * (lane >> 4) + r;
                    prev[n][r] = (!first && j < L) ? pc[2 * (col0 + j)] : 0.f;
                }
            }
            f32x4 d[NTW];
#pragma unroll
            for (int n = 0; n < NTW; ++n) d[n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < kG / 32; ++ks) {
                const int off = (mt * 16 + frow) * kRow + ks * 32 + fk;
                const bf16x8 ah = load_frag(Ah[b] + off);
                const bf16x8 al = load_frag(Al[b] + off);
#pragma unroll
                for (int n = 0; n < NTW; ++n) {
                    d[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[n][ks], d[n], 0, 0, 0);
                    d[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[n][ks], d[n], 0, 0, 0);
                    d[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[n][ks], d[n], 0, 0, 0);
                }
            }
            recur_tile(jb + kLT, b ^ 1);
            // D[row][col]: row = 4*(lane/16) + r, col = lane % 16 (checked layout)
#pragma unroll
            for (int n = 0; n < NTW; ++n) {
                const int col = (nt0 + n) * 16 + frow;
                float *pc = part + (int64_t)(col >> 1) * 2 * T + (col & 1);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = jb + mt * 16 + 4 * (lane >> 4) + r;
                    if (j < L) pc[2 * (col0 + j)] = prev[n][r] + d[n][r];
                }
            }
            // keep the chain inside the FP64 range (growth < 2^255 per 64 steps)
            if ((t & 1) == 1) {
                const double mx = fmax(fabs(E), fabs(O));
                if (mx > kChainAbove) {
                    const int e = frexp_exp_d(mx);
                    E = ldexp_d(E, -e);
                    O = ldexp_d(O, -e);
                    q += e;
                }
            }
            __syncthreads();
        }
    }
}

// out[v][k] = sigma_k * sum_s partial[s][v][k] (FP64 sum in slice order)
__global__ void multi_finish_kernel(const float *__restrict__ partial, int n_slices, int nw,
                                    const double *__restrict__ sigma, int64_t T, double *__restrict__ alm) {
    const int64_t total = (int64_t)nw * T;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e % T;
        double re = 0.0, im = 0.0;
        for (int s = 0; s < n_slices; ++s) {
            const float2 v = reinterpret_cast<const float2 *>(partial + (int64_t)s * nw * 2 * T)[e];
            re += (double)v.x;
            im += (double)v.y;
        }
        const double sg = sigma[k];
        reinterpret_cast<double2 *>(alm)[e] = make_double2(sg * re, sg * im);
    }
}

// weights FP64 -> FP32 copy (the B operand is formed in FP32 before its split)
__global__ void weights_to_f32_kernel(const double *__restrict__ w, int64_t count, float *__restrict__ w32) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
        w32[e] = (float)w[e];
}

unsigned grid_for(int64_t count, int threads) {
    int64_t b = (count + threads - 1) / threads;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

bool multi_nw_supported(int nw) { return nw == 16 || nw == 32; }

hipError_t launch_alm_multi(const MultiArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL(weights_to_f32_kernel, dim3(grid_for((int64_t)a.n_weights * a.n, 256)), dim3(256), 0, stream,
                       a.w, (int64_t)a.n_weights * a.n, a.w32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int blocks = (a.lmax + 1) * a.n_slices;
    if (a.n_weights == 32)
        hipLaunchKernelGGL(alm_multi_kernel<32>, dim3(blocks), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(alm_multi_kernel<16>, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_multi_finish(const MultiArgs &a, const double *sigma, double *alm, hipStream_t stream) {
    const int64_t T = tri_size(a.lmax);
    hipLaunchKernelGGL(multi_finish_kernel, dim3(grid_for((int64_t)a.n_weights * T, 256)), dim3(256), 0, stream,
                       a.partial32, a.n_slices, a.n_weights, sigma, T, alm);
    return hipGetLastError();
}

}  // namespace ptalm
