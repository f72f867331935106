// FP64 direct point-to-harmonic transform: a_lm = sum_i w_i Y*_lm(theta_i, phi_i)
// (eq. alm_def, Sec. 2.2) for 0 <= m <= l <= lmax.
//
// Work decomposition.  Points are cut into groups of 64*KP (KP points per
// lane, lane-contiguous so loads coalesce); groups are cut into S contiguous
// slices; orders m are cut into R contiguous ranges of about equal work
// sum_m (lmax-m+1).  One workgroup = one wavefront = one (slice, range) item:
// it walks its slice group by group and, for every m of its range, runs the
// l-recurrence of App. A.1 for its 64*KP points in registers, accumulates the
// per-l sums in registers over an l-block of LB values, reduces them across the
// 64 lanes through LDS in a fixed order and adds them to its slice's partial
// a_lm column in global memory.  The first group of a slice stores instead of
// adding, so no clearing pass is needed.  A second kernel sums the S partials in
// slice order and applies the per-(l, m) output scale.  Every reduction order
// is fixed, so results are bitwise reproducible.
//
// Per point the kernel carries
//   Z = w s^m e^{-i m phi}  as a complex FP64 mantissa and an int exponent,
//       advanced from m to m+1 by one complex multiply with u = s e^{-i phi}
//       (angle addition) and renormalised every step;
//   (Ehat, Ohat), the split recurrence of tables.hip (one FMA per odd step,
//       one multiply + one FMA per even step);
//   q = exponent applied to Z when forming the weights W = Z 2^q (even l) and
//       V = x W (odd l).  Near the poles s^m underflows while the recurrence
//       grows: then W is 0 (ldexp underflow) and the chain keeps growing until
//       it is rescaled by a power of two, which raises q, until W re-enters the
//       FP64 range.  Contributions dropped this way are below 2^-900 |w|.
#include "ptalm_internal.h"

namespace ptalm {

namespace {

constexpr double kRescaleAbove = 0x1p+64;  // chain values are renormalised past this

__device__ inline double ldexp_d(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
__device__ inline int frexp_exp(double x) { return __builtin_amdgcn_frexp_exp(x); }

// (re, im) * 2^-e so that max(|re|, |im|) lies in [0.5, 1); exponent += e.
__device__ inline void renorm(double &re, double &im, int &exponent) {
    const double mx = fmax(fabs(re), fabs(im));
    const int e = (mx != 0.0) ? frexp_exp(mx) : 0;
    re = ldexp_d(re, -e);
    im = ldexp_d(im, -e);
    exponent += e;
}

template <int KP, int LB>
__global__ __launch_bounds__(64) void alm_fp64_kernel(AlmArgs args) {
    static_assert(LB % 2 == 0 && 64 % (2 * LB) == 0, "LB must be even and 2*LB must divide 64");
    constexpr int V = 2 * LB;            // values reduced per l-block (re, im per l)
    constexpr int P = 64 / V;            // lanes per reduced value
    constexpr int RESCALE_EVERY = (32 / LB) > 0 ? (32 / LB) : 1;  // l-blocks between chain checks

    __shared__ double red[V][64 + 1];

    const int lane = threadIdx.x;
    const int lmax = args.lmax;
    const int r = blockIdx.x % args.n_ranges;
    const int s = blockIdx.x / args.n_ranges;
    const int m_a = args.range_m[r];
    const int m_b = args.range_m[r + 1];
    const int64_t g_a = (int64_t)s * args.groups / args.n_slices;
    const int64_t g_b = (int64_t)(s + 1) * args.groups / args.n_slices;
    double *part = args.partial + (int64_t)s * 2 * tri_size(lmax);

    for (int64_t g = g_a; g < g_b; ++g) {
        const bool first = (g == g_a);
        // ---- point staging: coalesced SoA loads, FP64 trig -------------------
        double x[KP], Zr[KP], Zi[KP], ur[KP], ui[KP];
        int Ze[KP];
#pragma unroll
        for (int t = 0; t < KP; ++t) {
            const int64_t i = g * (64 * KP) + t * 64 + lane;
            double th = 1.5707963267948966, ph = 0.0, ww = 0.0;
            if (i < args.n) {
                th = args.theta[i];
                ph = args.phi[i];
                ww = args.w[i];
            }
            double st, ct, sp, cp;
            sincos(th, &st, &ct);
            sincos(ph, &sp, &cp);
            x[t] = ct;
            // u = s e^{-i phi}, normalised base for powering
            double br = st * cp, bi = -st * sp;
            int be = 0;
            renorm(br, bi, be);
            ur[t] = ldexp_d(br, be);   // keep u itself for the per-m step (|u| <= 1, no underflow)
            ui[t] = ldexp_d(bi, be);
            // Z = w * u^{m_a} by binary powering with exponent tracking
            double rr = 1.0, ri = 0.0;
            int re = 0;
            for (int k = m_a; k; k >>= 1) {
                if (k & 1) {
                    const double tr = rr * br - ri * bi;
                    const double ti = rr * bi + ri * br;
                    rr = tr;
                    ri = ti;
                    re += be;
                    renorm(rr, ri, re);
                }
                if (k > 1) {
                    const double tr = br * br - bi * bi;
                    const double ti = 2.0 * br * bi;
                    br = tr;
                    bi = ti;
                    be *= 2;
                    renorm(br, bi, be);
                }
            }
            Zr[t] = rr * ww;
            Zi[t] = ri * ww;
            Ze[t] = re;
            renorm(Zr[t], Zi[t], Ze[t]);
        }

        for (int m = m_a; m < m_b; ++m) {
            const int L = lmax - m + 1;  // number of l values of this order
            const double *cm = args.coef + coef_segment(lmax, m);
            double *pm = part + 2 * column_start(lmax, m);

            double E[KP], O[KP], y[KP], Wr[KP], Wi[KP], Vr[KP], Vi[KP];
            int q[KP];
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                E[t] = -1.0;
                O[t] = 0.0;
                y[t] = x[t] * x[t];
                q[t] = Ze[t];
                Wr[t] = ldexp_d(Zr[t], q[t]);
                Wi[t] = ldexp_d(Zi[t], q[t]);
                Vr[t] = Wr[t] * x[t];
                Vi[t] = Wi[t] * x[t];
            }

            int blk = 0;
            for (int jb = 0; jb < L; jb += LB, ++blk) {
                double c[LB];
#pragma unroll
                for (int k = 0; k < LB; ++k) c[k] = cm[jb + k];
                double ar[LB], ai[LB];
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    ar[k] = 0.0;
                    ai[k] = 0.0;
                }
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    if ((k & 1) == 0) {
#pragma unroll
                        for (int t = 0; t < KP; ++t) {
                            E[t] = fma(c[k] * y[t], O[t], -E[t]);
                            ar[k] = fma(E[t], Wr[t], ar[k]);
                            ai[k] = fma(E[t], Wi[t], ai[k]);
                        }
                    } else {
#pragma unroll
                        for (int t = 0; t < KP; ++t) {
                            O[t] = fma(c[k], E[t], -O[t]);
                            ar[k] = fma(O[t], Vr[t], ar[k]);
                            ai[k] = fma(O[t], Vi[t], ai[k]);
                        }
                    }
                }
                // ---- wave reduction of the l-block through LDS (fixed order) ----
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    red[2 * k][lane] = ar[k];
                    red[2 * k + 1][lane] = ai[k];
                }
                __syncthreads();
                const int v = lane / P;
                const int h = lane % P;
                double sum = 0.0;
#pragma unroll
                for (int k = 0; k < 64 / P; ++k) sum += red[v][h + k * P];
#pragma unroll
                for (int off = 1; off < P; off <<= 1) sum += __shfl_xor(sum, off, 64);
                if (h == 0 && jb + (v >> 1) < L) {
                    double *dst = pm + 2 * jb + v;
                    *dst = first ? sum : *dst + sum;
                }
                __syncthreads();

                // ---- keep the chain inside the FP64 range ----------------------
                if ((blk % RESCALE_EVERY) == RESCALE_EVERY - 1) {
                    bool big = false;
#pragma unroll
                    for (int t = 0; t < KP; ++t) big |= fmax(fabs(E[t]), fabs(O[t])) > kRescaleAbove;
                    if (__any(big)) {
#pragma unroll
                        for (int t = 0; t < KP; ++t) {
                            const double mx = fmax(fabs(E[t]), fabs(O[t]));
                            const int e = (mx > kRescaleAbove) ? frexp_exp(mx) : 0;
                            E[t] = ldexp_d(E[t], -e);
                            O[t] = ldexp_d(O[t], -e);
                            q[t] += e;
                            Wr[t] = ldexp_d(Zr[t], q[t]);
                            Wi[t] = ldexp_d(Zi[t], q[t]);
                            Vr[t] = Wr[t] * x[t];
                            Vi[t] = Wi[t] * x[t];
                        }
                    }
                }
            }
            // ---- next order: Z <- Z u (angle addition), renormalise -------------
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                const double tr = Zr[t] * ur[t] - Zi[t] * ui[t];
                const double ti = Zr[t] * ui[t] + Zi[t] * ur[t];
                Zr[t] = tr;
                Zi[t] = ti;
                renorm(Zr[t], Zi[t], Ze[t]);
            }
        }
    }
}

// Second pass: a_lm = sigma_lm * sum_{s<S} partial_s[l, m], slices in order.
__global__ void reduce_partials_kernel(const double *__restrict__ partial, int n_slices,
                                       const double *__restrict__ sigma, int64_t T, double *__restrict__ alm) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < T; k += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int s = 0; s < n_slices; ++s) {
            const double2 v = reinterpret_cast<const double2 *>(partial + (int64_t)s * 2 * T)[k];
            re += v.x;
            im += v.y;
        }
        const double sg = sigma[k];
        reinterpret_cast<double2 *>(alm)[k] = make_double2(sg * re, sg * im);
    }
}

template <int KP, int LB>
hipError_t launch_one(const AlmArgs &a, hipStream_t stream) {
    const int blocks = a.n_ranges * a.n_slices;
    hipLaunchKernelGGL((alm_fp64_kernel<KP, LB>), dim3(blocks), dim3(64), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

#define PTALM_FP64_VARIANTS(X) X(4, 8) X(6, 8) X(8, 8) X(10, 8) X(12, 8) X(8, 16) X(8, 32) X(16, 8)

bool fp64_variant_exists(int kp, int lb) {
#define X(K, L) if (kp == K && lb == L) return true;
    PTALM_FP64_VARIANTS(X)
#undef X
    return false;
}

hipError_t launch_alm_fp64(const AlmArgs &a, int kp, int lb, hipStream_t stream, bool *supported) {
    *supported = true;
#define X(K, L) if (kp == K && lb == L) return launch_one<K, L>(a, stream);
    PTALM_FP64_VARIANTS(X)
#undef X
    *supported = false;
    return hipSuccess;
}

hipError_t launch_reduce_partials(const double *partial, int n_slices, const double *sigma, int lmax,
                                  double *alm, hipStream_t stream) {
    const int64_t T = tri_size(lmax);
    const int threads = 256;
    int64_t blocks = (T + threads - 1) / threads;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, partial, n_slices,
                       sigma, T, alm);
    return hipGetLastError();
}

}  // namespace ptalm
