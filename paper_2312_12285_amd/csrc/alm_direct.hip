// Direct point-to-harmonic transform: a_lm = sum_i w_i Y*_lm(theta_i, phi_i)
// (eq. alm_def, Sec. 2.2) for 0 <= m <= l <= lmax.
//
// Work decomposition.  Points are cut into groups of 64*KP (KP points per
// lane, lane-contiguous so loads coalesce); groups are cut into S contiguous
// slices; orders m are cut into R contiguous ranges of about equal work
// sum_m (lmax-m+1).  One workgroup = one wavefront = one (slice, range) item:
// it walks its slice group by group and, for every m of its range, runs the
// l-recurrence of App. A.1 for its 64*KP points in registers, accumulates the
// per-l sums in registers over an l-block of LB values, reduces them across the
// 64 lanes in a fixed order and adds them to its slice's partial a_lm column
// (FP64) in global memory.  The first group of a slice stores instead of adding,
// so no clearing pass is needed.  A second kernel sums the S partials in slice
// order and applies the per-(l, m) output scale.  Every reduction order is
// fixed, so results are bitwise reproducible.
//
// Per point the kernel carries
//   Z = w s^m e^{-i m phi}  as a complex FP64 mantissa and an int exponent,
//       advanced from m to m+1 by one complex multiply with u = s e^{-i phi}
//       (angle addition) and renormalised every step;
//   (Ehat, Ohat), the split recurrence of tables.hip (one FMA per odd step,
//       one multiply + one FMA per even step), in the recurrence type RecT;
//   q = exponent applied to Z when forming the weights W = Z 2^q (even l) and
//       V = x W (odd l), in the product type AccT.  Near the poles s^m
//       underflows while the recurrence grows: then W is 0 (ldexp underflow)
//       and the chain keeps growing until it is rescaled by a power of two,
//       which raises q, until W re-enters the range of AccT.  Contributions
//       dropped this way are below 2^-700 |w| (FP64) or 2^-35 |w| (FP32).
//
// Arithmetic types: FP64 form RecT = AccT = double.  Mixed form: FP64
// recurrence, FP32 products, per-lane sums and cross-lane reduction, FP64
// partials.  FP32 form: FP32 recurrence and products (FP64 trig, seed exponent,
// phase and partials).  The trig, seed and phase are FP64 in every form.
//
// Per term (point, l, m) the inner loop issues 3.5 VALU instructions: 1.5 for
// the recurrence and 2 FMAs into the l-block sums.  The cross-lane reduction
// costs about one add per reduced value per lane, i.e. a fraction ~2/(3.5 KP)
// of the inner loop, and moves 64*sizeof(AccT) bytes of LDS per value and lane
// group (half with the register stage), which is what limits small KP.
#include <map>
#include <mutex>
#include <type_traits>

#include "ptalm.h"
#include "ptalm_internal.h"
#include "wave_common.h"

// Static scratch of the no-allocation transform (ptalm_alm_from_points_noalloc):
// the slice partials live here instead of in memory the call allocates.  Every
// device the library runs on holds its own copy until the process ends.  In host
// code this name is only a handle: the device address comes from
// hipGetSymbolAddress (noalloc_scratch below), never from the name itself.
static __device__ __align__(256) unsigned char scratch[PTALM_NOALLOC_SCRATCH_BYTES];

namespace ptalm {

// Device address of `scratch` on the current device, looked up once per device
// with that device current and kept for later calls.
hipError_t noalloc_scratch(void **out) {
    static std::mutex mu;
    static std::map<int, void *> addr;
    int dev;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        it = addr.emplace(dev, p).first;
    }
    *out = it->second;
    return hipSuccess;
}

namespace {

template <typename RecT, typename AccT, int KP, int LB, int SWAP, int PIPE>
__global__ __launch_bounds__(64) void alm_direct_kernel(AlmArgs args) {
    static_assert(LB % 2 == 0 && 64 % (2 * LB) == 0, "LB must be even and 2*LB must divide 64");
    constexpr int V = 2 * LB;  // values reduced per l-block (re, im per l)
    using R = Red<V, SWAP>;
    constexpr int P = R::P;
    // the chain is converted to AccT for the products, so it must stay inside the
    // range of the narrower of the two types
    using NarrowT = typename std::conditional<(sizeof(AccT) < sizeof(RecT)), AccT, RecT>::type;
    constexpr int RESCALE_EVERY = (ChainRange<NarrowT>::every_l / LB) > 0 ? (ChainRange<NarrowT>::every_l / LB) : 1;
    constexpr RecT kAbove = (RecT)ChainRange<NarrowT>::above;

    __shared__ AccT red[(PIPE ? 2 : 1) * R::BUF];

    const int lane = threadIdx.x;
    const int lmax = args.lmax;
    const int r = blockIdx.x % args.n_ranges;
    const int s = args.slice_base + (int)(blockIdx.x / args.n_ranges);
    // wave-uniform: keeps everything derived from m in scalar registers, so the
    // step coefficients below are fetched with scalar loads
    const int m_a = __builtin_amdgcn_readfirstlane(args.range_m[r]);
    const int m_b = __builtin_amdgcn_readfirstlane(args.range_m[r + 1]);
    const const_ptr<RecT> coef =
        (const_ptr<RecT>)(sizeof(RecT) == 8 ? (const void *)args.coef : (const void *)args.coef32);
    // the point count, from the device when the caller's count lives there
    const int64_t n = args.n_dev ? *args.n_dev : args.n;
    const int64_t groups = args.n_dev ? (n + 64 * KP - 1) / (64 * KP) : args.groups;
    const int64_t g_a = (int64_t)s * groups / args.n_slices;
    const int64_t g_b = (int64_t)(s + 1) * groups / args.n_slices;
    double *part = args.partial + (int64_t)s * 2 * tri_size(lmax);
    const int v = lane / P;  // reduced value this lane finishes (owner when h == 0)
    const int h = lane % P;

    if (g_a >= g_b) {
        // a slice without points (only when the count comes from the device and
        // is below the planned slice count): its partial columns are zero
        for (int m = m_a; m < m_b; ++m) {
            double *pm = part + 2 * column_start(lmax, m);
            for (int k = lane; k < 2 * (lmax - m + 1); k += 64) pm[k] = 0.0;
        }
        return;
    }

    for (int64_t g = g_a; g < g_b; ++g) {
        const bool first = (g == g_a);
        // ---- point staging: coalesced SoA loads, FP64 trig -------------------
        double x[KP], Zr[KP], Zi[KP], ur[KP], ui[KP];
        int Ze[KP];
#pragma unroll
        for (int t = 0; t < KP; ++t) {
            const int64_t i = g * (64 * KP) + t * 64 + lane;
            double th = 1.5707963267948966, ph = 0.0, ww = 0.0;
            if (i < n) {
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
            ur[t] = ldexp_t(br, be);  // u itself for the per-m step (|u| <= 1)
            ui[t] = ldexp_t(bi, be);
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
            const const_ptr<RecT> cm = coef + coef_segment(lmax, m);
            double *pm = part + 2 * column_start(lmax, m);

            RecT E[KP], O[KP], y[KP];
            AccT Wr[KP], Wi[KP], Vr[KP], Vi[KP];
            int q[KP];
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                E[t] = RecT(-1);
                O[t] = RecT(0);
                y[t] = (RecT)(x[t] * x[t]);
                q[t] = Ze[t];
                const double wr = ldexp_t(Zr[t], q[t]), wi = ldexp_t(Zi[t], q[t]);
                Wr[t] = (AccT)wr;
                Wi[t] = (AccT)wi;
                Vr[t] = (AccT)(wr * x[t]);
                Vi[t] = (AccT)(wi * x[t]);
            }

            // with the pipelined reduction the block finished now is the previous one
            bool pending = false;
            bool p_owner = false;
            double *p_dst = pm;
            double p_prev = 0.0;
            int cur = 0;
            int blk = 0;
            for (int jb = 0; jb < L; jb += LB, ++blk) {
                // fetch this lane's previous partial early: its latency hides behind the block
                const bool owner = (h == 0) && (jb + (v >> 1) < L);
                double *dst = pm + 2 * jb + v;
                double prev = 0.0;
                if (owner && !first) prev = *dst;
                RecT c[LB];
#pragma unroll
                for (int k = 0; k < LB; ++k) c[k] = cm[jb + k];
                AccT vals[V];
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    AccT ar = AccT(0), ai = AccT(0);
                    if ((k & 1) == 0) {
#pragma unroll
                        for (int t = 0; t < KP; ++t) {
                            E[t] = fma(c[k] * y[t], O[t], -E[t]);
                            const AccT e = (AccT)E[t];
                            ar = fma(e, Wr[t], ar);
                            ai = fma(e, Wi[t], ai);
                        }
                    } else {
#pragma unroll
                        for (int t = 0; t < KP; ++t) {
                            O[t] = fma(c[k], E[t], -O[t]);
                            const AccT o = (AccT)O[t];
                            ar = fma(o, Vr[t], ar);
                            ai = fma(o, Vi[t], ai);
                        }
                    }
                    vals[2 * k] = ar;
                    vals[2 * k + 1] = ai;
                }
                // ---- wave reduction of the l-block (fixed order) ----------------
                if constexpr (PIPE) {
                    if (pending) {
                        wave_lds_sync();
                        const AccT sum = reduce_finish<AccT, V, SWAP>(red + (cur ^ 1) * R::BUF, v, h);
                        if (p_owner) *p_dst = p_prev + (double)sum;
                    }
                    reduce_write<AccT, V, SWAP>(red + cur * R::BUF, vals, lane);
                    pending = true;
                    p_owner = owner;
                    p_dst = dst;
                    p_prev = prev;
                    cur ^= 1;
                } else {
                    reduce_write<AccT, V, SWAP>(red, vals, lane);
                    wave_lds_sync();
                    const AccT sum = reduce_finish<AccT, V, SWAP>(red, v, h);
                    if (owner) *dst = prev + (double)sum;
                    wave_lds_sync();
                }

                // ---- keep the chain inside the range of RecT -------------------
                if ((blk % RESCALE_EVERY) == RESCALE_EVERY - 1) {
                    bool big = false;
#pragma unroll
                    for (int t = 0; t < KP; ++t) big |= fmax(fabs(E[t]), fabs(O[t])) > kAbove;
                    if (__any(big)) {
#pragma unroll
                        for (int t = 0; t < KP; ++t) {
                            const RecT mx = fmax(fabs(E[t]), fabs(O[t]));
                            const int e = (mx > kAbove) ? frexp_exp_t(mx) : 0;
                            E[t] = ldexp_t(E[t], -e);
                            O[t] = ldexp_t(O[t], -e);
                            q[t] += e;
                            const double wr = ldexp_t(Zr[t], q[t]), wi = ldexp_t(Zi[t], q[t]);
                            Wr[t] = (AccT)wr;
                            Wi[t] = (AccT)wi;
                            Vr[t] = (AccT)(wr * x[t]);
                            Vi[t] = (AccT)(wi * x[t]);
                        }
                    }
                }
            }
            if constexpr (PIPE) {
                if (pending) {
                    wave_lds_sync();
                    const AccT sum = reduce_finish<AccT, V, SWAP>(red + (cur ^ 1) * R::BUF, v, h);
                    if (p_owner) *p_dst = p_prev + (double)sum;
                    wave_lds_sync();
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

// Second pass: a_lm = sigma_lm * sum_{s<S} partial_s[l, m], slices in order, in
// FP64 with compensation (the cross-slice sum is the last reduction of every form,
// so the reduced-precision forms end in a compensated FP64 reduction too).
__global__ void reduce_partials_kernel(const double *__restrict__ partial, int n_slices,
                                       const double *__restrict__ sigma, int64_t T, double *__restrict__ alm) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < T; k += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0, cre = 0.0, cim = 0.0;
        for (int s = 0; s < n_slices; ++s) {
            const double2 v = reinterpret_cast<const double2 *>(partial + (int64_t)s * 2 * T)[k];
            neumaier_add(re, cre, v.x);
            neumaier_add(im, cim, v.y);
        }
        const double sg = sigma[k];
        reinterpret_cast<double2 *>(alm)[k] = make_double2(sg * (re + cre), sg * (im + cim));
    }
}

template <typename RecT, typename AccT, int KP, int LB, int SWAP, int PIPE>
hipError_t launch_one(const AlmArgs &a, hipStream_t stream) {
    const int blocks = a.n_ranges * (a.slice_count > 0 ? a.slice_count : a.n_slices);
    hipLaunchKernelGGL((alm_direct_kernel<RecT, AccT, KP, LB, SWAP, PIPE>), dim3(blocks), dim3(64), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

// Compiled variants: (points per lane, l-block, register stage, pipelined reduction),
// mode = register stage | pipelined << 1.
#define PTALM_FP64_VARIANTS(X)                                                                    \
    X(6, 8, 0, 0) X(7, 8, 0, 0) X(6, 16, 0, 0) X(6, 16, 1, 0) X(6, 16, 1, 1) X(6, 16, 0, 1)     \
    X(5, 16, 1, 1) X(8, 16, 1, 1) X(10, 16, 1, 1) X(12, 16, 1, 1) X(12, 16, 0, 1) X(14, 8, 0, 1) \
    X(14, 8, 1, 1) X(12, 8, 1, 1) X(4, 8, 0, 0) X(8, 32, 0, 0) X(16, 8, 0, 0) X(7, 8, 1, 1)     \
    X(8, 8, 1, 1) X(6, 8, 1, 1) X(7, 16, 1, 1)

// Mixed (FP64 recurrence, FP32 products) and FP32 (FP32 recurrence) variants.
#define PTALM_MIXED_VARIANTS(X) X(6, 16, 1, 1) X(7, 16, 1, 1) X(8, 16, 1, 1) X(8, 8, 1, 1) X(10, 8, 1, 1)
#define PTALM_FP32_VARIANTS(X) X(8, 16, 1, 1) X(10, 16, 1, 1) X(12, 16, 1, 1) X(12, 8, 1, 1) X(14, 8, 1, 1)

#define PTALM_MATCH(K, L, S, P) (kp == K && lb == L && mode == (S | (P << 1)))

int list_variants(int precision, int (*out)[3], int max) {
    int k = 0;
#define X(K, L, S, P)               \
    if (k < max) {                  \
        out[k][0] = K;              \
        out[k][1] = L;              \
        out[k][2] = S | (P << 1);   \
    }                               \
    ++k;
    if (precision == 0) { PTALM_FP64_VARIANTS(X) }
    else if (precision == 1) { PTALM_MIXED_VARIANTS(X) }
    else if (precision == 2) { PTALM_FP32_VARIANTS(X) }
#undef X
    return k;
}

bool fp64_variant_exists(int kp, int lb, int mode) {
#define X(K, L, S, P) if (PTALM_MATCH(K, L, S, P)) return true;
    PTALM_FP64_VARIANTS(X)
#undef X
    return false;
}

bool mixed_variant_exists(int kp, int lb, int mode) {
#define X(K, L, S, P) if (PTALM_MATCH(K, L, S, P)) return true;
    PTALM_MIXED_VARIANTS(X)
#undef X
    return false;
}

bool fp32_variant_exists(int kp, int lb, int mode) {
#define X(K, L, S, P) if (PTALM_MATCH(K, L, S, P)) return true;
    PTALM_FP32_VARIANTS(X)
#undef X
    return false;
}

hipError_t launch_alm_fp64(const AlmArgs &a, int kp, int lb, int mode, hipStream_t stream, bool *supported) {
    *supported = true;
#define X(K, L, S, P) if (PTALM_MATCH(K, L, S, P)) return launch_one<double, double, K, L, S, P>(a, stream);
    PTALM_FP64_VARIANTS(X)
#undef X
    *supported = false;
    return hipSuccess;
}

hipError_t launch_alm_mixed(const AlmArgs &a, int kp, int lb, int mode, hipStream_t stream, bool *supported) {
    *supported = true;
#define X(K, L, S, P) if (PTALM_MATCH(K, L, S, P)) return launch_one<double, float, K, L, S, P>(a, stream);
    PTALM_MIXED_VARIANTS(X)
#undef X
    *supported = false;
    return hipSuccess;
}

hipError_t launch_alm_fp32(const AlmArgs &a, int kp, int lb, int mode, hipStream_t stream, bool *supported) {
    *supported = true;
#define X(K, L, S, P) if (PTALM_MATCH(K, L, S, P)) return launch_one<float, float, K, L, S, P>(a, stream);
    PTALM_FP32_VARIANTS(X)
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
