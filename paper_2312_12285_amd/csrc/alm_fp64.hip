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
// 64 lanes in a fixed order and adds them to its slice's partial a_lm column in
// global memory.  The first group of a slice stores instead of adding, so no
// clearing pass is needed.  A second kernel sums the S partials in slice order
// and applies the per-(l, m) output scale.  Every reduction order is fixed, so
// results are bitwise reproducible.
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
//       FP64 range.  Contributions dropped this way are below 2^-700 |w|.
//
// Per term (point, l, m) the inner loop issues 3.5 FP64 VALU instructions:
// 1.5 for the recurrence and 2 FMAs into the l-block sums.  The cross-lane
// reduction costs about one FP64 add per reduced value per lane, i.e. a
// fraction ~2/(3.5 KP) of the inner loop, and moves 1 KB of LDS per value
// (half with the register stage), which is what limits small KP.
#include "ptalm_internal.h"

namespace ptalm {

namespace {

constexpr double kRescaleAbove = 0x1p+64;  // chain values are renormalised past this

// Read-only table pointer in the constant address space: uniform indices into
// it compile to scalar loads (s_load), so the step coefficients live in SGPRs.
typedef const double __attribute__((address_space(4))) *const_f64_ptr;

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

// Cross-lane reduction of the per-lane l-block sums (V values per lane, value
// v = 2k + c for l = jb + k and c = re/im).  Optional register stage (SWAP = 1):
// v_permlane32_swap exchanges the upper half of value i with the lower half of
// value i + V/2, so after one FP64 add each lane holds V/2 values summed over
// two lanes.  The rest goes through LDS as a transpose: every lane writes its
// values, then P = 64/V lanes per value each add an interleaved share of the
// entries and combine by DPP.  All orders are fixed.
template <int V, int SWAP>
struct Red {
    static constexpr int NV = V >> SWAP;        // values per lane entering LDS
    static constexpr int ENTRIES = 64 >> SWAP;  // lanes contributing to each value there
    static constexpr int P = 64 / V;            // lanes combining one value at the end
    static constexpr int ROW = ENTRIES + 1;     // padded LDS row (doubles)
    static constexpr int BUF = V * ROW;         // doubles per LDS buffer
};

// x from lane (lane ^ xor_mask) within each quad (DPP quad_perm), xor_mask 1 or 2
__device__ inline double dpp_xor(double x, int xor_mask) {
    const int lo = __double2loint(x), hi = __double2hiint(x);
    if (xor_mask == 1)
        return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false),
                                __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false));
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false),
                            __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false));
}

// Lanes 0-31 get value a summed over lanes j and j+32; lanes 32-63 get value b
// summed over lanes j-32 and j (v_permlane32_swap on both halves of each double).
__device__ inline double swap32_add(double a, double b) {
    unsigned al = __double2loint(a), ah = __double2hiint(a), bl = __double2loint(b), bh = __double2hiint(b);
    auto lo = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// Orders LDS accesses of this wavefront (each workgroup is one wavefront, and
// one wavefront's LDS operations complete in order).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int V, int SWAP>
__device__ inline void reduce_write(double *buf, const double (&vals)[V], int lane) {
    using R = Red<V, SWAP>;
    if constexpr (SWAP == 0) {
#pragma unroll
        for (int i = 0; i < V; ++i) buf[i * R::ROW + lane] = vals[i];
    } else {
        const int half = lane >> 5;
#pragma unroll
        for (int i = 0; i < V / 2; ++i) {
            const double u = swap32_add(vals[i], vals[i + V / 2]);
            buf[(i + half * (V / 2)) * R::ROW + (lane & 31)] = u;
        }
    }
}

template <int V, int SWAP>
__device__ inline double reduce_finish(const double *buf, int v, int h) {
    using R = Red<V, SWAP>;
    static_assert(R::P <= 4, "at most 4 lanes per value");
    double sum = buf[v * R::ROW + h];
#pragma unroll
    for (int k = 1; k < R::ENTRIES / R::P; ++k) sum += buf[v * R::ROW + h + k * R::P];
    if constexpr (R::P >= 2) sum += dpp_xor(sum, 1);
    if constexpr (R::P >= 4) sum += dpp_xor(sum, 2);
    return sum;
}

template <int KP, int LB, int SWAP, int PIPE>
__global__ __launch_bounds__(64) void alm_fp64_kernel(AlmArgs args) {
    static_assert(LB % 2 == 0 && 64 % (2 * LB) == 0, "LB must be even and 2*LB must divide 64");
    constexpr int V = 2 * LB;  // values reduced per l-block (re, im per l)
    using R = Red<V, SWAP>;
    constexpr int P = R::P;
    constexpr int RESCALE_EVERY = (64 / LB) > 0 ? (64 / LB) : 1;  // l-blocks between chain checks

    __shared__ double red[(PIPE ? 2 : 1) * R::BUF];

    const int lane = threadIdx.x;
    const int lmax = args.lmax;
    const int r = blockIdx.x % args.n_ranges;
    const int s = blockIdx.x / args.n_ranges;
    // wave-uniform: keeps everything derived from m in scalar registers, so the
    // step coefficients below are fetched with scalar loads
    const int m_a = __builtin_amdgcn_readfirstlane(args.range_m[r]);
    const int m_b = __builtin_amdgcn_readfirstlane(args.range_m[r + 1]);
    const const_f64_ptr coef = (const_f64_ptr)args.coef;
    const int64_t g_a = (int64_t)s * args.groups / args.n_slices;
    const int64_t g_b = (int64_t)(s + 1) * args.groups / args.n_slices;
    double *part = args.partial + (int64_t)s * 2 * tri_size(lmax);
    const int v = lane / P;  // reduced value this lane finishes (owner when h == 0)
    const int h = lane % P;

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
            ur[t] = ldexp_d(br, be);  // u itself for the per-m step (|u| <= 1)
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
            const const_f64_ptr cm = coef + coef_segment(lmax, m);
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
                double c[LB];
#pragma unroll
                for (int k = 0; k < LB; ++k) c[k] = cm[jb + k];
                double vals[V];
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    double ar = 0.0, ai = 0.0;
                    if ((k & 1) == 0) {
#pragma unroll
                        for (int t = 0; t < KP; ++t) {
                            E[t] = fma(c[k] * y[t], O[t], -E[t]);
                            ar = fma(E[t], Wr[t], ar);
                            ai = fma(E[t], Wi[t], ai);
                        }
                    } else {
#pragma unroll
                        for (int t = 0; t < KP; ++t) {
                            O[t] = fma(c[k], E[t], -O[t]);
                            ar = fma(O[t], Vr[t], ar);
                            ai = fma(O[t], Vi[t], ai);
                        }
                    }
                    vals[2 * k] = ar;
                    vals[2 * k + 1] = ai;
                }
                // ---- wave reduction of the l-block (fixed order) ----------------
                if constexpr (PIPE) {
                    if (pending) {
                        wave_lds_sync();
                        const double sum = reduce_finish<V, SWAP>(red + (cur ^ 1) * R::BUF, v, h);
                        if (p_owner) *p_dst = p_prev + sum;
                    }
                    reduce_write<V, SWAP>(red + cur * R::BUF, vals, lane);
                    pending = true;
                    p_owner = owner;
                    p_dst = dst;
                    p_prev = prev;
                    cur ^= 1;
                } else {
                    reduce_write<V, SWAP>(red, vals, lane);
                    wave_lds_sync();
                    const double sum = reduce_finish<V, SWAP>(red, v, h);
                    if (owner) *dst = prev + sum;
                    wave_lds_sync();
                }

                // ---- keep the chain inside the FP64 range ----------------------
                // Growth over 64 steps stays below 2^255 even next to the poles
                // at m ~ 3000, so checking every 64 l against 2^64 cannot overflow.
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
            if constexpr (PIPE) {
                if (pending) {
                    wave_lds_sync();
                    const double sum = reduce_finish<V, SWAP>(red + (cur ^ 1) * R::BUF, v, h);
                    if (p_owner) *p_dst = p_prev + sum;
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

template <int KP, int LB, int SWAP, int PIPE>
hipError_t launch_one(const AlmArgs &a, hipStream_t stream) {
    const int blocks = a.n_ranges * a.n_slices;
    hipLaunchKernelGGL((alm_fp64_kernel<KP, LB, SWAP, PIPE>), dim3(blocks), dim3(64), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

// Compiled variants: (points per lane, l-block, register stage, pipelined reduction).
// mode = register stage | pipelined << 1.
#define PTALM_FP64_VARIANTS(X)                                                                    \
    X(6, 8, 0, 0) X(7, 8, 0, 0) X(6, 16, 0, 0) X(6, 16, 1, 0) X(6, 16, 1, 1) X(6, 16, 0, 1)     \
    X(5, 16, 1, 1) X(8, 16, 1, 1) X(10, 16, 1, 1) X(12, 16, 1, 1) X(12, 16, 0, 1) X(14, 8, 0, 1) \
    X(14, 8, 1, 1) X(12, 8, 1, 1) X(4, 8, 0, 0) X(8, 32, 0, 0) X(16, 8, 0, 0)

bool fp64_variant_exists(int kp, int lb, int mode) {
#define X(K, L, S, P) \
    if (kp == K && lb == L && mode == (S | (P << 1))) return true;
    PTALM_FP64_VARIANTS(X)
#undef X
    return false;
}

hipError_t launch_alm_fp64(const AlmArgs &a, int kp, int lb, int mode, hipStream_t stream, bool *supported) {
    *supported = true;
#define X(K, L, S, P) \
    if (kp == K && lb == L && mode == (S | (P << 1))) return launch_one<K, L, S, P>(a, stream);
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
