// Spin-weighted direct transform for shear (spin +-2 harmonics, end of Sec. 4):
//     _{+2}a_lm = sum_i w_i (g1_i + i g2_i) _{+2}Y*_lm(theta_i, phi_i),
//     _{-2}a_lm = sum_i w_i (g1_i - i g2_i) _{-2}Y*_lm(theta_i, phi_i),
//     a^E = -(_{+2}a + _{-2}a) / 2,   a^B = i (_{+2}a - _{-2}a) / 2,
// for 2 <= l <= lmax, 0 <= m <= l, with
//     _sY_lm(theta, phi) = (-1)^m sqrt((2l+1)/4pi) d^l_{m,-s}(theta) e^{i m phi}
// (the convention of Goldberg et al. 1967, healpy's E/B signs).
//
// Recurrence.  For fixed m and m' = -s the Wigner d obey the three-term relation
//     d_{l+1} = (a_l x - b_l m m') d_l - c_l d_{l-1},   x = cos(theta),
//     a_l = (2l+1) l (l+1) / D_l,  b_l = (2l+1) / D_l,
//     c_l = (l+1) sqrt((l^2-m^2)(l^2-4)) / D_l,  D_l = l sqrt(((l+1)^2-m^2)((l+1)^2-4)),
// started at l0 = max(m, 2), where the Wigner sum has a single term.  Writing
// d_l = kappa_l E_l with kappa_{l0} = kappa_{l0+1} = 1 and kappa_{l+1} = c_l kappa_{l-1}
// turns it into
//     E_{l+1} = (alpha_l x -+ beta_l) E_l - E_{l-1},
//     alpha_l = a_l kappa_l / kappa_{l+1},  beta_l = 2m (2l+1) kappa_l / (D_l kappa_{l+1}),
// the upper sign for s = -2 and the lower for s = +2, so the two spins share
// alpha, beta and kappa and each step is two FMAs per spin.
//
// Seeds (per point; c, s = cos, sin(theta/2); sin(theta) = 2cs):
//     m = 0:  d^2_{0,-+2} = (sqrt6/4) sin^2 theta
//     m = 1:  d^2_{1,-2} = sin theta * s^2,     d^2_{1,2} = sin theta * (-c^2)
//     m >= 2: d^m_{m,-+2} = K'_m sin^{m-2} theta * (s^4 or c^4),
//             K'_m = sqrt(C(2m, m+2)) 2^{2-m} = prod_{k=2}^{m-1} sqrt((2k+2)(2k+1)/((k+3)(k-1)))/2
// The sin^p theta e^{-i m phi} part is carried per point as a complex FP64
// mantissa with a binary exponent (advanced with u = sin(theta) e^{-i phi}), the
// (s^4, c^4)-type factor starts the two chains, and K'_m, kappa_l and the
// normalisation go into the per-(l, m) output scale
//     sigma_lm = (-1)^m sqrt((2l+1)/4pi) kappa_l K'_m   (0 for l < 2).
//
// Work decomposition as in the scalar kernel: groups of 64*KP points, S point
// slices, R balanced order ranges; one wavefront per (slice, range) item, the
// per-l sums of both spins (4 reals per l) reduced across lanes in a fixed
// order into the slice's partial column; a finishing kernel sums the slices in
// order, applies sigma and forms E and B.  Per term (point, l, m) the inner loop
// issues 8 FP64 FMAs: 2 for the two step factors, 2 for the two chains, 4 for
// the complex accumulations.  A second form runs one spin per wavefront
// (twice the wavefronts, 2 reals per l reduced, 4 FMAs per point and step); the
// host picks the form.
#include "ptalm_internal.h"
#include "wave_common.h"

namespace ptalm {

namespace {

constexpr double kInv4Pi = 0.25 / 3.14159265358979323846;

// One thread per order m: step pairs (alpha, beta) at coef[segment(m) + j]
// (the pair that produces E_l, l = m + j; (0, 0) at l = l0 so that the kernel's
// general step turns its start state into the seed; zero before l0 and past
// lmax through the padding) and sigma at column_start(m) + j.
__global__ void spin_tables_kernel(int lmax, double2 *coef, double *sigma) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m > lmax) return;
    const int l0 = m > 2 ? m : 2;
    double K;
    if (m == 0) {
        K = 0.6123724356957945;  // sqrt(6) / 4
    } else {
        K = 1.0;
        for (int k = 2; k < m; ++k)
            K *= 0.5 * sqrt(((2.0 * k + 2.0) * (2.0 * k + 1.0)) / ((k + 3.0) * (k - 1.0)));
    }
    double2 *seg = coef + coef_segment(lmax, m);
    const int64_t col = column_start(lmax, m);
    const int jmax = lmax - m;
    for (int j = 0; j <= jmax + kCoefPad; ++j) seg[j] = make_double2(0.0, 0.0);
    for (int j = 0; j < l0 - m && j <= jmax; ++j) sigma[col + j] = 0.0;
    if (l0 > lmax) return;
    // kappa_{l-1}, kappa_l while stepping l -> l+1
    double kap_prev = 1.0, kap = 1.0;
    const double sgn = (m & 1) ? -1.0 : 1.0;
    sigma[col + (l0 - m)] = sgn * sqrt((2.0 * l0 + 1.0) * kInv4Pi) * K;
    for (int l = l0; l < lmax; ++l) {
        const double lp1 = l + 1.0, dl = l, dm = m;
        const double D = dl * sqrt((lp1 * lp1 - dm * dm) * (lp1 * lp1 - 4.0));
        const double a = (2.0 * l + 1.0) * dl * lp1 / D;
        const double b = 2.0 * dm * (2.0 * l + 1.0) / D;
        double kap_next;
        if (l == l0) {
            kap_next = 1.0;
        } else {
            const double c = lp1 * sqrt((dl * dl - dm * dm) * (dl * dl - 4.0)) / D;
            kap_next = c * kap_prev;
        }
        const double r = kap / kap_next;
        seg[l + 1 - m] = make_double2(a * r, b * r);
        sigma[col + (l + 1 - m)] = sgn * sqrt((2.0 * l + 3.0) * kInv4Pi) * kap_next * K;
        kap_prev = kap;
        kap = kap_next;
    }
}

// Per-point state for order m: x, u = sin(theta) e^{-i phi}, the chain start
// factors s2 = sin^2(theta/2), c2 = cos^2(theta/2), and the seed
// Z = w sin^p(theta) e^{-i m phi} (p = m for m < 2, m - 2 for m >= 2) as a
// normalised complex mantissa with exponent Ze.
__device__ inline void spin_point_seed(double th, double ph, double ww, int m, double &x, double &ur, double &ui,
                                       double &s2, double &c2, double &Zr, double &Zi, int &Ze) {
    double sh, ch, sp, cp;
    sincos(0.5 * th, &sh, &ch);
    sincos(ph, &sp, &cp);
    x = (ch - sh) * (ch + sh);
    s2 = sh * sh;
    c2 = ch * ch;
    const double st = 2.0 * sh * ch;
    double br = st * cp, bi = -st * sp;
    int be = 0;
    renorm(br, bi, be);
    ur = ldexp_t(br, be);
    ui = ldexp_t(bi, be);
    double rr = 1.0, ri = 0.0;
    if (m >= 2) {  // e^{-2 i phi}
        rr = (cp - sp) * (cp + sp);
        ri = -2.0 * sp * cp;
    }
    int re = 0;
    for (int k = (m < 2 ? m : m - 2); k; k >>= 1) {
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
    Zr = rr * ww;
    Zi = ri * ww;
    Ze = re;
    renorm(Zr, Zi, Ze);
}

template <int KP, int LB>
__global__ __launch_bounds__(64) void spin_direct_kernel(SpinArgs args) {
    static_assert(LB % 2 == 0 && 64 % (4 * LB) == 0, "4*LB must divide 64");
    constexpr int V = 4 * LB;  // values reduced per l-block: (+2 re, +2 im, -2 re, -2 im) per l
    using R = Red<V, 1>;
    constexpr int P = R::P;
    constexpr int RESCALE_EVERY = ChainRange<double>::every_l / LB;
    constexpr double kAbove = ChainRange<double>::above;

    __shared__ double red[2 * R::BUF];

    const int lane = threadIdx.x;
    const int lmax = args.lmax;
    const int r = blockIdx.x % args.n_ranges;
    const int s = blockIdx.x / args.n_ranges;
    const int m_a = __builtin_amdgcn_readfirstlane(args.range_m[r]);
    const int m_b = __builtin_amdgcn_readfirstlane(args.range_m[r + 1]);
    // (alpha, beta) pairs read as two doubles each: uniform indices, scalar loads
    const const_ptr<double> coef = (const_ptr<double>)(const void *)args.coef;
    const int64_t g_a = (int64_t)s * args.groups / args.n_slices;
    const int64_t g_b = (int64_t)(s + 1) * args.groups / args.n_slices;
    double *part = args.partial + (int64_t)s * 4 * tri_size(lmax);
    const int v = lane / P;
    const int h = lane % P;

    for (int64_t g = g_a; g < g_b; ++g) {
        const bool first = (g == g_a);
        double x[KP], ur[KP], ui[KP], s2[KP], c2[KP], Zr[KP], Zi[KP], gr[KP], gi[KP];
        int Ze[KP];
#pragma unroll
        for (int t = 0; t < KP; ++t) {
            const int64_t i = g * (64 * KP) + t * 64 + lane;
            double th = 1.5707963267948966, ph = 0.0, ww = 0.0, a1 = 0.0, a2 = 0.0;
            if (i < args.n) {
                th = args.theta[i];
                ph = args.phi[i];
                ww = args.w[i];
                a1 = args.g1[i];
                a2 = args.g2[i];
            }
            gr[t] = a1;
            gi[t] = a2;
            spin_point_seed(th, ph, ww, m_a, x[t], ur[t], ui[t], s2[t], c2[t], Zr[t], Zi[t], Ze[t]);
        }

        for (int m = m_a; m < m_b; ++m) {
            if (m == 2 && m_a < 2) {
                // the seed's power of sin(theta) restarts at m = 2 (from 1 at m = 1)
#pragma unroll
                for (int t = 0; t < KP; ++t) {
                    const int64_t i = g * (64 * KP) + t * 64 + lane;
                    double th = 1.5707963267948966, ph = 0.0, ww = 0.0;
                    if (i < args.n) {
                        th = args.theta[i];
                        ph = args.phi[i];
                        ww = args.w[i];
                    }
                    spin_point_seed(th, ph, ww, 2, x[t], ur[t], ui[t], s2[t], c2[t], Zr[t], Zi[t], Ze[t]);
                }
            }
            const int L = lmax - m + 1;          // entries of order m's column
            const int j0 = (m >= 2) ? 0 : 2 - m;  // first l >= 2
            const const_ptr<double> cm = coef + 2 * coef_segment(lmax, m);
            double *pm = part + 4 * column_start(lmax, m);

            double Ep[KP], Epp[KP], Em[KP], Emp[KP];
            double Wpr[KP], Wpi[KP], Wmr[KP], Wmi[KP];
            int q[KP];
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                // chain start: (E, E_prev) = (0, -v) and a (0, 0) step give E = v at l0
                double vp, vm;
                if (m == 0) {
                    vp = 4.0 * s2[t] * c2[t];
                    vm = vp;
                } else if (m == 1) {
                    vp = s2[t];
                    vm = -c2[t];
                } else {
                    vp = s2[t] * s2[t];
                    vm = c2[t] * c2[t];
                }
                Ep[t] = 0.0;
                Epp[t] = -vp;
                Em[t] = 0.0;
                Emp[t] = -vm;
                q[t] = Ze[t];
                const double zr = ldexp_t(Zr[t], q[t]), zi = ldexp_t(Zi[t], q[t]);
                // W+ = Z G, W- = Z conj(G)
                Wpr[t] = zr * gr[t] - zi * gi[t];
                Wpi[t] = zr * gi[t] + zi * gr[t];
                Wmr[t] = zr * gr[t] + zi * gi[t];
                Wmi[t] = zi * gr[t] - zr * gi[t];
            }

            bool pending = false;
            bool p_owner = false;
            double *p_dst = pm;
            double p_prev = 0.0;
            int cur = 0;
            int blk = 0;
            for (int jb = j0; jb < L; jb += LB, ++blk) {
                const bool owner = (h == 0) && (jb + (v >> 2) < L);
                double *dst = pm + 4 * jb + v;
                double prev = 0.0;
                if (owner && !first) prev = *dst;
                double ca[LB], cb[LB];
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    ca[k] = cm[2 * (jb + k)];
                    cb[k] = cm[2 * (jb + k) + 1];
                }
                double vals[V];
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    double pr = 0.0, pi = 0.0, mr = 0.0, mi = 0.0;
#pragma unroll
                    for (int t = 0; t < KP; ++t) {
                        const double tp = fma(ca[k], x[t], cb[k]);   // s = +2
                        const double tm = fma(ca[k], x[t], -cb[k]);  // s = -2
                        const double ep = fma(tp, Ep[t], -Epp[t]);
                        const double em = fma(tm, Em[t], -Emp[t]);
                        Epp[t] = Ep[t];
                        Ep[t] = ep;
                        Emp[t] = Em[t];
                        Em[t] = em;
                        pr = fma(ep, Wpr[t], pr);
                        pi = fma(ep, Wpi[t], pi);
                        mr = fma(em, Wmr[t], mr);
                        mi = fma(em, Wmi[t], mi);
                    }
                    vals[4 * k] = pr;
                    vals[4 * k + 1] = pi;
                    vals[4 * k + 2] = mr;
                    vals[4 * k + 3] = mi;
                }
                if (pending) {
                    wave_lds_sync();
                    const double sum = reduce_finish<double, V, 1>(red + (cur ^ 1) * R::BUF, v, h);
                    if (p_owner) *p_dst = p_prev + sum;
                }
                reduce_write<double, V, 1>(red + cur * R::BUF, vals, lane);
                pending = true;
                p_owner = owner;
                p_dst = dst;
                p_prev = prev;
                cur ^= 1;

                if ((blk % RESCALE_EVERY) == RESCALE_EVERY - 1) {
                    bool big = false;
#pragma unroll
                    for (int t = 0; t < KP; ++t)
                        big |= fmax(fmax(fabs(Ep[t]), fabs(Epp[t])), fmax(fabs(Em[t]), fabs(Emp[t]))) > kAbove;
                    if (__any(big)) {
#pragma unroll
                        for (int t = 0; t < KP; ++t) {
                            const double mx = fmax(fmax(fabs(Ep[t]), fabs(Epp[t])), fmax(fabs(Em[t]), fabs(Emp[t])));
                            const int e = (mx > kAbove) ? frexp_exp_t(mx) : 0;
                            Ep[t] = ldexp_t(Ep[t], -e);
                            Epp[t] = ldexp_t(Epp[t], -e);
                            Em[t] = ldexp_t(Em[t], -e);
                            Emp[t] = ldexp_t(Emp[t], -e);
                            q[t] += e;
                            const double zr = ldexp_t(Zr[t], q[t]), zi = ldexp_t(Zi[t], q[t]);
                            Wpr[t] = zr * gr[t] - zi * gi[t];
                            Wpi[t] = zr * gi[t] + zi * gr[t];
                            Wmr[t] = zr * gr[t] + zi * gi[t];
                            Wmi[t] = zi * gr[t] - zr * gi[t];
                        }
                    }
                }
            }
            if (pending) {
                wave_lds_sync();
                const double sum = reduce_finish<double, V, 1>(red + (cur ^ 1) * R::BUF, v, h);
                if (p_owner) *p_dst = p_prev + sum;
                wave_lds_sync();
            }
            // next order: Z <- Z u (the restart at m = 2 overrides it)
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

// One spin per wavefront.  Items (slice, range, spin) with the spin fastest, so the
// two wavefronts of one (slice, range) run side by side over the same points and step
// pairs.  A wavefront carries one chain per point and reduces 2 reals per l (its spin's
// re and im) into its half of the 4 reals per (l, m) of the partial, so per term it
// does half the two-spin kernel's cross-lane work and has the registers for more
// points per lane.  Per point and step: the step factor, the chain and two
// accumulations (4 FMAs); the lane values are those of the two-spin kernel.
template <int KP, int LB, int SGN>
__device__ __forceinline__ void spin_single_body(const SpinArgs &args, int r, int s, double *red) {
    constexpr int V = 2 * LB;  // values reduced per l-block: (re, im) of this spin per l
    using R = Red<V, 1>;
    constexpr int P = R::P;
    constexpr int RESCALE_EVERY = ChainRange<double>::every_l / LB;
    constexpr double kAbove = ChainRange<double>::above;
    constexpr int OFF = SGN > 0 ? 0 : 2;  // this spin's (re, im) within the 4 reals per (l, m)

    const int lane = threadIdx.x;
    const int lmax = args.lmax;
    const int m_a = __builtin_amdgcn_readfirstlane(args.range_m[r]);
    const int m_b = __builtin_amdgcn_readfirstlane(args.range_m[r + 1]);
    const const_ptr<double> coef = (const_ptr<double>)(const void *)args.coef;
    const int64_t g_a = (int64_t)s * args.groups / args.n_slices;
    const int64_t g_b = (int64_t)(s + 1) * args.groups / args.n_slices;
    double *part = args.partial + (int64_t)s * 4 * tri_size(lmax);
    const int v = lane / P;
    const int h = lane % P;

    for (int64_t g = g_a; g < g_b; ++g) {
        const bool first = (g == g_a);
        double x[KP], ur[KP], ui[KP], s2[KP], c2[KP], Zr[KP], Zi[KP], gr[KP], gi[KP];
        int Ze[KP];
#pragma unroll
        for (int t = 0; t < KP; ++t) {
            const int64_t i = g * (64 * KP) + t * 64 + lane;
            double th = 1.5707963267948966, ph = 0.0, ww = 0.0, a1 = 0.0, a2 = 0.0;
            if (i < args.n) {
                th = args.theta[i];
                ph = args.phi[i];
                ww = args.w[i];
                a1 = args.g1[i];
                a2 = args.g2[i];
            }
            gr[t] = a1;
            gi[t] = a2;
            spin_point_seed(th, ph, ww, m_a, x[t], ur[t], ui[t], s2[t], c2[t], Zr[t], Zi[t], Ze[t]);
        }

        for (int m = m_a; m < m_b; ++m) {
            if (m == 2 && m_a < 2) {
#pragma unroll
                for (int t = 0; t < KP; ++t) {
                    const int64_t i = g * (64 * KP) + t * 64 + lane;
                    double th = 1.5707963267948966, ph = 0.0, ww = 0.0;
                    if (i < args.n) {
                        th = args.theta[i];
                        ph = args.phi[i];
                        ww = args.w[i];
                    }
                    spin_point_seed(th, ph, ww, 2, x[t], ur[t], ui[t], s2[t], c2[t], Zr[t], Zi[t], Ze[t]);
                }
            }
            const int L = lmax - m + 1;
            const int j0 = (m >= 2) ? 0 : 2 - m;
            const const_ptr<double> cm = coef + 2 * coef_segment(lmax, m);
            double *pm = part + 4 * column_start(lmax, m) + OFF;

            double E[KP], Ep[KP], Wr[KP], Wi[KP];
            int q[KP];
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                double sv;
                if (m == 0) sv = 4.0 * s2[t] * c2[t];
                else if (m == 1) sv = SGN > 0 ? s2[t] : -c2[t];
                else sv = SGN > 0 ? s2[t] * s2[t] : c2[t] * c2[t];
                E[t] = 0.0;
                Ep[t] = -sv;
                q[t] = Ze[t];
                const double zr = ldexp_t(Zr[t], q[t]), zi = ldexp_t(Zi[t], q[t]);
                // W+ = Z G, W- = Z conj(G)
                Wr[t] = SGN > 0 ? zr * gr[t] - zi * gi[t] : zr * gr[t] + zi * gi[t];
                Wi[t] = SGN > 0 ? zr * gi[t] + zi * gr[t] : zi * gr[t] - zr * gi[t];
            }

            bool pending = false;
            bool p_owner = false;
            double *p_dst = pm;
            double p_prev = 0.0;
            int cur = 0;
            int blk = 0;
            for (int jb = j0; jb < L; jb += LB, ++blk) {
                const bool owner = (h == 0) && (jb + (v >> 1) < L);
                double *dst = pm + 4 * (jb + (v >> 1)) + (v & 1);
                double prev = 0.0;
                if (owner && !first) prev = *dst;
                double ca[LB], cb[LB];
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    ca[k] = cm[2 * (jb + k)];
                    cb[k] = SGN > 0 ? cm[2 * (jb + k) + 1] : -cm[2 * (jb + k) + 1];
                }
                double vals[V];
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    double re = 0.0, im = 0.0;
#pragma unroll
                    for (int t = 0; t < KP; ++t) {
                        const double f = fma(ca[k], x[t], cb[k]);
                        const double e = fma(f, E[t], -Ep[t]);
                        Ep[t] = E[t];
                        E[t] = e;
                        re = fma(e, Wr[t], re);
                        im = fma(e, Wi[t], im);
                    }
                    vals[2 * k] = re;
                    vals[2 * k + 1] = im;
                }
                if (pending) {
                    wave_lds_sync();
                    const double sum = reduce_finish<double, V, 1>(red + (cur ^ 1) * R::BUF, v, h);
                    if (p_owner) *p_dst = p_prev + sum;
                }
                reduce_write<double, V, 1>(red + cur * R::BUF, vals, lane);
                pending = true;
                p_owner = owner;
                p_dst = dst;
                p_prev = prev;
                cur ^= 1;

                if ((blk % RESCALE_EVERY) == RESCALE_EVERY - 1) {
                    bool big = false;
#pragma unroll
                    for (int t = 0; t < KP; ++t) big |= fmax(fabs(E[t]), fabs(Ep[t])) > kAbove;
                    if (__any(big)) {
#pragma unroll
                        for (int t = 0; t < KP; ++t) {
                            const double mx = fmax(fabs(E[t]), fabs(Ep[t]));
                            const int e = (mx > kAbove) ? frexp_exp_t(mx) : 0;
                            E[t] = ldexp_t(E[t], -e);
                            Ep[t] = ldexp_t(Ep[t], -e);
                            q[t] += e;
                            const double zr = ldexp_t(Zr[t], q[t]), zi = ldexp_t(Zi[t], q[t]);
                            Wr[t] = SGN > 0 ? zr * gr[t] - zi * gi[t] : zr * gr[t] + zi * gi[t];
                            Wi[t] = SGN > 0 ? zr * gi[t] + zi * gr[t] : zi * gr[t] - zr * gi[t];
                        }
                    }
                }
            }
            if (pending) {
                wave_lds_sync();
                const double sum = reduce_finish<double, V, 1>(red + (cur ^ 1) * R::BUF, v, h);
                if (p_owner) *p_dst = p_prev + sum;
                wave_lds_sync();
            }
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

template <int KP, int LB>
__global__ __launch_bounds__(64) void spin_single_kernel(SpinArgs args) {
    static_assert(LB % 2 == 0 && 64 % (2 * LB) == 0 && 2 * LB >= 16, "2*LB must divide 64, LB >= 8");
    __shared__ double red[2 * Red<2 * LB, 1>::BUF];
    const int item = (int)(blockIdx.x >> 1);
    const int r = item % args.n_ranges;
    const int s = item / args.n_ranges;
    if (blockIdx.x & 1u)
        spin_single_body<KP, LB, -1>(args, r, s, red);
    else
        spin_single_body<KP, LB, 1>(args, r, s, red);
}

// E = -sigma (S+ + S-) / 2, B = i sigma (S+ - S-) / 2 with S+-, the compensated slice sums in
// slice order; entries with sigma = 0 (l < 2) are written as 0 without reading
// the partials (never written for them).
__global__ void spin_finish_kernel(const double *__restrict__ partial, int n_slices, const double *__restrict__ sigma,
                                   int64_t T, double *__restrict__ alm_e, double *__restrict__ alm_b) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < T; k += (int64_t)gridDim.x * blockDim.x) {
        const double sg = sigma[k];
        double pr = 0.0, pi = 0.0, mr = 0.0, mi = 0.0, cpr = 0.0, cpi = 0.0, cmr = 0.0, cmi = 0.0;
        if (sg != 0.0) {
            for (int s = 0; s < n_slices; ++s) {
                const double4 v = reinterpret_cast<const double4 *>(partial + (int64_t)s * 4 * T)[k];
                neumaier_add(pr, cpr, v.x);
                neumaier_add(pi, cpi, v.y);
                neumaier_add(mr, cmr, v.z);
                neumaier_add(mi, cmi, v.w);
            }
        }
        pr += cpr;
        pi += cpi;
        mr += cmr;
        mi += cmi;
        const double h = 0.5 * sg;
        reinterpret_cast<double2 *>(alm_e)[k] = make_double2(-h * (pr + mr), -h * (pi + mi));
        reinterpret_cast<double2 *>(alm_b)[k] = make_double2(-h * (pi - mi), h * (pr - mr));
    }
}

template <int KP, int LB>
hipError_t launch_spin_one(const SpinArgs &a, hipStream_t stream) {
    const int blocks = a.n_ranges * a.n_slices;
    hipLaunchKernelGGL((spin_direct_kernel<KP, LB>), dim3(blocks), dim3(64), 0, stream, a);
    return hipGetLastError();
}

template <int KP, int LB>
hipError_t launch_spin_single(const SpinArgs &a, hipStream_t stream) {
    const int blocks = 2 * a.n_ranges * a.n_slices;
    hipLaunchKernelGGL((spin_single_kernel<KP, LB>), dim3(blocks), dim3(64), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

#define PTALM_SPIN_VARIANTS(X) X(4, 8) X(3, 8) X(2, 8) X(4, 16) X(3, 16) X(5, 8) X(6, 4) X(4, 4)
#define PTALM_SPIN_SINGLE_VARIANTS(X) X(4, 8) X(5, 8) X(6, 8) X(7, 8) X(8, 8) X(4, 16) X(5, 16) X(6, 16)

bool spin_variant_exists(int kp, int lb, bool single) {
#define X(K, L) if (kp == K && lb == L) return true;
    if (single) {
        PTALM_SPIN_SINGLE_VARIANTS(X)
    } else {
        PTALM_SPIN_VARIANTS(X)
    }
#undef X
    return false;
}

hipError_t launch_spin(const SpinArgs &a, int kp, int lb, bool single, hipStream_t stream, bool *supported) {
    *supported = true;
    if (single) {
#define X(K, L) if (kp == K && lb == L) return launch_spin_single<K, L>(a, stream);
        PTALM_SPIN_SINGLE_VARIANTS(X)
#undef X
    } else {
#define X(K, L) if (kp == K && lb == L) return launch_spin_one<K, L>(a, stream);
        PTALM_SPIN_VARIANTS(X)
#undef X
    }
    *supported = false;
    return hipSuccess;
}

hipError_t launch_spin_finish(const double *partial, int n_slices, const double *sigma, int lmax, double *alm_e,
                              double *alm_b, hipStream_t stream) {
    const int64_t T = tri_size(lmax);
    const int threads = 256;
    int64_t blocks = (T + threads - 1) / threads;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(spin_finish_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, partial, n_slices, sigma,
                       T, alm_e, alm_b);
    return hipGetLastError();
}

hipError_t build_spin_tables(int lmax, SpinTables *t, hipStream_t stream) {
    hipError_t e;
    if ((e = hipMalloc(&t->coef, sizeof(double2) * coef_table_size(lmax))) != hipSuccess) return e;
    if ((e = hipMalloc(&t->sigma, sizeof(double) * tri_size(lmax))) != hipSuccess) return e;
    const int threads = 64;
    const int blocks = (lmax + 1 + threads - 1) / threads;
    hipLaunchKernelGGL(spin_tables_kernel, dim3(blocks), dim3(threads), 0, stream, lmax, t->coef, t->sigma);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    t->lmax = lmax;
    return hipSuccess;
}

}  // namespace ptalm
