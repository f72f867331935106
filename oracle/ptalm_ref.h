/*
 * ptalm_ref.h -- CPU oracle of the direct point-to-harmonic transform.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no source, header, table or helper with the GPU library.
 *
 * All pointers are HOST pointers.  a_lm arrays hold 2*T doubles, (re, im)
 * interleaved, in healpy order: index(l, m) = m*(2*lmax+1-m)/2 + l, 0<=m<=l<=lmax,
 * T = (lmax+1)(lmax+2)/2.  Functions return 0 on success, -1 on bad arguments.
 */
#ifndef PTALM_REF_H
#define PTALM_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* a_lm = sum_i w_i Y*_lm(theta_i, phi_i) for 0<=m<=l<=lmax (eq. alm_def, Sec. 2.2).
 * FP64 recurrence of App. A.1 with an exponent-tracked sectoral seed; sums in
 * long double, in point order; parallel over m (each m owns its column), so the
 * result does not depend on nthreads.  nthreads<=0 uses the OpenMP default. */
int ptalm_ref_alm_from_points(const double *theta, const double *phi, const double *w,
                              int64_t n, int lmax, double *alm, int nthreads);

/* Same sum, computed entirely in long double with no exponent tracking (the
 * x87 exponent range holds every seed that can matter up to lmax ~ 3e4).  Used
 * to check the FP64 variant's exponent bookkeeping and rounding.  With
 * fp64_trig != 0 the inputs x = cos(theta), s = sin(theta) are first rounded
 * to double exactly as the FP64 variant rounds them, which isolates the error
 * of the recurrence from the conditioning of P_l^m in x near the poles. */
int ptalm_ref_alm_from_points_ld(const double *theta, const double *phi, const double *w,
                                 int64_t n, int lmax, double *alm, int nthreads, int fp64_trig);

/* Selected coefficients a_{ls[k], ms[k]}, k<count, over all n points, written
 * to out[2k], out[2k+1].  Points are summed in fixed chunks of 65536 whose
 * partial sums are added in chunk order, so the result does not depend on
 * nthreads.  Cost per entry: n*(l-m+1) recurrence steps. */
int ptalm_ref_alm_entries(const double *theta, const double *phi, const double *w,
                          int64_t n, int count, const int *ls, const int *ms,
                          double *out, int nthreads);

/* T = (lmax+1)(lmax+2)/2, the number of stored (l, m) pairs. */
int64_t ptalm_ref_alm_size(int lmax);

/* Pseudo-spectrum C_l = (2l+1)^-1 sum_{m=-l..l} |a_lm|^2 (eq. pseudoCl), with the
 * m<0 half from a_{l,-m} = (-1)^m conj(a_lm) (Sec. 2.2). */
int ptalm_ref_cl_from_alm(const double *alm, int lmax, double *cl);

/* Cross spectrum C^AB_l = (2l+1)^-1 sum_{m=-l..l} Re(a_lm conj(b_lm)). */
int ptalm_ref_cross_cl(const double *alm1, const double *alm2, int lmax, double *cl);

/* Wigner 3j symbol (l1 l2 l3; 0 0 0) (App. B), from its closed form for zero
 * projections evaluated in long double with log-gamma:
 *   (-1)^(L/2) sqrt[(L-2l1)! (L-2l2)! (L-2l3)! / (L+1)!] (L/2)! / [(L/2-l1)! (L/2-l2)! (L/2-l3)!],
 * L = l1+l2+l3; 0 when L is odd or the triangle condition fails. */
double ptalm_ref_threej000(int l1, int l2, int l3);

/* Mode-coupling matrix of eq. chat (Sec. 2.1):
 *   M[l][l'] = (2l'+1)/(4 pi) sum_lambda (2 lambda + 1) (l l' lambda; 0 0 0)^2 W_lambda,
 * for 0 <= l, l' <= lmax, the sum over lambda <= lmax_w (W_lambda, lambda <= lmax_w,
 * given; larger lambda taken as 0).  M is (lmax+1)^2 doubles, row-major in l.
 * 3j values from ptalm_ref_threej000, sums in long double in lambda order;
 * parallel over l.  Returns 0, or -1 on bad arguments. */
int ptalm_ref_coupling_matrix(const double *Wl, int lmax_w, int lmax, double *M, int nthreads);

/* Rows of the same matrix: out[k][l'] = M[rows[k]][l'] for k < nrows, l' <= lmax
 * (for sampled checks at sizes where the full matrix is too slow). */
int ptalm_ref_coupling_rows(const double *Wl, int lmax_w, int lmax, const int *rows, int nrows, double *out,
                            int nthreads);

/* Spin-weighted transform for shear (spin +-2 harmonics, end of Sec. 4),
 * selected coefficients over every point:
 *   out[4k..4k+1] = sum_i w_i (g1_i + i g2_i) _{+2}Y*_{l m}(theta_i, phi_i),
 *   out[4k+2..4k+3] = sum_i w_i (g1_i - i g2_i) _{-2}Y*_{l m}(theta_i, phi_i),
 * (l, m) = (ls[k], ms[k]), 0 <= m <= l, l >= 2; with
 * _sY_lm = (-1)^m sqrt((2l+1)/4pi) d^l_{m,-s}(theta) e^{i m phi} (Wigner d).
 * d from the one-term value at l0 = max(m, 2) by the three-term recurrence in
 * l (FP64, seed exponent carried separately as in the scalar transform), sums
 * in long double.  Returns 0, or -1 on bad arguments. */
int ptalm_ref_spin_entries(const double *theta, const double *phi, const double *w, const double *g1,
                           const double *g2, int64_t n, int count, const int *ls, const int *ms, double *out,
                           int nthreads);

/* The same transform for every coefficient: alm_p2 = _{+2}a_lm, alm_m2 = _{-2}a_lm,
 * healpy order, complex interleaved (2T doubles each; 0 for l < 2).  Parallel
 * over m; per point the two d columns by the recurrence above, sums in long
 * double in point order.  Returns 0, or -1 on bad arguments. */
int ptalm_ref_spin_alm(const double *theta, const double *phi, const double *w, const double *g1,
                       const double *g2, int64_t n, int lmax, double *alm_p2, double *alm_m2, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
