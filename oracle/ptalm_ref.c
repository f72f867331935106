/*
 * ptalm_ref.c -- CPU oracle of the direct point-to-harmonic transform
 * (Baleato Lizancos & White, "Harmonic analysis of discrete tracers of
 * large-scale structure", arXiv:2312.12285).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow and written to be checked by eye
 * against the paper.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may call it.  It shares nothing with the GPU library.
 *
 * What it computes (eq. alm_def, Sec. 2.2):
 *     a_lm = sum_i w_i Y*_lm(theta_i, phi_i),   0 <= m <= l <= lmax,
 *     Y_lm = sqrt((2l+1)/4pi) Pbar_l^m(cos theta) e^{i m phi}          (App. A.1)
 * with Pbar_l^m from the recurrences of App. A.1:
 *     Pbar_0^0 = 1,  Pbar_m^m = -sqrt(1-x^2) sqrt(1-1/(2m)) Pbar_{m-1}^{m-1},
 *     Pbar_{m+1}^m = sqrt(2m+1) x Pbar_m^m,
 *     Pbar_l^m = sqrt((l-m)/(l+m)) [ (2l-1)/(l-m) x Pbar_{l-1}^m
 *                 - sqrt((l-m-1)/(l+m-1)) (l+m-1)/(l-m) Pbar_{l-2}^m ].
 *
 * Readings where the paper is silent:
 *  - sqrt(1-x^2) is taken as sin(theta) computed from theta: the printed form
 *    loses all relative accuracy near the poles.
 *  - The sectoral recurrence, unrolled, is Pbar_m^m = (-1)^m c_m s^m with
 *    c_m = prod_{k=1..m} sqrt(1-1/(2k)).  s^m underflows FP64 for points near
 *    the poles at large m while the later Pbar_l^m grow back to O(1), so the
 *    FP64 variant carries the seed as a mantissa and a separate integer binary
 *    exponent until the value re-enters the normal range.  Values that stay
 *    below 2^-900 are treated as zero: a term w*Pbar with |Pbar| <= 1 that small
 *    cannot change an FP64 sum.
 *  - The phase e^{-i m phi} is evaluated directly with long-double cosl/sinl.
 */
#include "ptalm_ref.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define PI_L 3.141592653589793238462643383279502884L

static int64_t tri_size(int lmax) { return (int64_t)(lmax + 1) * (lmax + 2) / 2; }

/* healpy order: all l for m = 0, then all l for m = 1, ... */
static int64_t hp_index(int lmax, int l, int m) { return (int64_t)m * (2 * lmax + 1 - m) / 2 + l; }

/* c_m = prod_{k=1..m} sqrt(1 - 1/(2k)): the sectoral recurrence of App. A.1
 * without its sin(theta) factor, built by that recurrence. */
static void sectoral_constants(int lmax, double *c)
{
    c[0] = 1.0;
    for (int m = 1; m <= lmax; ++m) c[m] = c[m - 1] * sqrt(1.0 - 1.0 / (2.0 * m));
}

static void sectoral_constants_ld(int lmax, long double *c)
{
    c[0] = 1.0L;
    for (int m = 1; m <= lmax; ++m) c[m] = c[m - 1] * sqrtl(1.0L - 1.0L / (2.0L * m));
}

/* s^m as f * 2^e with f in [0.5, 1) (or f = 0), by binary powering; the
 * exponent lives in a 64-bit integer so nothing underflows. */
static void pow_with_exponent(double s, int m, double *f_out, long *e_out)
{
    if (m == 0) { *f_out = 1.0; *e_out = 0; return; }
    if (s == 0.0) { *f_out = 0.0; *e_out = 0; return; }
    int t;
    double bf = frexp(s, &t);
    long be = t;
    double rf = 1.0;
    long re = 0;
    while (m) {
        if (m & 1) {
            rf = frexp(rf * bf, &t);
            re += be + t;
        }
        m >>= 1;
        if (m) {
            bf = frexp(bf * bf, &t);
            be = 2 * be + t;
        }
    }
    *f_out = rf;
    *e_out = re;
}

/* The two coefficients of the l-recurrence of App. A.1, written as printed:
 *   Pbar_l = A_l x Pbar_{l-1} - B_l Pbar_{l-2},  for l >= m+2,
 *   A_l = sqrt((l-m)/(l+m)) (2l-1)/(l-m),
 *   B_l = sqrt((l-m)/(l+m)) sqrt((l-m-1)/(l+m-1)) (l+m-1)/(l-m).
 * Stored at index j = l - m (entries 0 and 1 unused). */
static void lrec_coefficients(int m, int lmax, double *A, double *B)
{
    for (int l = m + 2; l <= lmax; ++l) {
        double lm = (double)(l - m), lp = (double)(l + m);
        double outer = sqrt(lm / lp);
        A[l - m] = outer * ((2.0 * l - 1.0) / lm);
        B[l - m] = outer * sqrt((lm - 1.0) / (lp - 1.0)) * ((lp - 1.0) / lm);
    }
}

static void lrec_coefficients_ld(int m, int lmax, long double *A, long double *B)
{
    for (int l = m + 2; l <= lmax; ++l) {
        long double lm = (long double)(l - m), lp = (long double)(l + m);
        long double outer = sqrtl(lm / lp);
        A[l - m] = outer * ((2.0L * l - 1.0L) / lm);
        B[l - m] = outer * sqrtl((lm - 1.0L) / (lp - 1.0L)) * ((lp - 1.0L) / lm);
    }
}

/* Pbar_{m+j}^m(x) for j = 0 .. lmax-m at one point, written to p[j] (FP64).
 * While the seed is below 2^-900 the values are carried as p * 2^e with one
 * shared integer exponent e < 0; they are rescaled by 2^-600 when
 * they grow past 2^600 and converted to plain doubles once above 2^-900.
 * Until then the written value is 0. */
static void pbar_column(double x, double s, int m, int lmax, double cm,
                        const double *A, const double *B, double *p)
{
    double f;
    long e;
    pow_with_exponent(s, m, &f, &e);
    f *= cm;
    if (m & 1) f = -f;
    if (e > -900) {          /* seed already in the normal range: plain doubles */
        f = ldexp(f, (int)e);
        e = 0;
    }

    double prev2 = 0.0, prev1 = 0.0;  /* Pbar_{l-2}, Pbar_{l-1}, scaled by 2^-e */
    const double a1 = sqrt(2.0 * m + 1.0);
    for (int j = 0; j <= lmax - m; ++j) {
        double v;
        if (j == 0) v = f;                               /* Pbar_m^m */
        else if (j == 1) v = a1 * x * prev1;             /* Pbar_{m+1}^m */
        else v = A[j] * x * prev1 - B[j] * prev2;        /* three-term step */
        if (e < 0) {
            if (fabs(v) > 0x1p600) {
                v *= 0x1p-600;
                prev1 *= 0x1p-600;
                e += 600;
            }
            int ve;
            frexp(v, &ve);
            if (v != 0.0 && (long)ve + e > -900) {
                v = ldexp(v, (int)e);
                prev1 = ldexp(prev1, (int)e);
                e = 0;
            }
        }
        p[j] = (e == 0) ? v : 0.0;
        prev2 = prev1;
        prev1 = v;
    }
}

/* Same column in long double, seed by powl, no exponent tracking. */
static void pbar_column_ld(long double x, long double s, int m, int lmax, long double cm,
                           const long double *A, const long double *B, long double *p)
{
    long double v, prev2 = 0.0L, prev1 = 0.0L;
    const long double a1 = sqrtl(2.0L * m + 1.0L);
    for (int j = 0; j <= lmax - m; ++j) {
        if (j == 0) {
            v = cm * powl(s, (long double)m);
            if (m & 1) v = -v;
        } else if (j == 1) {
            v = a1 * x * prev1;
        } else {
            v = A[j] * x * prev1 - B[j] * prev2;
        }
        p[j] = v;
        prev2 = prev1;
        prev1 = v;
    }
}

static int check_args(const double *theta, const double *phi, const double *w, int64_t n, int lmax,
                      const void *out)
{
    if (n < 0 || lmax < 0 || out == NULL) return -1;
    if (n > 0 && (theta == NULL || phi == NULL || w == NULL)) return -1;
    return 0;
}

int ptalm_ref_alm_from_points(const double *theta, const double *phi, const double *w,
                              int64_t n, int lmax, double *alm, int nthreads)
{
    if (check_args(theta, phi, w, n, lmax, alm)) return -1;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    double *c = malloc(sizeof(double) * (lmax + 1));
    double *xs = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *ss = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!c || !xs || !ss) { free(c); free(xs); free(ss); return -1; }
    sectoral_constants(lmax, c);
    for (int64_t i = 0; i < n; ++i) { xs[i] = cos(theta[i]); ss[i] = sin(theta[i]); }

#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int m = 0; m <= lmax; ++m) {
        const int L = lmax - m + 1;
        double *A = malloc(sizeof(double) * (L + 2));
        double *B = malloc(sizeof(double) * (L + 2));
        double *p = malloc(sizeof(double) * L);
        long double *acc = calloc((size_t)2 * L, sizeof(long double));
        lrec_coefficients(m, lmax, A, B);
        for (int64_t i = 0; i < n; ++i) {
            long double ang = (long double)m * (long double)phi[i];
            long double wr = (long double)w[i] * cosl(ang);
            long double wi = -(long double)w[i] * sinl(ang);
            pbar_column(xs[i], ss[i], m, lmax, c[m], A, B, p);
            for (int j = 0; j < L; ++j) {
                if (p[j] == 0.0) continue;
                acc[2 * j] += (long double)p[j] * wr;
                acc[2 * j + 1] += (long double)p[j] * wi;
            }
        }
        for (int j = 0; j < L; ++j) {
            int l = m + j;
            long double norm = sqrtl((2.0L * l + 1.0L) / (4.0L * PI_L));
            int64_t k = hp_index(lmax, l, m);
            alm[2 * k] = (double)(norm * acc[2 * j]);
            alm[2 * k + 1] = (m == 0) ? 0.0 : (double)(norm * acc[2 * j + 1]);
        }
        free(A); free(B); free(p); free(acc);
    }
    free(c); free(xs); free(ss);
    return 0;
}

int ptalm_ref_alm_from_points_ld(const double *theta, const double *phi, const double *w,
                                 int64_t n, int lmax, double *alm, int nthreads, int fp64_trig)
{
    if (check_args(theta, phi, w, n, lmax, alm)) return -1;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    long double *c = malloc(sizeof(long double) * (lmax + 1));
    if (!c) return -1;
    sectoral_constants_ld(lmax, c);

#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int m = 0; m <= lmax; ++m) {
        const int L = lmax - m + 1;
        long double *A = malloc(sizeof(long double) * (L + 2));
        long double *B = malloc(sizeof(long double) * (L + 2));
        long double *p = malloc(sizeof(long double) * L);
        long double *acc = calloc((size_t)2 * L, sizeof(long double));
        lrec_coefficients_ld(m, lmax, A, B);
        for (int64_t i = 0; i < n; ++i) {
            long double th = (long double)theta[i];
            long double x = fp64_trig ? (long double)cos(theta[i]) : cosl(th);
            long double s = fp64_trig ? (long double)sin(theta[i]) : sinl(th);
            long double ang = (long double)m * (long double)phi[i];
            long double wr = (long double)w[i] * cosl(ang);
            long double wi = -(long double)w[i] * sinl(ang);
            pbar_column_ld(x, s, m, lmax, c[m], A, B, p);
            for (int j = 0; j < L; ++j) {
                acc[2 * j] += p[j] * wr;
                acc[2 * j + 1] += p[j] * wi;
            }
        }
        for (int j = 0; j < L; ++j) {
            int l = m + j;
            long double norm = sqrtl((2.0L * l + 1.0L) / (4.0L * PI_L));
            int64_t k = hp_index(lmax, l, m);
            alm[2 * k] = (double)(norm * acc[2 * j]);
            alm[2 * k + 1] = (m == 0) ? 0.0 : (double)(norm * acc[2 * j + 1]);
        }
        free(A); free(B); free(p); free(acc);
    }
    free(c);
    return 0;
}

#define ENTRY_CHUNK 65536

int ptalm_ref_alm_entries(const double *theta, const double *phi, const double *w,
                          int64_t n, int count, const int *ls, const int *ms,
                          double *out, int nthreads)
{
    if (n < 0 || count < 0 || out == NULL || (count > 0 && (ls == NULL || ms == NULL))) return -1;
    if (n > 0 && (theta == NULL || phi == NULL || w == NULL)) return -1;
    int lmax_all = 0;
    for (int k = 0; k < count; ++k) {
        if (ms[k] < 0 || ls[k] < ms[k]) return -1;
        if (ls[k] > lmax_all) lmax_all = ls[k];
    }
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    double *c = malloc(sizeof(double) * (lmax_all + 1));
    if (!c) return -1;
    sectoral_constants(lmax_all, c);
    const int64_t nchunk = (n + ENTRY_CHUNK - 1) / ENTRY_CHUNK;
    long double *part = malloc(sizeof(long double) * 2 * (size_t)(nchunk > 0 ? nchunk : 1));
    double *A = malloc(sizeof(double) * (lmax_all + 3));
    double *B = malloc(sizeof(double) * (lmax_all + 3));
    if (!part || !A || !B) { free(c); free(part); free(A); free(B); return -1; }

    for (int k = 0; k < count; ++k) {
        const int l = ls[k], m = ms[k];
        lrec_coefficients(m, l, A, B);
#pragma omp parallel num_threads(nthreads)
        {
            double *p = malloc(sizeof(double) * (l - m + 1));
#pragma omp for schedule(dynamic, 1)
            for (int64_t ch = 0; ch < nchunk; ++ch) {
                long double sr = 0.0L, si = 0.0L;
                int64_t i1 = (ch + 1) * ENTRY_CHUNK;
                if (i1 > n) i1 = n;
                for (int64_t i = ch * ENTRY_CHUNK; i < i1; ++i) {
                    pbar_column(cos(theta[i]), sin(theta[i]), m, l, c[m], A, B, p);
                    double v = p[l - m];
                    if (v == 0.0) continue;
                    long double ang = (long double)m * (long double)phi[i];
                    sr += (long double)v * (long double)w[i] * cosl(ang);
                    si -= (long double)v * (long double)w[i] * sinl(ang);
                }
                part[2 * ch] = sr;
                part[2 * ch + 1] = si;
            }
            free(p);
        }
        long double sr = 0.0L, si = 0.0L;
        for (int64_t ch = 0; ch < nchunk; ++ch) { sr += part[2 * ch]; si += part[2 * ch + 1]; }
        long double norm = sqrtl((2.0L * l + 1.0L) / (4.0L * PI_L));
        out[2 * k] = (double)(norm * sr);
        out[2 * k + 1] = (m == 0) ? 0.0 : (double)(norm * si);
    }
    free(c); free(part); free(A); free(B);
    return 0;
}

int ptalm_ref_cl_from_alm(const double *alm, int lmax, double *cl)
{
    if (alm == NULL || cl == NULL || lmax < 0) return -1;
    for (int l = 0; l <= lmax; ++l) {
        long double s = 0.0L;
        for (int m = 0; m <= l; ++m) {
            int64_t k = hp_index(lmax, l, m);
            long double re = alm[2 * k], im = alm[2 * k + 1];
            long double sq = re * re + im * im;
            s += (m == 0) ? sq : 2.0L * sq;   /* m and -m have equal modulus */
        }
        cl[l] = (double)(s / (2.0L * l + 1.0L));
    }
    return 0;
}

int ptalm_ref_cross_cl(const double *alm1, const double *alm2, int lmax, double *cl)
{
    if (alm1 == NULL || alm2 == NULL || cl == NULL || lmax < 0) return -1;
    for (int l = 0; l <= lmax; ++l) {
        long double s = 0.0L;
        for (int m = 0; m <= l; ++m) {
            int64_t k = hp_index(lmax, l, m);
            long double re = (long double)alm1[2 * k] * alm2[2 * k] + (long double)alm1[2 * k + 1] * alm2[2 * k + 1];
            s += (m == 0) ? re : 2.0L * re;
        }
        cl[l] = (double)(s / (2.0L * l + 1.0L));
    }
    return 0;
}

/* keep tri_size referenced for callers that size buffers from the header's formula */
int64_t ptalm_ref_alm_size(int lmax) { return lmax < 0 ? 0 : tri_size(lmax); }

/* ---------------------------------------------------------------------------
 * Mode coupling (Sec. 2.1 eq. chat) and the 3j symbols it needs (App. B).
 * ------------------------------------------------------------------------- */

static long double lfact(int k) { return lgammal((long double)k + 1.0L); }

double ptalm_ref_threej000(int l1, int l2, int l3)
{
    if (l1 < 0 || l2 < 0 || l3 < 0) return 0.0;
    const int L = l1 + l2 + l3;
    if (L & 1) return 0.0;
    if (l1 > l2 + l3 || l2 > l1 + l3 || l3 > l1 + l2) return 0.0;
    const int h = L / 2;
    const long double lg = 0.5L * (lfact(L - 2 * l1) + lfact(L - 2 * l2) + lfact(L - 2 * l3) - lfact(L + 1))
                         + lfact(h) - lfact(h - l1) - lfact(h - l2) - lfact(h - l3);
    const long double v = expl(lg);
    return (double)((h & 1) ? -v : v);
}

static double coupling_entry(const double *Wl, int lmax_w, int l, int lp)
{
    const long double inv4pi = 1.0L / (4.0L * 3.14159265358979323846264338327950288L);
    long double sum = 0.0L;
    const int lo = l > lp ? l - lp : lp - l;
    const int hi = l + lp < lmax_w ? l + lp : lmax_w;
    for (int lam = lo; lam <= hi; lam += 2) {
        const long double t = (long double)ptalm_ref_threej000(l, lp, lam);
        sum += (2.0L * lam + 1.0L) * t * t * (long double)Wl[lam];
    }
    return (double)((2.0L * lp + 1.0L) * inv4pi * sum);
}

int ptalm_ref_coupling_matrix(const double *Wl, int lmax_w, int lmax, double *M, int nthreads)
{
    if (Wl == NULL || M == NULL || lmax < 0 || lmax_w < 0) return -1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
    for (int l = 0; l <= lmax; ++l)
        for (int lp = 0; lp <= lmax; ++lp) M[(int64_t)l * (lmax + 1) + lp] = coupling_entry(Wl, lmax_w, l, lp);
    return 0;
}

int ptalm_ref_coupling_rows(const double *Wl, int lmax_w, int lmax, const int *rows, int nrows, double *out,
                            int nthreads)
{
    if (Wl == NULL || rows == NULL || out == NULL || lmax < 0 || lmax_w < 0 || nrows < 0) return -1;
    for (int k = 0; k < nrows; ++k)
        if (rows[k] < 0 || rows[k] > lmax) return -1;
#pragma omp parallel for collapse(2) schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
    for (int k = 0; k < nrows; ++k)
        for (int lp = 0; lp <= lmax; ++lp) out[(int64_t)k * (lmax + 1) + lp] = coupling_entry(Wl, lmax_w, rows[k], lp);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Spin-weighted transform for shear (spin +-2 harmonics, end of Sec. 4).
 * _sY_lm(theta, phi) = (-1)^m sqrt((2l+1)/4pi) d^l_{m,-s}(theta) e^{i m phi}
 * (Goldberg et al. 1967).  For fixed (m, mp) the Wigner d obey
 *   l sqrt(((l+1)^2-m^2)((l+1)^2-mp^2)) d^{l+1}
 *     = (2l+1) (l(l+1) cos theta - m mp) d^l - (l+1) sqrt((l^2-m^2)(l^2-mp^2)) d^{l-1},
 * started at l0 = max(m, |mp|), where the Wigner sum has one term:
 *   l0 = m:   d^m_{m,mp} = sqrt(C(2m, m+mp)) cos^{m+mp}(theta/2) sin^{m-mp}(theta/2);
 *   l0 = 2 > m (mp = +-2, m = 0, 1): from the same sum,
 *     d^2_{0,+-2} = sqrt(6) c^2 s^2,  d^2_{1,-2} = 2 c s^3,  d^2_{1,2} = -2 c^3 s.
 * ------------------------------------------------------------------------- */

/* sqrt(C(2m, m+2)) as mantissa * 2^exponent (running product, renormalised). */
static void spin_seed_constant(int m, long double *f_out, long *e_out)
{
    long double f = 1.0L;
    long e = 0;
    for (int k = 1; k <= m + 2; ++k) {      /* C(2m, m+2) = prod_k (m-2+k)/k */
        int t;
        f = frexpl(f * ((long double)(m - 2 + k) / (long double)k), &t);
        e += t;
    }
    if (e & 1) { f *= 2.0L; e -= 1; }
    *f_out = sqrtl(f);
    *e_out = e / 2;
}

/* d^l_{m,mp}(theta) for mp = +-2 and l0 <= l <= lend (0 while below 2^-900):
 * written to d[l] when d != NULL; the value at lend is returned. */
static double spin_column(double c, double s, double x, int m, int mp, int lend, long double kf, long ke,
                          const double *A, const double *B, const double *C, double *d)
{
    const int l0 = m > 2 ? m : 2;
    double f;
    long e = 0;
    if (m >= 2) {
        double fc, fs;
        long ec, es;
        pow_with_exponent(c, m + mp, &fc, &ec);
        pow_with_exponent(s, m - mp, &fs, &es);
        int t;
        f = frexp((double)kf * fc * fs, &t);
        e = ke + ec + es + t;
    } else if (m == 0) {
        f = sqrt(6.0) * c * c * s * s;
    } else {
        f = (mp < 0) ? 2.0 * c * s * s * s : -2.0 * c * c * c * s;
    }
    if (e > -900) { f = ldexp(f, (int)e); e = 0; }
    double prev = 0.0, cur = f;              /* d^{l-1}, d^l scaled by 2^-e */
    if (d) d[l0] = (e == 0) ? cur : 0.0;
    for (int l = l0; l < lend; ++l) {
        double v = (A[l] * x - B[l]) * cur - C[l] * prev;
        if (e < 0) {
            if (fabs(v) > 0x1p600) {
                v *= 0x1p-600;
                cur *= 0x1p-600;
                e += 600;
            }
            int ve;
            frexp(v, &ve);
            if (v != 0.0 && (long)ve + e > -900) {
                v = ldexp(v, (int)e);
                cur = ldexp(cur, (int)e);
                e = 0;
            }
        }
        prev = cur;
        cur = v;
        if (d) d[l + 1] = (e == 0) ? cur : 0.0;
    }
    return (e == 0) ? cur : 0.0;
}

/* A, B, C of the step l -> l+1 for l0 <= l < lend (index l). */
static void spin_coefficients(int m, int mp, int lend, double *A, double *B, double *C)
{
    for (int l = (m > 2 ? m : 2); l < lend; ++l) {
        const double dl = l, l1 = l + 1.0, dm = m, dp = mp;
        const double D = dl * sqrt((l1 * l1 - dm * dm) * (l1 * l1 - dp * dp));
        A[l] = (2.0 * l + 1.0) * dl * l1 / D;
        B[l] = (2.0 * l + 1.0) * dm * dp / D;
        C[l] = l1 * sqrt((dl * dl - dm * dm) * (dl * dl - dp * dp)) / D;
    }
}

int ptalm_ref_spin_entries(const double *theta, const double *phi, const double *w, const double *g1,
                           const double *g2, int64_t n, int count, const int *ls, const int *ms, double *out,
                           int nthreads)
{
    if (n < 0 || count < 0 || out == NULL || (count > 0 && (ls == NULL || ms == NULL))) return -1;
    if (n > 0 && (theta == NULL || phi == NULL || w == NULL || g1 == NULL || g2 == NULL)) return -1;
    int lmax_all = 2;
    for (int k = 0; k < count; ++k) {
        if (ms[k] < 0 || ls[k] < ms[k] || ls[k] < 2) return -1;
        if (ls[k] > lmax_all) lmax_all = ls[k];
    }
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    const int64_t nchunk = (n + ENTRY_CHUNK - 1) / ENTRY_CHUNK;
    long double *part = malloc(sizeof(long double) * 4 * (size_t)(nchunk > 0 ? nchunk : 1));
    double *co = malloc(sizeof(double) * 6 * (size_t)(lmax_all + 1));
    if (!part || !co) { free(part); free(co); return -1; }
    for (int k = 0; k < count; ++k) {
        const int l = ls[k], m = ms[k];
        double *Ap = co, *Bp = co + (lmax_all + 1), *Cp = co + 2 * (lmax_all + 1);   /* mp = -2: s = +2 */
        double *Am = co + 3 * (lmax_all + 1), *Bm = co + 4 * (lmax_all + 1), *Cm = co + 5 * (lmax_all + 1);
        spin_coefficients(m, -2, l, Ap, Bp, Cp);
        spin_coefficients(m, 2, l, Am, Bm, Cm);
        long double kf = 1.0L;
        long ke = 0;
        if (m >= 2) spin_seed_constant(m, &kf, &ke);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
        for (int64_t ch = 0; ch < nchunk; ++ch) {
            long double pr = 0.0L, pi = 0.0L, mr = 0.0L, mi = 0.0L;
            int64_t i1 = (ch + 1) * ENTRY_CHUNK;
            if (i1 > n) i1 = n;
            for (int64_t i = ch * ENTRY_CHUNK; i < i1; ++i) {
                const double c = cos(0.5 * theta[i]), s = sin(0.5 * theta[i]);
                const double x = (c - s) * (c + s);
                const double dp = spin_column(c, s, x, m, -2, l, kf, ke, Ap, Bp, Cp, NULL);
                const double dm = spin_column(c, s, x, m, 2, l, kf, ke, Am, Bm, Cm, NULL);
                if (dp == 0.0 && dm == 0.0) continue;
                const long double ang = (long double)m * (long double)phi[i];
                const long double er = cosl(ang), ei = -sinl(ang);      /* e^{-i m phi} */
                const long double a = g1[i], b = g2[i], ww = w[i];
                /* w (a + i b) d+ e^{-i m phi} and w (a - i b) d- e^{-i m phi} */
                pr += ww * dp * (a * er - b * ei);
                pi += ww * dp * (a * ei + b * er);
                mr += ww * dm * (a * er + b * ei);
                mi += ww * dm * (a * ei - b * er);
            }
            part[4 * ch] = pr;
            part[4 * ch + 1] = pi;
            part[4 * ch + 2] = mr;
            part[4 * ch + 3] = mi;
        }
        long double acc[4] = {0.0L, 0.0L, 0.0L, 0.0L};
        for (int64_t ch = 0; ch < nchunk; ++ch)
            for (int q = 0; q < 4; ++q) acc[q] += part[4 * ch + q];
        long double norm = sqrtl((2.0L * l + 1.0L) / (4.0L * PI_L));
        if (m & 1) norm = -norm;
        for (int q = 0; q < 4; ++q) out[4 * k + q] = (double)(norm * acc[q]);
    }
    free(part);
    free(co);
    return 0;
}

int ptalm_ref_spin_alm(const double *theta, const double *phi, const double *w, const double *g1,
                       const double *g2, int64_t n, int lmax, double *alm_p2, double *alm_m2, int nthreads)
{
    if (check_args(theta, phi, w, n, lmax, alm_p2) || alm_m2 == NULL || (n > 0 && (g1 == NULL || g2 == NULL)))
        return -1;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    memset(alm_p2, 0, sizeof(double) * 2 * (size_t)tri_size(lmax));
    memset(alm_m2, 0, sizeof(double) * 2 * (size_t)tri_size(lmax));
    if (lmax < 2) return 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int m = 0; m <= lmax; ++m) {
        const int l0 = m > 2 ? m : 2;
        double *co = malloc(sizeof(double) * 6 * (size_t)(lmax + 1));
        double *dp = malloc(sizeof(double) * (size_t)(lmax + 1));
        double *dm = malloc(sizeof(double) * (size_t)(lmax + 1));
        long double *acc = calloc((size_t)4 * (lmax + 1), sizeof(long double));
        double *Ap = co, *Bp = co + (lmax + 1), *Cp = co + 2 * (lmax + 1);
        double *Am = co + 3 * (lmax + 1), *Bm = co + 4 * (lmax + 1), *Cm = co + 5 * (lmax + 1);
        spin_coefficients(m, -2, lmax, Ap, Bp, Cp);
        spin_coefficients(m, 2, lmax, Am, Bm, Cm);
        long double kf = 1.0L;
        long ke = 0;
        if (m >= 2) spin_seed_constant(m, &kf, &ke);
        for (int64_t i = 0; i < n; ++i) {
            const double c = cos(0.5 * theta[i]), s = sin(0.5 * theta[i]);
            const double x = (c - s) * (c + s);
            spin_column(c, s, x, m, -2, lmax, kf, ke, Ap, Bp, Cp, dp);
            spin_column(c, s, x, m, 2, lmax, kf, ke, Am, Bm, Cm, dm);
            const long double ang = (long double)m * (long double)phi[i];
            const long double er = cosl(ang), ei = -sinl(ang);
            const long double a = g1[i], b = g2[i], ww = w[i];
            const long double qpr = ww * (a * er - b * ei), qpi = ww * (a * ei + b * er);
            const long double qmr = ww * (a * er + b * ei), qmi = ww * (a * ei - b * er);
            for (int l = l0; l <= lmax; ++l) {
                acc[4 * l] += qpr * dp[l];
                acc[4 * l + 1] += qpi * dp[l];
                acc[4 * l + 2] += qmr * dm[l];
                acc[4 * l + 3] += qmi * dm[l];
            }
        }
        for (int l = l0; l <= lmax; ++l) {
            long double norm = sqrtl((2.0L * l + 1.0L) / (4.0L * PI_L));
            if (m & 1) norm = -norm;
            const int64_t k = hp_index(lmax, l, m);
            alm_p2[2 * k] = (double)(norm * acc[4 * l]);
            alm_p2[2 * k + 1] = (double)(norm * acc[4 * l + 1]);
            alm_m2[2 * k] = (double)(norm * acc[4 * l + 2]);
            alm_m2[2 * k + 1] = (double)(norm * acc[4 * l + 3]);
        }
        free(co); free(dp); free(dm); free(acc);
    }
    return 0;
}
