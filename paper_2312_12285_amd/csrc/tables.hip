// Step coefficients and output scales of the split even/odd Legendre recurrence.
//
// For fixed m write l = m + j.  Pbar_l^m(x) = s^m * q_j(x) with q_j a polynomial
// of degree j in x = cos(theta) that is even in x for even j and odd for odd j.
// The three-term recurrence of App. A.1,
//     Pbar_l = a_l x Pbar_{l-1} - b_l Pbar_{l-2},
//     a_l = (2l-1)/sqrt((l-m)(l+m)),  b_l = sqrt((l-m-1)(l+m-1)/((l-m)(l+m))),
// (the printed form with the outer square root multiplied in), splits into
//     even j:  E_j = a_l y O_{j-1} - b_l E_{j-2}      (q_j = E_j,    y = x^2)
//     odd  j:  O_j = a_l E_{j-1}   - b_l O_{j-2}      (q_j = x O_j)
// Rescaling E_j = e_j Ehat_j, O_j = o_j Ohat_j with e_j = b_l e_{j-2},
// o_j = b_l o_{j-2} makes the second coefficient 1:
//     even j:  Ehat_j = G_j y Ohat_{j-1} - Ehat_{j-2},   G_j = a_l o_{j-1} / e_j
//     odd  j:  Ohat_j = A_j Ehat_{j-1}   - Ohat_{j-2},   A_j = a_l e_{j-1} / o_j
// so an odd step is one FMA and an even step one multiply and one FMA.  The
// start is Ehat_0 = 1 with e_0 = (-1)^m c_m (the sectoral value of App. A.1
// without s^m, c_m = prod_{k<=m} sqrt(1-1/(2k))) and Ohat_1 = 1 with
// o_1 = sqrt(2m+1) e_0 (the second start value of App. A.1).
//
// coef[segment(m) + j] holds G_j (even j >= 2) or A_j (odd j >= 3); entry 0 is 0
// and entry 1 is 1 so that the kernels can run the general step from the
// initial state (Ehat, Ohat) = (-1, 0).  Entries past lmax - m are 0.
// sigma[index(l, m)] = sqrt((2l+1)/4pi) * (e_j or o_j): the factor that turns
// the accumulated sums over points of w s^m e^{-im phi} Ehat_j (even j) or
// w s^m e^{-im phi} x Ohat_j (odd j) into a_lm (Sec. 2.2 normalisation).
//
// Because G_j and A_j are formed from the same rounded e, o that sigma uses,
// the recurrence the kernels effectively run on e_j Ehat_j, o_j Ohat_j has
// coefficients a_l(1+d1), b_l(1+d2) with |d| of a few ulp: the rounding of the
// running products does not accumulate along l.
#include "ptalm_internal.h"

namespace ptalm {

__global__ void tables_kernel(int lmax, double *coef, float *coef32, double *sigma) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m > lmax) return;
    const double inv4pi = 0.25 / 3.14159265358979323846;
    // c_m by the sectoral recurrence
    double cm = 1.0;
    for (int k = 1; k <= m; ++k) cm *= sqrt(1.0 - 1.0 / (2.0 * k));
    double *seg = coef + coef_segment(lmax, m);
    float *seg32 = coef32 + coef_segment(lmax, m);
    const int jmax = lmax - m;
    const int64_t col = column_start(lmax, m);

    double e_last = (m & 1) ? -cm : cm;  // e_0
    double o_last = 0.0;
    seg[0] = 0.0;
    sigma[col] = sqrt((2.0 * m + 1.0) * inv4pi) * e_last;
    if (jmax >= 1) {
        o_last = sqrt(2.0 * m + 1.0) * e_last;  // o_1
        seg[1] = 1.0;
        sigma[col + 1] = sqrt((2.0 * m + 3.0) * inv4pi) * o_last;
    }
    for (int j = 2; j <= jmax; ++j) {
        const int l = m + j;
        const double lm = (double)(l - m), lp = (double)(l + m);
        const double a = (2.0 * l - 1.0) / sqrt(lm * lp);
        const double b = sqrt(((lm - 1.0) * (lp - 1.0)) / (lm * lp));
        double c, scale;
        if ((j & 1) == 0) {
            const double e = b * e_last;
            c = a * o_last / e;
            e_last = e;
            scale = e;
        } else {
            const double o = b * o_last;
            c = a * e_last / o;
            o_last = o;
            scale = o;
        }
        seg[j] = c;
        sigma[col + j] = sqrt((2.0 * l + 1.0) * inv4pi) * scale;
    }
    for (int j = jmax + 1; j <= jmax + kCoefPad; ++j) seg[j] = 0.0;
    for (int j = 0; j <= jmax + kCoefPad; ++j) seg32[j] = (float)seg[j];
}

hipError_t build_tables(int lmax, Tables *t, hipStream_t stream) {
    const int64_t nc = coef_table_size(lmax);
    const int64_t ns = tri_size(lmax);
    hipError_t e;
    if ((e = hipMalloc(&t->coef, sizeof(double) * nc)) != hipSuccess) return e;
    if ((e = hipMalloc(&t->coef32, sizeof(float) * nc)) != hipSuccess) return e;
    if ((e = hipMalloc(&t->sigma, sizeof(double) * ns)) != hipSuccess) return e;
    const int threads = 64;
    const int blocks = (lmax + 1 + threads - 1) / threads;
    hipLaunchKernelGGL(tables_kernel, dim3(blocks), dim3(threads), 0, stream, lmax, t->coef, t->coef32, t->sigma);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    t->lmax = lmax;
    return hipSuccess;
}

}  // namespace ptalm
