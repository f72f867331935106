// Mode coupling and bandpowers (Sec. 2.1 eq. chat, eq. mode_coupling, eq. expectation_value; App. B).
//
// M[l][l'] = (2l'+1)/(4 pi) sum_lambda (2 lambda + 1) (l l' lambda; 0 0 0)^2 W_lambda.
//
// Only squares of 3j symbols with even L = l + l' + lambda enter.  With J = L/2
// and a(n) = binom(2n, n) / 4^n the closed form of (l l' lambda; 000)^2 is
//   a(J-l) a(J-l') a(J-lambda) / ((2J+1) a(J)),
// which splits into a factor that depends on (s = l + l', lambda) and one that
// depends on (d = |l - l'|, lambda).  Writing s = 2i + p, d = 2j + p,
// lambda = 2k + p (p the parity of s; J - l' etc. become i - k, k - j, ...):
//   S_p[i][j] = sum_{k=j..i} H_p[i][k] K_p[j][k],
//   H_p[i][k] = a(i-k) b(i+k+p) (2 lambda + 1) W_lambda,   b(J) = 1/((2J+1) a(J)),
//   K_p[j][k] = a(k-j) a(k+j+p),
//   M[l][l'] = (2l'+1)/(4 pi) S_p[i][j],  M[l'][l] = (2l+1)/(4 pi) S_p[i][j],
// so the whole matrix is a triangular FP64 matrix product, run on the matrix
// cores (16x16x4 f64) with operands formed on the fly from three short tables.
// Every factor is positive, so with W >= 0 the sums carry no cancellation;
// a(n) comes from a double-double prefix product and is correct to rounding.
// The paper's own route (its App. B recurrence for the 3j symbols) gives the
// same numbers; the oracle uses the factorial closed form.
//
// Bandpowers: theta_b^l = 1/delta_l on complete bins [lmin + b delta_l, lmin + (b+1) delta_l).
// Mode-decoupled (eq. mode_coupling): C~ = Mbb^-1 theta C^ with Mbb = theta M chi, and the
// window cal M = Mbb^-1 theta M (eq. expectation_value): LU factorisation of Mbb with
// partial pivoting in one workgroup, then forward and back substitution for all
// right-hand sides at once, a panel of columns per workgroup.  Normalised:
// C~' = N theta C^, cal M' = N theta M, 1/N = sum_l (2l+1) W_l / (4 pi).
#include "ptalm_internal.h"

namespace ptalm {

namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;

typedef double v4d __attribute__((ext_vector_type(4)));

struct dd {
    double hi, lo;
};

__device__ inline dd dd_mul(dd x, dd y) {
    const double p = x.hi * y.hi;
    double e = fma(x.hi, y.hi, -p);
    e = fma(x.hi, y.lo, e);
    e = fma(x.lo, y.hi, e);
    const double s = p + e;
    return {s, e - (s - p)};
}

// (2n-1)/(2n) as a double-double (the remainder of the division is exact)
__device__ inline dd odd_even_ratio(int n) {
    const double num = 2.0 * n - 1.0, den = 2.0 * n;
    const double q = num / den;
    return {q, fma(-q, den, num) / den};
}

constexpr int kTabThreads = 1024;
constexpr int kTabPad = 128;   // zeros on either side of each coupling table

// Tables of the contraction, each with kTabPad zeros before and after:
//   A[n] = a(n) = prod_{m=1..n} (2m-1)/(2m)       n in [0, lmax]
//   B[J] = 1 / ((2J+1) a(J))                      J in [0, 2 lmax]
//   T[lambda] = (2 lambda + 1)(W_lambda - shot)   lambda in [0, 2 lmax + 1], 0 beyond lmax_w
// (A, B and T point at entry 0).  a(n) is a prefix product, taken in
// double-double: each thread multiplies its chunk of factors, a Hillis-Steele
// scan over the workgroup gives each chunk its starting value.
__global__ __launch_bounds__(kTabThreads) void coupling_tables_kernel(const double *__restrict__ Wl, int lmax_w,
                                                                      const double *__restrict__ shot, int lmax,
                                                                      double *__restrict__ A, double *__restrict__ B,
                                                                      double *__restrict__ T,
                                                                      int *__restrict__ counter) {
    __shared__ double sh[kTabThreads], sl[kTabThreads];
    const int tid = threadIdx.x;
    if (tid == 0) *counter = 0;   // block counter of coupling_mfma_kernel
    const int N = 2 * lmax + 1;
    for (int e = tid; e < kTabPad; e += kTabThreads) {
        A[e - kTabPad] = 0.0;
        A[lmax + 1 + e] = 0.0;
        B[e - kTabPad] = 0.0;
        B[N + e] = 0.0;
        T[e - kTabPad] = 0.0;
        T[N + 1 + e] = 0.0;
    }
    const int chunk = (N + kTabThreads - 1) / kTabThreads;
    const int n_lo = tid * chunk < N ? tid * chunk : N;
    const int n_hi = n_lo + chunk < N ? n_lo + chunk : N;
    dd P = {1.0, 0.0};
    for (int n = n_lo > 1 ? n_lo : 1; n < n_hi; ++n) P = dd_mul(P, odd_even_ratio(n));
    sh[tid] = P.hi;
    sl[tid] = P.lo;
    __syncthreads();
    for (int off = 1; off < kTabThreads; off <<= 1) {
        dd v = {sh[tid], sl[tid]};
        if (tid >= off) v = dd_mul(dd{sh[tid - off], sl[tid - off]}, v);
        __syncthreads();
        sh[tid] = v.hi;
        sl[tid] = v.lo;
        __syncthreads();
    }
    dd r = tid > 0 ? dd{sh[tid - 1], sl[tid - 1]} : dd{1.0, 0.0};
    for (int n = n_lo; n < n_hi; ++n) {
        if (n >= 1) r = dd_mul(r, odd_even_ratio(n));
        if (n <= lmax) A[n] = r.hi;
        const double c = 2.0 * n + 1.0;
        const double dh = r.hi * c;
        const double dl = fma(r.hi, c, -dh) + r.lo * c;
        const double q = 1.0 / dh;
        B[n] = fma(q, fma(-q, dh, 1.0) - q * dl, q);
    }
    const double sub = shot ? shot[0] : 0.0;
    for (int lam = tid; lam <= N; lam += kTabThreads) T[lam] = lam <= lmax_w ? (2.0 * lam + 1.0) * (Wl[lam] - sub) : 0.0;
}

// Workgroup barrier that orders LDS accesses only: global stores still in
// flight are not waited for.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kCB = 64;   // output block edge in i and in j
constexpr int kSPitch = kCB + 2;
constexpr size_t kCouplingLds = sizeof(double) * 4 * kCB * kSPitch;

// Persistent kernel, one workgroup (4 waves) per CU: its LDS keeps a second
// workgroup off the CU, so each wave has a SIMD's matrix core to itself.  The
// workgroups take 64 x 64 blocks (i0.., j0..) of S_p from a counter, in order of
// decreasing i0 - j0 (decreasing length of the k sum; both parities of a block
// in turn), until none is left.  In a block the k range is split over the
// waves in steps of 4; the four partial blocks go to LDS and are summed in wave
// order while M is written.
__global__ __launch_bounds__(256, 2) void coupling_mfma_kernel(const double *__restrict__ A,
                                                               const double *__restrict__ B,
                                                               const double *__restrict__ T, int lmax, int kw0,
                                                               int kw1, int nblk, int *__restrict__ counter,
                                                               double *__restrict__ M) {
    // 4 partial blocks in dynamic LDS (kCouplingLds bytes): its size keeps a
    // second workgroup off the CU, while the register budget is that of two
    extern __shared__ double Sd[];
    __shared__ int64_t unit_s;
    const int64_t units = (int64_t)nblk * (nblk + 1);   // candidate blocks x 2 parities
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    // thread 0 takes the next block number one block ahead, so that the
    // atomic's latency is hidden behind the current block
    int next = 0;
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    for (;;) {
        if (threadIdx.x == 0) unit_s = next;
        lds_barrier();
        const int64_t u = unit_s;
        if (u >= units) break;
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        const int p = (int)(u & 1);
        const int64_t t = u >> 1;
        int q = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((int64_t)(q + 1) * (q + 2) / 2 <= t) ++q;
        while ((int64_t)q * (q + 1) / 2 > t) --q;
        const int jb = (int)(t - (int64_t)q * (q + 1) / 2);
        const int ib = jb + (nblk - 1 - q);
        const int i0 = ib * kCB, j0 = jb * kCB;
        if (i0 + j0 > lmax - p) {   // no (i, j) with l = i + j + p <= lmax
            lds_barrier();
            continue;
        }
        const int kw = p ? kw1 : kw0;
        const int ke = min(min(i0 + kCB - 1, lmax - p - j0), kw);

        v4d acc[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = v4d{0.0, 0.0, 0.0, 0.0};

        // Operands of one k step (four consecutive k across the lane groups, 64 rows
        // i and 64 columns j).  The tables carry kTabPad zeros on both sides, which
        // make the terms with k > i or k < j vanish without a test, and every index
        // below stays within the padding for k <= ke + 3.  Two register sets
        // alternate so that the loads of one step are in flight during the matrix
        // products of the previous one.
        int k = j0 + 4 * wave + lk;
        const double *pa = A + (i0 + lr - k);       // a(i - k),      i = i0 + 16 mt + lr
        const double *pb = B + (i0 + lr + k + p);   // b(i + k + p)
        const double *pt = T + (2 * k + p);         // (2 lambda + 1) W_lambda
        const double *pc = A + (k - j0 - lr);       // a(k - j),      j = j0 + 16 nt + lr
        const double *pd = A + (k + j0 + lr + p);   // a(k + j + p)
        struct Ops {
            double a[4], b[4], c[4], d[4], t;
        };
        auto load = [&](Ops &o) {
            o.t = pt[0];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                o.a[u] = pa[16 * u];
                o.b[u] = pb[16 * u];
                o.c[u] = pc[-16 * u];
                o.d[u] = pd[16 * u];
            }
            pa -= 16;
            pb += 16;
            pt += 32;
            pc += 16;
            pd += 16;
        };
        auto mma = [&](const Ops &o) {
            double h[4], g[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                h[u] = o.a[u] * o.b[u] * o.t;
                g[u] = o.c[u] * o.d[u];
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(h[mt], g[nt], acc[mt][nt], 0, 0, 0);
        };
        const int kw0_ = j0 + 4 * wave;
        const int nsteps = kw0_ <= ke ? (ke - kw0_) / 16 + 1 : 0;   // this wave's k steps
        Ops X, Y;
        if (nsteps > 0) load(X);
        int st = 0;
        for (; st + 2 <= nsteps; st += 2) {
            load(Y);
            mma(X);
            if (st + 2 < nsteps) load(X);
            mma(Y);
        }
        if (st < nsteps) mma(X);

        // partial blocks to LDS (16x16 f64 result: register r of a lane holds row
        // lane / 16 + 4 r, column lane % 16)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Sd[(wave * kCB + 16 * mt + lk + 4 * r) * kSPitch + 16 * nt + lr] = acc[mt][nt][r];
        lds_barrier();
        // the block: sum of the four partials in wave order, into partial 0
#pragma unroll
        for (int e = threadIdx.x; e < kCB * kCB; e += 256) {
            double *x = Sd + (e >> 6) * kSPitch + (e & 63);
            constexpr int w = kCB * kSPitch;
            x[0] = ((x[0] + x[w]) + x[2 * w]) + x[3 * w];
        }
        lds_barrier();

        const int64_t n1 = lmax + 1;
        // M is written once and not read here: streaming stores keep the tables in the caches.
        // M[l][l'] (l >= l'): rows sigma = i + j of the block, one lane per i
#pragma unroll 4
        for (int it = 0; it < kCB / 2; ++it) {
            const int rs = wave + 4 * it;
            const int sigma = i0 + j0 + rs;
            const int l = sigma + p;
            const int i = max(i0, sigma - (j0 + kCB - 1)) + lane;
            const int j = sigma - i;
            if (rs < 2 * kCB - 1 && l <= lmax && i <= min(i0 + kCB - 1, sigma - j0) && i >= j) {
                const int lp = i - j;
                const double v = (2.0 * lp + 1.0) * kInv4Pi * Sd[(i - i0) * kSPitch + j - j0];
                __builtin_nontemporal_store(v, M + l * n1 + lp);
            }
        }
        // M[l'][l] (l > l'): rows tau = i - j of the block, one lane per j
#pragma unroll 4
        for (int it = 0; it < kCB / 2; ++it) {
            const int rt = wave + 4 * it;
            const int tau = i0 - j0 - (kCB - 1) + rt;
            const int j = max(j0, i0 - tau) + lane;
            const int i = tau + j;
            const int l = i + j + p;
            if (rt < 2 * kCB - 1 && tau >= 0 && j <= min(j0 + kCB - 1, i0 + kCB - 1 - tau) && l <= lmax &&
                (j > 0 || p > 0)) {
                const double v = (2.0 * l + 1.0) * kInv4Pi * Sd[(i - i0) * kSPitch + j - j0];
                __builtin_nontemporal_store(v, M + tau * n1 + l);
            }
        }
        lds_barrier();   // S and unit_s are reused by the next block
    }
}

// dst[b][c] = scale * (1/delta_l) sum_{l in b} src[l][c] for c < ncols (row-major, ld ncols);
// scale = *scale_ptr, or 1 when NULL
__global__ void bin_rows_kernel(const double *__restrict__ src, int ncols, int lmin, int delta_l, int nb,
                                const double *__restrict__ scale_ptr, double *__restrict__ dst) {
    const double scale = scale_ptr ? scale_ptr[0] : 1.0;
    const int64_t total = (int64_t)nb * ncols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / ncols), c = (int)(e % ncols);
        const int l0 = lmin + b * delta_l;
        double s = 0.0;
        for (int k = 0; k < delta_l; ++k) s += src[(int64_t)(l0 + k) * ncols + c];
        dst[e] = scale * (s / delta_l);
    }
}

// Mbb[b][c] = sum_{l' in bin c} R[b][l'] (R = theta M, nb x n1)
__global__ void binned_coupling_kernel(const double *__restrict__ R, int n1, int lmin, int delta_l, int nb,
                                       double *__restrict__ Mbb) {
    const int64_t total = (int64_t)nb * nb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / nb), c = (int)(e % nb);
        const double *row = R + (int64_t)b * n1 + lmin + c * delta_l;
        double s = 0.0;
        for (int k = 0; k < delta_l; ++k) s += row[k];
        Mbb[e] = s;
    }
}

constexpr int kLuThreads = 1024;
constexpr int kLuLdsMaxNb = 140;   // nb^2 doubles in LDS up to this size

// LU factorisation with partial pivoting (largest |pivot|, lowest row on ties)
// of the nb x nb row-major matrix Ag, in place, in one workgroup: afterwards
// the strict lower triangle holds L (unit diagonal), the upper triangle U, and
// perm[i] is the original row now at row i.  The matrix is worked on in LDS
// when it fits.  Each step: wave 0 finds the pivot, the rows are swapped, and
// every row below scales its multiplier and updates itself (one row per 32
// threads).
template <bool kInLds>
__global__ __launch_bounds__(kLuThreads) void lu_kernel(double *__restrict__ Ag, int nb, int *__restrict__ perm_out) {
    __shared__ double lds[kInLds ? kLuLdsMaxNb * kLuLdsMaxNb : 1];
    __shared__ int perm[1024];
    __shared__ int piv;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *A = kInLds ? lds : Ag;
    if (kInLds)
        for (int e = tid; e < nb * nb; e += kLuThreads) A[e] = Ag[e];
    for (int i = tid; i < nb; i += kLuThreads) perm[i] = i;
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        if (wave == 0) {
            double best = -1.0;
            int bi = nb;
            for (int i = k + lane; i < nb; i += 64) {
                const double v = fabs(A[i * nb + k]);
                if (v > best) {
                    best = v;
                    bi = i;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(best, off);
                const int oi = __shfl_xor(bi, off);
                if (ov > best || (ov == best && oi < bi)) {
                    best = ov;
                    bi = oi;
                }
            }
            if (lane == 0) {
                const int pr = bi < nb ? bi : k;
                piv = pr;
                if (pr != k) {
                    const int t = perm[k];
                    perm[k] = perm[pr];
                    perm[pr] = t;
                }
            }
        }
        __syncthreads();
        const int pr = piv;
        if (pr != k) {
            for (int c = tid; c < nb; c += kLuThreads) {
                const double t = A[k * nb + c];
                A[k * nb + c] = A[pr * nb + c];
                A[pr * nb + c] = t;
            }
            __syncthreads();
        }
        const double inv = 1.0 / A[k * nb + k];
        for (int i = k + 1 + (tid >> 5); i < nb; i += kLuThreads / 32) {
            const double l = A[i * nb + k] * inv;
            for (int c = k + 1 + (tid & 31); c < nb; c += 32) A[i * nb + c] = fma(-l, A[k * nb + c], A[i * nb + c]);
            if ((tid & 31) == 0) A[i * nb + k] = l;
        }
        __syncthreads();
    }
    if (kInLds)
        for (int e = tid; e < nb * nb; e += kLuThreads) Ag[e] = A[e];
    for (int i = tid; i < nb; i += kLuThreads) perm_out[i] = perm[i];
}

constexpr int kSolveThreads = 256;
constexpr int kSolveLds = 20224;   // doubles of LDS per workgroup (factors and/or right-hand sides)

// Columns of the right-hand sides per workgroup of lu_solve_kernel, and whether
// the factors are copied into LDS next to them (when both fit).
inline void solve_shape(int nb, int *cols, bool *lu_in_lds) {
    const int room = kSolveLds - nb * nb;
    *lu_in_lds = room >= 16 * nb;
    const int fit = *lu_in_lds ? room / nb : kSolveLds / nb;
    *cols = fit >= 64 ? 64 : (fit >= 32 ? 32 : 16);
}

// X = U^-1 L^-1 P [C^_b | R] for the columns [col0, col0 + cols) of that
// (nb x (n1 + 1)) right-hand side, held in LDS (nb x cols): forward then back
// substitution, one row of the factors per step.  Column 0 is the binned
// pseudo-spectrum (-> cb), column 1 + l' is column l' of R (-> window).
template <bool kLuInLds>
__global__ __launch_bounds__(kSolveThreads) void lu_solve_kernel(const double *__restrict__ LUg,
                                                                 const int *__restrict__ perm, int nb,
                                                                 const double *__restrict__ R,
                                                                 const double *__restrict__ cl_hat, int lmin,
                                                                 int delta_l, int n1, int cols,
                                                                 double *__restrict__ cb,
                                                                 double *__restrict__ window) {
    __shared__ double lds[kSolveLds];
    const int tid = threadIdx.x;
    const double *LU = LUg;
    double *X = lds;   // nb x cols
    if (kLuInLds) {
        for (int e = tid; e < nb * nb; e += kSolveThreads) lds[e] = LUg[e];
        LU = lds;
        X = lds + nb * nb;
    }
    const int col0 = blockIdx.x * cols;
    const int c = tid % cols, r0 = tid / cols, rstep = kSolveThreads / cols;
    const int gc = col0 + c;
    const bool live = gc <= n1;
    for (int i = r0; i < nb; i += rstep) {
        double v = 0.0;
        if (live) {
            const int src = perm[i];
            if (gc == 0) {
                const int l0 = lmin + src * delta_l;
                double s = 0.0;
                for (int k = 0; k < delta_l; ++k) s += cl_hat[l0 + k];
                v = s / delta_l;
            } else {
                v = R[(int64_t)src * n1 + gc - 1];
            }
        }
        X[i * cols + c] = v;
    }
    __syncthreads();
    for (int k = 0; k < nb - 1; ++k) {   // L y = P b
        const double xk = X[k * cols + c];
        for (int i = k + 1 + r0; i < nb; i += rstep) X[i * cols + c] = fma(-LU[i * nb + k], xk, X[i * cols + c]);
        __syncthreads();
    }
    for (int k = nb - 1; k >= 0; --k) {   // U x = y
        const double xk = X[k * cols + c] / LU[k * nb + k];
        __syncthreads();
        if (r0 == 0) X[k * cols + c] = xk;
        for (int i = r0; i < k; i += rstep) X[i * cols + c] = fma(-LU[i * nb + k], xk, X[i * cols + c]);
        __syncthreads();
    }
    if (!live) return;
    for (int i = r0; i < nb; i += rstep) {
        const double v = X[i * cols + c];
        if (gc == 0) cb[i] = v;
        else if (window) window[(int64_t)i * n1 + gc - 1] = v;
    }
}

// Normalised convention: N = 1 / sum_l (2l+1) W_l / (4 pi) (one workgroup, fixed-order
// tree) into *N_out, and cb[b] = N (theta C^)_b.
__global__ __launch_bounds__(1024) void normalisation_kernel(const double *__restrict__ Wl, int lmax_w,
                                                             const double *__restrict__ cl_hat, int lmin, int delta_l,
                                                             int nb, double *__restrict__ N_out,
                                                             double *__restrict__ cb) {
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
    if (tid == 0) N_out[0] = N;
    for (int b = tid; b < nb; b += blockDim.x) {
        const int l0 = lmin + b * delta_l;
        double c = 0.0;
        for (int k = 0; k < delta_l; ++k) c += cl_hat[l0 + k];
        cb[b] = N * (c / delta_l);
    }
}

// Shot noise, out = scale^2 sum_i w_i^2 / (4 pi) with scale = *alpha or 1, in two
// fixed-order passes: block b sums w_i^2 over its contiguous range into
// partial[b], then one workgroup sums the partials.
constexpr int kShotBlocks = 1024;

__global__ __launch_bounds__(256) void shot_partial_kernel(const double *__restrict__ w, int64_t n,
                                                           double *__restrict__ partial) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    // four independent loads in flight per thread, four accumulators
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t i = lo + tid;
    for (; i + 3 * 256 < hi; i += 4 * 256) {
        const double a = w[i], b = w[i + 256], c = w[i + 512], d = w[i + 768];
        s0 = fma(a, a, s0);
        s1 = fma(b, b, s1);
        s2 = fma(c, c, s2);
        s3 = fma(d, d, s3);
    }
    for (; i < hi; i += 256) s0 = fma(w[i], w[i], s0);
    red[tid] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k) red[tid] += red[tid + k];
        __syncthreads();
    }
    if (tid == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kShotBlocks) void shot_final_kernel(const double *__restrict__ partial,
                                                                 const double *__restrict__ alpha,
                                                                 double *__restrict__ out) {
    __shared__ double red[kShotBlocks];
    const int tid = threadIdx.x;
    red[tid] = partial[tid];
    __syncthreads();
    for (int k = kShotBlocks / 2; k > 0; k >>= 1) {
        if (tid < k) red[tid] += red[tid + k];
        __syncthreads();
    }
    if (tid == 0) {
        const double a = alpha ? *alpha : 1.0;
        out[0] = a * a * red[0] * kInv4Pi;
    }
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

size_t coupling_scratch_doubles(int lmax) {
    const size_t L = (size_t)lmax;
    return (L + 1) + (2 * L + 1) + (2 * L + 2) + 6 * kTabPad + 1;
}

hipError_t launch_coupling(const double *Wl, int lmax_w, const double *shot, double *scratch, int lmax, double *M,
                           hipStream_t stream) {
    double *A = scratch + kTabPad;
    double *B = A + (lmax + 1) + 2 * kTabPad;
    double *T = B + (2 * lmax + 1) + 2 * kTabPad;
    int *counter = (int *)(T + (2 * lmax + 2) + kTabPad);
    hipLaunchKernelGGL(coupling_tables_kernel, dim3(1), dim3(kTabThreads), 0, stream, Wl, lmax_w, shot, lmax, A, B, T,
                       counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    const int lw = lmax_w < 2 * lmax ? lmax_w : 2 * lmax;
    const int kw0 = lw >> 1, kw1 = lw >= 1 ? (lw - 1) >> 1 : -1;
    const int nblk = (lmax + kCB) / kCB;
    const int64_t units = (int64_t)nblk * (nblk + 1);
    const unsigned grid = (unsigned)(units < cus ? units : (cus > 0 ? cus : 1));
    if ((e = hipFuncSetAttribute((const void *)coupling_mfma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kCouplingLds)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(coupling_mfma_kernel, dim3(grid), dim3(256), kCouplingLds, stream, (const double *)A, (const double *)B,
                       (const double *)T, lmax, kw0, kw1, nblk, counter, M);
    return hipGetLastError();
}

size_t bandpower_scratch_doubles(int lmax, int nb) {
    const size_t n1 = (size_t)lmax + 1;
    // R = theta M, Mbb and its factors, the row permutation (ints), N
    return (size_t)nb * n1 + (size_t)nb * nb + ((size_t)nb + 1) / 2 + 1;
}

hipError_t launch_bandpowers(const double *cl_hat, const double *M, const double *Wl, int lmax_w, int lmax, int lmin,
                             int delta_l, int nb, int mode, double *cb, double *window, double *scratch,
                             hipStream_t stream) {
    const int n1 = lmax + 1;
    hipError_t e;
    if (mode == 1) {
        double *N = scratch;
        hipLaunchKernelGGL(normalisation_kernel, dim3(1), dim3(1024), 0, stream, Wl, lmax_w, cl_hat, lmin, delta_l, nb,
                           N, cb);
        if ((e = hipGetLastError()) != hipSuccess || window == nullptr) return e;
        hipLaunchKernelGGL(bin_rows_kernel, dim3(blocks_for((int64_t)nb * n1, 256)), dim3(256), 0, stream, M, n1, lmin,
                           delta_l, nb, N, window);
        return hipGetLastError();
    }
    double *R = scratch;
    double *Mbb = R + (size_t)nb * n1;
    int *perm = (int *)(Mbb + (size_t)nb * nb);
    hipLaunchKernelGGL(bin_rows_kernel, dim3(blocks_for((int64_t)nb * n1, 256)), dim3(256), 0, stream, M, n1, lmin,
                       delta_l, nb, (const double *)nullptr, R);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(binned_coupling_kernel, dim3(blocks_for((int64_t)nb * nb, 256)), dim3(256), 0, stream, R, n1,
                       lmin, delta_l, nb, Mbb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (nb <= kLuLdsMaxNb)
        hipLaunchKernelGGL(lu_kernel<true>, dim3(1), dim3(kLuThreads), 0, stream, Mbb, nb, perm);
    else
        hipLaunchKernelGGL(lu_kernel<false>, dim3(1), dim3(kLuThreads), 0, stream, Mbb, nb, perm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int cols;
    bool lu_lds;
    solve_shape(nb, &cols, &lu_lds);
    const unsigned grid = (unsigned)((n1 + 1 + cols - 1) / cols);
    if (lu_lds)
        hipLaunchKernelGGL(lu_solve_kernel<true>, dim3(grid), dim3(kSolveThreads), 0, stream, Mbb, perm, nb, R, cl_hat,
                           lmin, delta_l, n1, cols, cb, window);
    else
        hipLaunchKernelGGL(lu_solve_kernel<false>, dim3(grid), dim3(kSolveThreads), 0, stream, Mbb, perm, nb, R, cl_hat,
                           lmin, delta_l, n1, cols, cb, window);
    return hipGetLastError();
}

size_t shot_noise_scratch_doubles() { return kShotBlocks; }

hipError_t launch_shot_noise(const double *w, int64_t n, const double *alpha, double *out, double *partial,
                             hipStream_t stream) {
    hipLaunchKernelGGL(shot_partial_kernel, dim3(kShotBlocks), dim3(256), 0, stream, w, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(shot_final_kernel, dim3(1), dim3(kShotBlocks), 0, stream, (const double *)partial, alpha, out);
    return hipGetLastError();
}

}  // namespace ptalm
