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
constexpr int kCouplingThreads = 512;   // 4 matrix waves + 4 store waves
constexpr size_t kCouplingLds = sizeof(double) * 4 * kCB * kSPitch;

// The blocks of S_p (64 x 64 in (i, j) from (i0, j0) = 64 (ib, jb), one parity p)
// that hold an entry of M, in the order the workgroups take them: decreasing
// d = ib - jb (so decreasing length of the k sum), then increasing jb, the two
// parities in turn.  A block holds one when its first entry has
// l = i0 + j0 + p <= lmax, i.e. 2 jb + d <= L_p = floor((lmax - p) / 64); that is
// floor((L_p - d) / 2) + 1 blocks for each d <= L_p, and
// sum_{e = 0..E} (floor(e / 2) + 1) = floor(E^2 / 4) + E + 1 of them with d >= L_p - E.
__device__ inline int64_t blocks_from(int L, int d) {   // blocks of one parity with d' >= d
    if (d > L) return 0;
    const int64_t E = L - d;
    return E * E / 4 + E + 1;
}

struct CouplingBlock {
    int i0, j0, p;
};

// The unit-th block of that order (0 <= unit < blocks_from(L0, 0) + blocks_from(L1, 0)).
__device__ inline CouplingBlock coupling_block(int64_t unit, int L0, int L1) {
    // the largest d whose predecessors (the blocks with d' > d) number at most unit
    int lo = 0, hi = L0;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blocks_from(L0, mid) + blocks_from(L1, mid) <= unit)
            hi = mid - 1;
        else
            lo = mid;
    }
    const int d = lo;
    const int64_t r = unit - (blocks_from(L0, d + 1) + blocks_from(L1, d + 1));
    const int jb = (int)(r >> 1), p = (int)(r & 1);
    return {(jb + d) * kCB, jb * kCB, p};
}

// One matrix wave's share of block (i0, j0, p): the k steps k = j0 + 4 wave + lk + 16 s
// (lk = lane / 16 picks one of four consecutive k, as the f64 MFMA's K = 4),
// accumulated into the 4 x 4 tiles of 16 x 16 f64 results.  A step's operands
// are windows of five sequences, each of which slides by one entry per step:
//   a(i - k_s) for i = i0 + lr + 16 mt:   al[s - mt],  al[n] = A[i0 + lr - k - 16 n]
//   b(i + k_s + p):                        be[s + mt],  be[n] = B[i0 + lr + k + p + 16 n]
//   a(k_s - j) for j = j0 + lr + 16 nt:   ga[s - nt],  ga[n] = A[k - j0 - lr + 16 n]
//   a(k_s + j + p):                        de[s + nt],  de[n] = A[k + j0 + lr + p + 16 n]
//   (2 lambda + 1) W_lambda:               ta[s],       ta[n] = T[2 k + p + 32 n]
// so a step loads one new entry of each, kDist steps ahead, into rings of kRing
// registers indexed by n mod kRing; the loop is unrolled kRing times so that
// every ring index is a constant.  The tables carry kTabPad zeros on both sides:
// they make the terms with k > i, k < j, k + j + p > lmax or lambda > lmax_w
// vanish without a test, and every index read here (at most kDist steps past a
// wave's last step) stays inside them.
__device__ inline void coupling_mma(const double *__restrict__ A, const double *__restrict__ B,
                                    const double *__restrict__ T, int i0, int j0, int p, int ke, int wave, int lane,
                                    v4d (&acc)[4][4]) {
    constexpr int kDist = 2, kRing = kDist + 4;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = v4d{0.0, 0.0, 0.0, 0.0};
    const int kw = j0 + 4 * wave;   // the wave's first k
    const int nsteps = __builtin_amdgcn_readfirstlane(kw <= ke ? (ke - kw) / 16 + 1 : 0);
    if (nsteps == 0) return;
    const int k = kw + lk;
    const double *pa = A + (i0 + lr - k);
    const double *pb = B + (i0 + lr + k + p);
    const double *pc = A + (k - j0 - lr);
    const double *pd = A + (k + j0 + lr + p);
    const double *pt = T + (2 * k + p);
    double al[kRing], be[kRing], ga[kRing], de[kRing], ta[kRing];
    // al and ga from n = -3, be and de from n = 0, up to what steps 0 .. kDist - 1 use
#pragma unroll
    for (int n = -3; n < kDist; ++n) {
        al[(n + kRing) % kRing] = pa[-16 * n];
        ga[(n + kRing) % kRing] = pc[16 * n];
    }
#pragma unroll
    for (int n = 0; n < kDist + 3; ++n) {
        be[n % kRing] = pb[16 * n];
        de[n % kRing] = pd[16 * n];
    }
#pragma unroll
    for (int n = 0; n < kDist; ++n) ta[n] = pt[32 * n];
    // step s = s0 + r at ring phase r; the pointers stand at step s0, so every offset is a constant
    auto step = [&](int r) {
        const int n = r + kDist;
        al[(r + kDist) % kRing] = pa[-16 * n];
        ga[(r + kDist) % kRing] = pc[16 * n];
        be[(r + kDist + 3) % kRing] = pb[16 * (n + 3)];
        de[(r + kDist + 3) % kRing] = pd[16 * (n + 3)];
        ta[(r + kDist) % kRing] = pt[32 * n];
        double h[4], g[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            h[u] = al[(r - u + kRing) % kRing] * be[(r + u) % kRing] * ta[r];
            g[u] = ga[(r - u + kRing) % kRing] * de[(r + u) % kRing];
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(h[mt], g[nt], acc[mt][nt], 0, 0, 0);
    };
    int s0 = 0;
    for (; s0 + kRing <= nsteps; s0 += kRing) {
#pragma unroll
        for (int r = 0; r < kRing; ++r) step(r);
        pa -= 16 * kRing;
        pc += 16 * kRing;
        pb += 16 * kRing;
        pd += 16 * kRing;
        pt += 32 * kRing;
    }
#pragma unroll
    for (int r = 0; r < kRing - 1; ++r)
        if (s0 + r < nsteps) step(r);
}

// Writes one block of S_p (P0 + P1 in LDS, 64 x 64 in (i, j) from (i0, j0)) to both
// triangles of M, scaled by (2l'+1)/(4 pi) resp. (2l+1)/(4 pi); store wave sw
// takes every fourth row of each.  A row of M meets the block along a diagonal
// of (i, j), so a block writes every other entry of up to 64 x 2 in each row.
// Eight rows are read from LDS before any of them is stored (the empty asm
// statement keeps the compiler from moving the reads under the store
// conditions).  M is written once and not read here: streaming stores keep the
// tables in the caches.
__device__ inline void store_block(const double *__restrict__ P0, const double *__restrict__ P1, int i0, int j0,
                                   int p, int sw, int lane, int lmax, double *__restrict__ M) {
    const int64_t n1 = lmax + 1;
    const int dij = i0 - j0;
    // M[l][l'] (l >= l'): row rs = i + j - i0 - j0 of the block, one lane per i;
    // rs < 64: i - i0 = lane, j - j0 = rs - lane; rs >= 64: i - i0 = rs - 63 + lane, j - j0 = 63 - lane
#pragma unroll 1
    for (int it0 = 0; it0 < kCB / 2; it0 += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int rs = sw + 4 * (it0 + u);
            const int x = rs < kCB ? (kCB + 1) * lane + rs : kSPitch * (rs - (kCB - 1)) + (kCB + 1) * lane + (kCB - 1);
            const int xc = x < kCB * kSPitch ? x : 0;
            v[u] = P0[xc] + P1[xc];
        }
        asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int rs = sw + 4 * (it0 + u);
            const int l = i0 + j0 + rs + p;
            const int lp = rs < kCB ? dij + 2 * lane - rs : dij + rs - 2 * (kCB - 1) + 2 * lane;   // i - j
            const bool in_block = rs < kCB ? lane <= rs : lane <= 2 * (kCB - 1) - rs;
            if (rs < 2 * kCB - 1 && l <= lmax && in_block && lp >= 0)
                __builtin_nontemporal_store((2.0 * lp + 1.0) * kInv4Pi * v[u], M + l * n1 + lp);
        }
    }
    // M[l'][l] (l > l'): row rt = i - j - (i0 - j0) + 63 of the block, one lane per j;
    // rt < 64: j - j0 = 63 - rt + lane, i - i0 = lane; rt >= 64: j - j0 = lane, i - i0 = rt - 63 + lane
#pragma unroll 1
    for (int it0 = 0; it0 < kCB / 2; it0 += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int rt = sw + 4 * (it0 + u);
            const int x = rt < kCB ? kSPitch * lane + (kCB - 1) - rt + lane : kSPitch * (rt - (kCB - 1) + lane) + lane;
            const int xc = x < kCB * kSPitch ? x : 0;
            v[u] = P0[xc] + P1[xc];
        }
        asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int rt = sw + 4 * (it0 + u);
            const int tau = dij - (kCB - 1) + rt;
            const int jj = rt < kCB ? (kCB - 1) - rt + lane : lane;
            const int l = 2 * (j0 + jj) + tau + p;   // i + j + p with i = tau + j
            const bool in_block = rt < kCB ? lane <= rt : lane <= 2 * (kCB - 1) - rt;
            if (rt < 2 * kCB - 1 && tau >= 0 && in_block && l <= lmax && (j0 + jj > 0 || p > 0))
                __builtin_nontemporal_store((2.0 * l + 1.0) * kInv4Pi * v[u], M + tau * n1 + l);
        }
    }
}

// Persistent kernel, one workgroup per CU (its LDS keeps a second one off the
// CU).  Waves 0-3 run the matrix products: each has a SIMD's matrix core to
// itself and takes a quarter of the k steps of the current block.  Waves 4-7
// write the previous block to M meanwhile (at a raised issue priority, as the
// matrix waves would otherwise take nearly every issue slot), so that the
// stores overlap the matrix work instead of following it.  The four partial
// blocks are summed in LDS as (w0 + w2) + (w1 + w3): waves 2 and 3 hand theirs
// to waves 0 and 1 through buffers P0 and P1, which then hold the two sums; two
// such buffer pairs alternate between consecutive blocks.
__global__ __launch_bounds__(kCouplingThreads, 1) void coupling_mfma_kernel(const double *__restrict__ A,
                                                                           const double *__restrict__ B,
                                                                           const double *__restrict__ T, int lmax,
                                                                           int kw0, int kw1,
                                                                           int *__restrict__ counter,
                                                                           double *__restrict__ M) {
    extern __shared__ double Sd[];   // [2 buffer pairs][P0, P1][kCB][kSPitch], kCouplingLds bytes
    __shared__ int64_t unit_s;
    constexpr int kBuf = 2 * kCB * kSPitch;
    const int L0 = lmax / kCB, L1 = lmax >= 1 ? (lmax - 1) / kCB : -1;
    const int64_t units = blocks_from(L0, 0) + blocks_from(L1, 0);
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    // thread 0 takes block numbers one block ahead, so that the atomic's latency
    // is hidden behind the current block
    int next = 0;
    if (threadIdx.x == 0) {
        unit_s = atomicAdd(counter, 1);
        next = atomicAdd(counter, 1);
    }
    lds_barrier();
    int64_t u = unit_s;
    if (wave >= 4) __builtin_amdgcn_s_setprio(3);
    bool pending = false;   // the previous block waits in buffer pair (n - 1) & 1
    CouplingBlock prev{0, 0, 0};
    for (int n = 0;; ++n) {
        if (u >= units && !pending) break;
        const bool have = u < units;
        const CouplingBlock cb = have ? coupling_block(u, L0, L1) : CouplingBlock{0, 0, 0};
        double *Q = Sd + (n & 1) * kBuf;
        if (wave < 4) {
            if (have) {
                const int kw = cb.p ? kw1 : kw0;
                const int ke = min(min(cb.i0 + kCB - 1, lmax - cb.p - cb.j0), kw);
                v4d acc[4][4];
                coupling_mma(A, B, T, cb.i0, cb.j0, cb.p, ke, wave, lane, acc);
                // (16x16 f64 result tile: register r of a lane holds row lane / 16 + 4 r, column lane % 16)
                if (wave >= 2) {
                    double *P = Q + (wave - 2) * (kCB * kSPitch);
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                P[(16 * mt + lk + 4 * r) * kSPitch + 16 * nt + lr] = acc[mt][nt][r];
                }
                lds_barrier();
                if (wave < 2) {
                    double *P = Q + wave * (kCB * kSPitch);
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                double *x = P + (16 * mt + lk + 4 * r) * kSPitch + 16 * nt + lr;
                                *x = acc[mt][nt][r] + *x;
                            }
                }
            } else {
                lds_barrier();
            }
            if (threadIdx.x == 0) {
                unit_s = next;
                next = atomicAdd(counter, 1);
            }
        } else {
            if (pending) {
                const double *P0 = Sd + ((n - 1) & 1) * kBuf;
                store_block(P0, P0 + kCB * kSPitch, prev.i0, prev.j0, prev.p, wave - 4, lane, lmax, M);
            }
            lds_barrier();
        }
        lds_barrier();   // the block's sums are in Q; unit_s holds the next block
        pending = have;
        prev = cb;
        u = unit_s;
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
    const unsigned grid = (unsigned)(cus > 0 ? cus : 1);
    if ((e = hipFuncSetAttribute((const void *)coupling_mfma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kCouplingLds)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(coupling_mfma_kernel, dim3(grid), dim3(kCouplingThreads), kCouplingLds, stream,
                       (const double *)A, (const double *)B, (const double *)T, lmax, kw0, kw1, counter, M);
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
