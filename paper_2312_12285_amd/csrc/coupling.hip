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
#include <map>
#include <mutex>

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

// 1/d for d > 0 to about half an ulp: the hardware reciprocal and one Newton step
// (an IEEE division is several times as many instructions)
__device__ inline double recip(double d) {
    double x = __builtin_amdgcn_rcp(d);
    x = fma(x, fma(-d, x, 1.0), x);
    return fma(x, fma(-d, x, 1.0), x);
}

// (2n-1)/(2n) as a double-double: q plus the exact remainder of num - q den, divided by den
__device__ inline dd odd_even_ratio(int n) {
    const double num = 2.0 * n - 1.0, den = 2.0 * n;
    const double inv = recip(den);
    const double q = num * inv;
    return {q, fma(-q, den, num) * inv};
}

// inclusive product scan of a double-double over the 64 lanes of a wave
__device__ inline dd wave_scan_mul(dd v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double h = __shfl_up(v.hi, off), l = __shfl_up(v.lo, off);
        if (lane >= off) v = dd_mul(dd{h, l}, v);
    }
    return v;
}

constexpr int kTabThreads = 1024;
constexpr int kTabPad = 128;   // zeros on either side of each coupling table

// Tables of the contraction, each with kTabPad zeros before and after:
//   A[n] = a(n) = prod_{m=1..n} (2m-1)/(2m)       n in [0, lmax]
//   B[J] = 1 / ((2J+1) a(J))                      J in [0, 2 lmax]
//   T[lambda] = (2 lambda + 1)(W_lambda - shot)   lambda in [0, 2 lmax + 1], 0 beyond lmax_w
// (A, B and T point at entry 0).  A and B depend on lmax only.  a(n) is a prefix
// product, taken in double-double: each thread multiplies its chunk of factors;
// a scan within each wave (lane shuffles) and one over the 16 wave totals
// (through LDS, one barrier) give each chunk its starting value.
__global__ __launch_bounds__(kTabThreads) void coupling_ab_kernel(int lmax, double *__restrict__ A,
                                                                  double *__restrict__ B) {
    constexpr int kWaves = kTabThreads / 64;
    __shared__ double wh[kWaves], wl[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int N = 2 * lmax + 1;
    for (int e = tid; e < kTabPad; e += kTabThreads) {
        A[e - kTabPad] = 0.0;
        A[lmax + 1 + e] = 0.0;
        B[e - kTabPad] = 0.0;
        B[N + e] = 0.0;
    }
    const int chunk = (N + kTabThreads - 1) / kTabThreads;
    const int n_lo = tid * chunk < N ? tid * chunk : N;
    const int n_hi = n_lo + chunk < N ? n_lo + chunk : N;
    dd P = {1.0, 0.0};
    for (int n = n_lo > 1 ? n_lo : 1; n < n_hi; ++n) P = dd_mul(P, odd_even_ratio(n));
    const dd inc = wave_scan_mul(P, lane);   // product of the chunks of lanes 0..lane of this wave
    if (lane == 63) {
        wh[wave] = inc.hi;
        wl[wave] = inc.lo;
    }
    __syncthreads();
    dd r = {1.0, 0.0};   // product of all chunks before this thread's
    for (int w = 0; w < wave; ++w) r = dd_mul(r, dd{wh[w], wl[w]});
    const dd prev = {__shfl_up(inc.hi, 1), __shfl_up(inc.lo, 1)};
    if (lane > 0) r = dd_mul(r, prev);
    for (int n = n_lo; n < n_hi; ++n) {
        if (n >= 1) r = dd_mul(r, odd_even_ratio(n));
        if (n <= lmax) A[n] = r.hi;
        const double c = 2.0 * n + 1.0;
        const double dh = r.hi * c;
        const double dl = fma(r.hi, c, -dh) + r.lo * c;
        const double q = recip(dh);
        B[n] = fma(q, fma(-q, dh, 1.0) - q * dl, q);
    }
}

// T with its padding, and the unit counter of coupling_mfma_kernel set to 0
__global__ __launch_bounds__(kTabThreads) void coupling_t_kernel(const double *__restrict__ Wl, int lmax_w,
                                                                 const double *__restrict__ shot, int lmax,
                                                                 double *__restrict__ T, int *__restrict__ counter) {
    const int N = 2 * lmax + 1;
    const double sub = shot ? shot[0] : 0.0;
    const int e = blockIdx.x * kTabThreads + threadIdx.x - kTabPad;   // lambda, from -kTabPad
    if (e == -kTabPad) *counter = 0;
    if (e < N + 1 + kTabPad) T[e] = e >= 0 && e <= lmax_w && e <= N ? (2.0 * e + 1.0) * (Wl[e] - sub) : 0.0;
}

// Workgroup barrier that orders LDS accesses only: global stores still in
// flight are not waited for.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kCI = 64;                     // unit edge in i
constexpr int kCJ = 32;                     // unit edge in j
constexpr int kPitch = kCJ + 2;             // LDS row pitch of a partial tile (doubles)
constexpr int kTile = kCI * kPitch;         // one parity's 64 x 32 tile
constexpr int kCouplingThreads = 512;       // 4 matrix waves + 4 store waves
constexpr size_t kCouplingLds = sizeof(double) * 2 * 2 * 2 * kTile;   // [buffer pair][P0, P1][parity]

// Work units: the 64 x 32 blocks (i0, j0) = (64 ib, 64 jb + 32 h) of S_0 and S_1
// together (both parities, h the half of a 64-wide column block) that hold an
// entry of M, in the order the workgroups take them: decreasing d = ib - jb (so
// decreasing length of the k sum), then increasing jb, the two halves in turn.
// A unit holds one when its first entry has l = i0 + j0 <= lmax, i.e.
// 2 jb + d <= L_h = floor((lmax - 32 h) / 64); that is floor((L_h - d) / 2) + 1
// units for each d <= L_h, and sum_{e = 0..E} (floor(e / 2) + 1) =
// floor(E^2 / 4) + E + 1 of them with d >= L_h - E.
__device__ inline int64_t units_from(int L, int d) {   // units of one half with d' >= d
    if (d > L) return 0;
    const int64_t E = L - d;
    return E * E / 4 + E + 1;
}

struct CouplingUnit {
    int i0, j0;
};

// The unit-th unit of that order (0 <= unit < units_from(L0, 0) + units_from(L1, 0)).
__device__ inline CouplingUnit coupling_unit(int64_t unit, int L0, int L1) {
    // the largest d whose predecessors (the units with d' > d) number at most unit
    int lo = 0, hi = L0;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (units_from(L0, mid) + units_from(L1, mid) <= unit)
            hi = mid - 1;
        else
            lo = mid;
    }
    const int d = lo;
    const int64_t r = unit - (units_from(L0, d + 1) + units_from(L1, d + 1));
    const int jb = (int)(r >> 1), h = (int)(r & 1);
    return {(jb + d) * 2 * kCJ, jb * 2 * kCJ + h * kCJ};
}

// two adjacent table entries (p = 0 and p = 1), 8-byte aligned
struct Pair {
    double v[2];
};
__device__ inline Pair ld_pair(const double *p) { return Pair{{p[0], p[1]}}; }

// One matrix wave's share of unit (i0, j0): the k steps k = j0 + 4 wave + lk + 16 s
// (lk = lane / 16 picks one of four consecutive k, as the f64 MFMA's K = 4) for
// both parities, into 2 x 4 x 2 tiles of 16 x 16 f64 results.  A step's operands
// H_p[i][k] = a(i - k) b(i + k + p) and K_p[j][k] T(2k + p) = a(k - j) a(k + j + p) T(2k + p)
// are formed from windows of five sequences, each sliding by one entry per step:
//   a(i - k_s) for i = i0 + lr + 16 mt:   al[s - mt],  al[n] = A[i0 + lr - k - 16 n]
//   b(i + k_s + p):                        be[s + mt],  be[n] = B[i0 + lr + k + 16 n + p]
//   a(k_s - j) for j = j0 + lr + 16 nt:   ga[s - nt],  ga[n] = A[k - j0 - lr + 16 n]
//   a(k_s + j + p):                        de[s + nt],  de[n] = A[k + j0 + lr + 16 n + p]
//   (2 lambda + 1) W_lambda:               ta[s],       ta[n] = T[2 k + 32 n + p]
// (be, de and ta hold both parities, two adjacent table entries), so a step loads
// one new entry of each, one step ahead, into register rings indexed by n mod
// their length (6, 6, 3, 3, 2); the loop is unrolled 6 times so that every ring
// index is a constant.  The tables carry kTabPad zeros on both sides: they make
// the terms with k > i, k < j, k + j + p > lmax or lambda > lmax_w vanish without
// a test, and every index read here (at most a step past the wave's last step)
// stays inside them.
__device__ inline void coupling_mma(const double *__restrict__ A, const double *__restrict__ B,
                                    const double *__restrict__ T, int i0, int j0, int ke, int wave, int lane,
                                    v4d (&acc)[2][4][2]) {
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) acc[p][mt][nt] = v4d{0.0, 0.0, 0.0, 0.0};
    const int kw = j0 + 4 * wave;   // the wave's first k
    const int nsteps = __builtin_amdgcn_readfirstlane(kw <= ke ? (ke - kw) / 16 + 1 : 0);
    if (nsteps == 0) return;
    const int k = kw + lk;
    const double *pa = A + (i0 + lr - k);
    const double *pb = B + (i0 + lr + k);
    const double *pc = A + (k - j0 - lr);
    const double *pd = A + (k + j0 + lr);
    const double *pt = T + 2 * k;
    double al[6], ga[3];
    Pair be[6], de[3], ta[2];
#pragma unroll
    for (int n = -3; n <= 0; ++n) al[(n + 6) % 6] = pa[-16 * n];
#pragma unroll
    for (int n = 0; n <= 3; ++n) be[n] = ld_pair(pb + 16 * n);
#pragma unroll
    for (int n = -1; n <= 0; ++n) ga[(n + 3) % 3] = pc[16 * n];
#pragma unroll
    for (int n = 0; n <= 1; ++n) de[n] = ld_pair(pd + 16 * n);
    ta[0] = ld_pair(pt);
    // step s = s0 + r (r = s mod 6); the pointers stand at step s0, so every offset is a constant
    auto step = [&](int r) {
        al[(r + 1) % 6] = pa[-16 * (r + 1)];
        be[(r + 4) % 6] = ld_pair(pb + 16 * (r + 4));
        ga[(r + 1) % 3] = pc[16 * (r + 1)];
        de[(r + 2) % 3] = ld_pair(pd + 16 * (r + 2));
        ta[(r + 1) % 2] = ld_pair(pt + 32 * (r + 1));
        double h[2][4], g[2][2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) h[p][mt] = al[(r - mt + 6) % 6] * be[(r + mt) % 6].v[p];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) g[p][nt] = ga[(r - nt + 3) % 3] * de[(r + nt) % 3].v[p] * ta[r % 2].v[p];
        }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    acc[p][mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(h[p][mt], g[p][nt], acc[p][mt][nt], 0, 0, 0);
    };
    int s0 = 0;
    for (; s0 + 6 <= nsteps; s0 += 6) {
#pragma unroll
        for (int r = 0; r < 6; ++r) step(r);
        pa -= 16 * 6;
        pb += 16 * 6;
        pc += 16 * 6;
        pd += 16 * 6;
        pt += 32 * 6;
    }
#pragma unroll
    for (int r = 0; r < 5; ++r)
        if (s0 + r < nsteps) step(r);
}

// Writes unit (i0, j0) (the sums P0 + P1 in LDS, one 64 x 32 tile per parity) to
// both triangles of M, scaled by (2l'+1)/(4 pi) resp. (2l+1)/(4 pi); store wave sw
// takes every fourth row of each.  In a row of M the two parities alternate, so
// a row of the unit is one run of up to 64 consecutive entries: one store
// instruction of whole lines.  Eight rows are read from LDS before any of them is
// stored (the empty asm statement keeps the compiler from moving the reads under
// the store conditions).  M is written once and not read here: streaming stores
// keep the tables in the caches.
__device__ inline void store_unit(const double *__restrict__ P0, const double *__restrict__ P1, int i0, int j0,
                                  int sw, int nw, int lane, int lmax, double *__restrict__ M) {
    const int rows = (3 * kCJ + nw - 1) / nw;   // rows per wave in each triangle (the last ones may fall outside)
    const int64_t n1 = lmax + 1;
    const int dij = i0 - j0;
    // M[l][l'] (l >= l'): row sig = l - i0 - j0 in [0, 95]; lane at c = l' - (i0 - j0);
    // p = parity of sig + c, i - i0 = (sig - p + c) / 2, j - j0 = (sig - p - c) / 2
#pragma unroll 1
    for (int it0 = 0; it0 < rows; it0 += 8) {
        double v[8];
        bool ok[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int sig = sw + nw * (it0 + u);
            const int c = max(sig - (kCI - 1), -sig) + lane;
            const int p = (sig + c) & 1;
            const int ii = (sig - p + c) >> 1, jj = (sig - p - c) >> 1;
            ok[u] = ii >= 0 && ii < kCI && jj >= 0 && jj < kCJ && dij + c >= 0 && i0 + j0 + sig <= lmax;
            const int x = ok[u] ? p * kTile + ii * kPitch + jj : 0;
            v[u] = P0[x] + P1[x];
        }
        asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int sig = sw + nw * (it0 + u);
            const int lp = dij + max(sig - (kCI - 1), -sig) + lane;
            if (ok[u]) __builtin_nontemporal_store((2.0 * lp + 1.0) * kInv4Pi * v[u], M + (i0 + j0 + sig) * n1 + lp);
        }
    }
    // M[l'][l] (l > l'): row tau = l' = i - j, t = tau - (i0 - j0) in [-31, 63]; lane at
    // c = l - i0 - j0; p = parity of c + t, i - i0 = (c - p + t) / 2, j - j0 = (c - p - t) / 2
#pragma unroll 1
    for (int it0 = 0; it0 < rows; it0 += 8) {
        double v[8];
        bool ok[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = sw + nw * (it0 + u) - (kCJ - 1);
            const int c = abs(t) + lane;
            const int p = (c + t) & 1;
            const int ii = (c - p + t) >> 1, jj = (c - p - t) >> 1;
            ok[u] = ii >= 0 && ii < kCI && jj >= 0 && jj < kCJ && dij + t >= 0 && i0 + j0 + c <= lmax &&
                    (j0 + jj > 0 || p > 0);
            const int x = ok[u] ? p * kTile + ii * kPitch + jj : 0;
            v[u] = P0[x] + P1[x];
        }
        asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = sw + nw * (it0 + u) - (kCJ - 1);
            const int l = i0 + j0 + abs(t) + lane;
            if (ok[u]) __builtin_nontemporal_store((2.0 * l + 1.0) * kInv4Pi * v[u], M + (dij + t) * n1 + l);
        }
    }
}

// Persistent kernel, one workgroup per CU (its LDS keeps a second one off the
// CU).  Waves 0-3 run the matrix products: each has a SIMD's matrix core to
// itself and takes a quarter of the k steps of the current unit.  Waves 4-7
// write the previous unit to M meanwhile (at a raised issue priority, as the
// matrix waves would otherwise take nearly every issue slot), so that the
// stores overlap the matrix work instead of following it.  The four partial
// results are summed in LDS as (w0 + w2) + (w1 + w3): waves 2 and 3 hand theirs
// to waves 0 and 1 through buffers P0 and P1, which then hold the two sums; two
// such buffer pairs alternate between consecutive units.
__global__ __launch_bounds__(kCouplingThreads, 1) void coupling_mfma_kernel(const double *__restrict__ A,
                                                                           const double *__restrict__ B,
                                                                           const double *__restrict__ T, int lmax,
                                                                           int kw0, int *__restrict__ counter,
                                                                           double *__restrict__ M) {
    extern __shared__ double Sd[];   // [2 buffer pairs][P0, P1][parity][kCI][kPitch], kCouplingLds bytes
    __shared__ int64_t unit_s;
    constexpr int kBuf = 2 * 2 * kTile;
    const int L0 = lmax / (2 * kCJ), L1 = lmax >= kCJ ? (lmax - kCJ) / (2 * kCJ) : -1;
    const int64_t units = units_from(L0, 0) + units_from(L1, 0);
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    // thread 0 takes unit numbers one unit ahead, so that the atomic's latency
    // is hidden behind the current unit
    int next = 0;
    if (threadIdx.x == 0) {
        unit_s = atomicAdd(counter, 1);
        next = atomicAdd(counter, 1);
    }
    lds_barrier();
    int64_t u = unit_s;
    if (wave >= 4) __builtin_amdgcn_s_setprio(3);
    bool pending = false;   // the previous unit waits in buffer pair (n - 1) & 1
    CouplingUnit prev{0, 0};
    for (int n = 0;; ++n) {
        if (u >= units && !pending) break;
        const bool have = u < units;
        const CouplingUnit cu = have ? coupling_unit(u, L0, L1) : CouplingUnit{0, 0};
        double *Q = Sd + (n & 1) * kBuf;
        if (wave < 4 && have) {
            const int ke = min(min(cu.i0 + kCI - 1, lmax - cu.j0), kw0);
            v4d acc[2][4][2];
            coupling_mma(A, B, T, cu.i0, cu.j0, ke, wave, lane, acc);
            // (16x16 f64 result tile: register r of a lane holds row lane / 16 + 4 r, column lane % 16)
            if (wave >= 2) {
                double *P = Q + (wave - 2) * (2 * kTile);
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                P[p * kTile + (16 * mt + lk + 4 * r) * kPitch + 16 * nt + lr] = acc[p][mt][nt][r];
            }
            lds_barrier();
            if (wave < 2) {
                double *P = Q + wave * (2 * kTile);
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                double *x = P + p * kTile + (16 * mt + lk + 4 * r) * kPitch + 16 * nt + lr;
                                *x = acc[p][mt][nt][r] + *x;
                            }
            }
        } else {
            // the store waves write the previous unit; after the last unit all eight waves do
            if (pending && (wave >= 4 || !have)) {
                const double *P0 = Sd + ((n - 1) & 1) * kBuf;
                store_unit(P0, P0 + 2 * kTile, prev.i0, prev.j0, have ? wave - 4 : wave, have ? 4 : 8, lane, lmax, M);
            }
            lds_barrier();
        }
        if (threadIdx.x == 0) {
            unit_s = next;
            next = atomicAdd(counter, 1);
        }
        lds_barrier();   // the unit's sums are in Q; unit_s holds the next unit
        pending = have;
        prev = cu;
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

// One step of the pivot choice: combine with the lane rot places further round
// the lane's row of 16 (DPP row rotation), keeping the larger |value| and on a
// tie the lower row.
template <int ROT>
__device__ inline void lu_pivot_rotate(double &best, int &bi) {
    constexpr int ctrl = 0x120 + ROT;   // row_ror:ROT
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(best), ctrl, 0xF, 0xF, false);
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(best), ctrl, 0xF, 0xF, false);
    const int oi = __builtin_amdgcn_update_dpp(0, bi, ctrl, 0xF, 0xF, false);
    const double ov = __hiloint2double(hi, lo);
    if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
    }
}

// LU factorisation with partial pivoting (largest |pivot|, lowest row on ties)
// of the nb x nb row-major matrix Ag, in place, in one workgroup: afterwards
// the strict lower triangle holds L (unit diagonal), the upper triangle U, and
// perm[i] is the original row now at row i.  The matrix is worked on in LDS
// when it fits.  Each step: wave 0 finds the pivot (lane-local scan, then DPP
// rotations in rows of 16 and the four row results), the rows are swapped, and
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
            // largest |value|, lowest row on ties: a total order, so any combining
            // order gives the same row.  Within each row of 16 lanes by DPP
            // rotations (every lane ends with its row's choice), then over the four
            // rows from lanes 0, 16, 32, 48.
            lu_pivot_rotate<8>(best, bi);
            lu_pivot_rotate<4>(best, bi);
            lu_pivot_rotate<2>(best, bi);
            lu_pivot_rotate<1>(best, bi);
            double rv[4];
            int ri[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                rv[r] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(best), 16 * r),
                                         __builtin_amdgcn_readlane(__double2loint(best), 16 * r));
                ri[r] = __builtin_amdgcn_readlane(bi, 16 * r);
            }
            best = rv[0];
            bi = ri[0];
#pragma unroll
            for (int r = 1; r < 4; ++r)
                if (rv[r] > best || (rv[r] == best && ri[r] < bi)) {
                    best = rv[r];
                    bi = ri[r];
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
constexpr int kLuPB = 16;   // row block of the triangular solves
constexpr int kSolveLds = 20224;   // doubles of LDS per workgroup (factors and/or right-hand sides)
constexpr int kSolveBatch = 16;    // global loads in flight per thread when filling LDS

// Columns of the right-hand sides per workgroup of lu_solve_kernel, and whether
// the factors are copied into LDS next to them (when both fit).
inline void solve_shape(int nb, int *cols, bool *lu_in_lds) {
    const int room = kSolveLds - nb * nb;
    *lu_in_lds = room >= 16 * nb;
    // 16 columns (the least that fits any nb <= 1024): more workgroups, and each
    // thread's share of the rows (nb / 16) is shorter on the solve's critical path
    *cols = 16;
}

// X = U^-1 L^-1 P [C^_b | R] for the columns [col0, col0 + cols) of that
// (nb x (n1 + 1)) right-hand side, held in LDS (nb x cols): forward then back
// substitution, one row of the factors per step.  Column 0 is the binned
// pseudo-spectrum (-> cb), column 1 + l' is column l' of R (-> window).
template <bool kLuInLds>
__global__ __launch_bounds__(kSolveThreads) void lu_solve_kernel(const double *__restrict__ LUg,
                                                                 const int *__restrict__ perm, int nb,
                                                                 const double *__restrict__ R,
                                                                 const double *__restrict__ chat_b, int n1,
                                                                 int cols, double *__restrict__ cb,
                                                                 double *__restrict__ window) {
    __shared__ double lds[kSolveLds];
    const int tid = threadIdx.x;
    const double *LU = LUg;
    double *X = lds;   // nb x cols
    // global loads in batches of kSolveBatch per thread, all issued before their stores
    if (kLuInLds) {
        for (int e0 = 0; e0 < nb * nb; e0 += kSolveThreads * kSolveBatch) {
            double v[kSolveBatch];
#pragma unroll
            for (int u = 0; u < kSolveBatch; ++u) {
                const int e = e0 + u * kSolveThreads + tid;
                v[u] = e < nb * nb ? LUg[e] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kSolveBatch; ++u) {
                const int e = e0 + u * kSolveThreads + tid;
                if (e < nb * nb) lds[e] = v[u];
            }
        }
        LU = lds;
        X = lds + nb * nb;
    }
    const int col0 = blockIdx.x * cols;
    const int c = tid % cols, r0 = tid / cols, rstep = kSolveThreads / cols;
    const int gc = col0 + c;
    const bool live = gc <= n1;
    for (int i0 = r0; i0 < nb; i0 += rstep * kSolveBatch) {
        int src[kSolveBatch];
        double v[kSolveBatch];
#pragma unroll
        for (int u = 0; u < kSolveBatch; ++u) {
            const int i = i0 + u * rstep;
            src[u] = (live && i < nb) ? perm[i] : -1;
        }
#pragma unroll
        for (int u = 0; u < kSolveBatch; ++u)
            v[u] = src[u] < 0 ? 0.0 : (gc == 0 ? chat_b[src[u]] : R[(int64_t)src[u] * n1 + gc - 1]);
#pragma unroll
        for (int u = 0; u < kSolveBatch; ++u) {
            const int i = i0 + u * rstep;
            if (i < nb) X[i * cols + c] = v[u];
        }
    }
    __syncthreads();
    // L y = P b and then U x = y, by row blocks of kLuPB: a block's own rows are
    // solved in registers, one thread per column, then the rows beyond it are
    // updated by every thread.  Each entry receives the same multiply-adds in the
    // same order as in the row-by-row substitution (forward: ascending j; back:
    // descending j), so the result is the same bit for bit.
    for (int rb = 0; rb < nb; rb += kLuPB) {
        const int re = min(rb + kLuPB, nb);
        if (r0 == 0) {
            double xb[kLuPB];
#pragma unroll
            for (int a = 0; a < kLuPB; ++a) xb[a] = rb + a < re ? X[(rb + a) * cols + c] : 0.0;
#pragma unroll
            for (int a = 1; a < kLuPB; ++a)
                if (rb + a < re) {
#pragma unroll
                    for (int j = 0; j < a; ++j) xb[a] = fma(-LU[(rb + a) * nb + rb + j], xb[j], xb[a]);
                }
#pragma unroll
            for (int a = 1; a < kLuPB; ++a)
                if (rb + a < re) X[(rb + a) * cols + c] = xb[a];
        }
        __syncthreads();
        {
            double xj[kLuPB];   // the block's solved rows of this column
#pragma unroll
            for (int a = 0; a < kLuPB; ++a) xj[a] = rb + a < re ? X[(rb + a) * cols + c] : 0.0;
#pragma unroll 4
            for (int i = re + r0; i < nb; i += rstep) {
                double t = X[i * cols + c];
#pragma unroll
                for (int a = 0; a < kLuPB; ++a)
                    if (rb + a < re) t = fma(-LU[i * nb + rb + a], xj[a], t);
                X[i * cols + c] = t;
            }
        }
        __syncthreads();
    }
    for (int re = nb; re > 0; re -= kLuPB) {
        const int rb = max(re - kLuPB, 0);
        if (r0 == 0) {
            double xb[kLuPB];   // xb[a] holds row re - 1 - a
#pragma unroll
            for (int a = 0; a < kLuPB; ++a) xb[a] = re - 1 - a >= rb ? X[(re - 1 - a) * cols + c] : 0.0;
#pragma unroll
            for (int a = 0; a < kLuPB; ++a)
                if (re - 1 - a >= rb) {
                    const int i = re - 1 - a;
#pragma unroll
                    for (int j = 0; j < a; ++j) xb[a] = fma(-LU[i * nb + (re - 1 - j)], xb[j], xb[a]);
                    xb[a] = xb[a] / LU[i * nb + i];
                }
#pragma unroll
            for (int a = 0; a < kLuPB; ++a)
                if (re - 1 - a >= rb) X[(re - 1 - a) * cols + c] = xb[a];
        }
        __syncthreads();
        {
            double xj[kLuPB];   // xj[a] holds the solved row re - 1 - a of this column
#pragma unroll
            for (int a = 0; a < kLuPB; ++a) xj[a] = re - 1 - a >= rb ? X[(re - 1 - a) * cols + c] : 0.0;
#pragma unroll 4
            for (int i = r0; i < rb; i += rstep) {
                double t = X[i * cols + c];
#pragma unroll
                for (int a = 0; a < kLuPB; ++a)
                    if (re - 1 - a >= rb) t = fma(-LU[i * nb + re - 1 - a], xj[a], t);
                X[i * cols + c] = t;
            }
        }
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

namespace {

// A and B of coupling_ab_kernel for (device, lmax), kept for the process: built by
// the first call for that lmax outside stream capture (which waits for them once)
struct AbTables {
    double *buf;   // [pad | A | pad | pad | B | pad]
    const double *A() const { return buf + kTabPad; }
};
std::mutex g_ab_mu;
std::map<std::pair<int, int>, AbTables> g_ab;

}  // namespace

hipError_t release_coupling_tables() {
    std::lock_guard<std::mutex> lock(g_ab_mu);
    hipError_t first = hipSuccess;
    for (auto &kv : g_ab) {
        const hipError_t e = hipFree(kv.second.buf);
        if (first == hipSuccess) first = e;
    }
    g_ab.clear();
    return first;
}

hipError_t launch_coupling(const double *Wl, int lmax_w, const double *shot, double *scratch, int lmax, double *M,
                           hipStream_t stream) {
    // scratch: [pad | A | pad | pad | B | pad | pad | T | pad | counter]; A and B are
    // used only when the cached tables are not there (first call under capture)
    double *A = scratch + kTabPad;
    double *B = A + (lmax + 1) + 2 * kTabPad;
    double *T = B + (2 * lmax + 1) + 2 * kTabPad;
    int *counter = (int *)(T + (2 * lmax + 2) + kTabPad);
    const size_t ab_doubles = (size_t)(lmax + 1) + (2 * lmax + 1) + 4 * kTabPad;
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    const double *Ause = A, *Buse = B;
    {
        std::lock_guard<std::mutex> lock(g_ab_mu);
        auto it = g_ab.find({dev, lmax});
        if (it == g_ab.end()) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if ((e = hipStreamIsCapturing(stream, &cs)) != hipSuccess) return e;
            if (cs == hipStreamCaptureStatusNone) {
                double *buf = nullptr;
                if ((e = hipMalloc((void **)&buf, sizeof(double) * ab_doubles)) != hipSuccess) return e;
                double *a = buf + kTabPad, *b = a + (lmax + 1) + 2 * kTabPad;
                hipLaunchKernelGGL(coupling_ab_kernel, dim3(1), dim3(kTabThreads), 0, stream, lmax, a, b);
                if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(stream)) != hipSuccess) {
                    (void)hipFree(buf);
                    return e;
                }
                it = g_ab.emplace(std::make_pair(dev, lmax), AbTables{buf}).first;
            }
        }
        if (it != g_ab.end()) {
            Ause = it->second.A();
            Buse = Ause + (lmax + 1) + 2 * kTabPad;
        } else {
            hipLaunchKernelGGL(coupling_ab_kernel, dim3(1), dim3(kTabThreads), 0, stream, lmax, A, B);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    const int nt = 2 * lmax + 2 + 2 * kTabPad;
    hipLaunchKernelGGL(coupling_t_kernel, dim3((nt + kTabThreads - 1) / kTabThreads), dim3(kTabThreads), 0, stream, Wl,
                       lmax_w, shot, lmax, T, counter);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the CU count and the kernel's LDS attribute, once per device (host calls
    // between the launches would leave the GPU idle)
    static std::mutex mu;
    static std::map<int, int> cus_of;
    int cus = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cus_of.find(dev);
        if (it == cus_of.end()) {
            if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
            if ((e = hipFuncSetAttribute((const void *)coupling_mfma_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCouplingLds)) != hipSuccess)
                return e;
            it = cus_of.emplace(dev, cus > 0 ? cus : 1).first;
        }
        cus = it->second;
    }
    const int lw = lmax_w < 2 * lmax ? lmax_w : 2 * lmax;
    const int kw0 = lw >> 1;   // k range of the even parity (the odd one's extra terms vanish)
    const unsigned grid = (unsigned)cus;
    hipLaunchKernelGGL(coupling_mfma_kernel, dim3(grid), dim3(kCouplingThreads), kCouplingLds, stream, Ause, Buse,
                       (const double *)T, lmax, kw0, counter, M);
    return hipGetLastError();
}

size_t bandpower_scratch_doubles(int lmax, int nb) {
    const size_t n1 = (size_t)lmax + 1;
    // R = theta M, Mbb and its factors, theta C^, the row permutation (ints), N
    return (size_t)nb * n1 + (size_t)nb * nb + (size_t)nb + ((size_t)nb + 1) / 2 + 1;
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
    double *chat_b = Mbb + (size_t)nb * nb;
    int *perm = (int *)(chat_b + nb);
    hipLaunchKernelGGL(bin_rows_kernel, dim3(blocks_for((int64_t)nb * n1, 256)), dim3(256), 0, stream, M, n1, lmin,
                       delta_l, nb, (const double *)nullptr, R);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // (theta C^)_b, the first right-hand side
    hipLaunchKernelGGL(bin_rows_kernel, dim3(blocks_for(nb, 256)), dim3(256), 0, stream, cl_hat, 1, lmin, delta_l, nb,
                       (const double *)nullptr, chat_b);
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
        hipLaunchKernelGGL(lu_solve_kernel<true>, dim3(grid), dim3(kSolveThreads), 0, stream, Mbb, perm, nb, R,
                           (const double *)chat_b, n1, cols, cb, window);
    else
        hipLaunchKernelGGL(lu_solve_kernel<false>, dim3(grid), dim3(kSolveThreads), 0, stream, Mbb, perm, nb, R,
                           (const double *)chat_b, n1, cols, cb, window);
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
