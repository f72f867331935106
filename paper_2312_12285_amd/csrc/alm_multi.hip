// Multi-weight transform on the matrix cores: NW weight vectors share one
// position set, a^(v)_lm = sum_i w_v[i] Y*_lm(theta_i, phi_i) (eq. alm_def for
// each v).  For a fixed order m the sum over points is a dense contraction
//     D[l][c] = sum_i A[l][i] B[i][c],
//     A[l][i] = Pbar_l^m(x_i) / (s_i^m e_j)       (the scaled recurrence value),
//     B[i][2v + part] = w_v[i] * (cos, -sin)(m phi_i) * s_i^m   (as a normalised
//                       mantissa; its exponent is folded into A),
// with M = l, K = points, N = 2 NW columns, which maps onto MFMA.  Operands are
// split into bf16 hi + lo parts and three products (hi.hi + hi.lo + lo.hi) are
// accumulated in FP32 on v_mfma_f32_16x16x32_bf16; the neglected lo.lo term and
// the residual of the two-term split leave ~2^-16 relative error per product.
//
// Work decomposition.  One workgroup (8 wavefronts, 512 threads, one per compute
// unit) per (slice, m) item, dispatched in increasing m (largest work first).  It
// streams its slice in groups of 512 points, one point per thread:
//   1. each thread computes its point's x, s^m e^{-i m phi} (FP64, exponent
//      tracked) and stages its row of B (FP32) and x in LDS; each wavefront
//      then splits the B fragments of its half of the points (256) into bf16
//      hi/lo registers kept for all l;
//   2. per tile of 32 l: each thread advances the FP64 split recurrence of
//      tables.hip 32 steps and writes A (bf16 hi/lo) for its point to LDS, the
//      16 even-l rows first, then the 16 odd-l rows.  An odd-l value of the
//      recurrence lacks a factor x, which the wavefronts that own the odd rows
//      fold into their copy of B instead.  Wavefront w multiplies M-tile
//      (w & 1) by N-tiles of its quarter of the columns over the 256 points of
//      its half (8 K-steps x 3 products per D tile), interleaved with the
//      recurrence of the next tile.  The two wavefronts that hold the same D
//      block for the two point halves exchange half of it through LDS; each adds
//      its half of the block for all 512 points into the slice's FP32 partial
//      (the first group of a slice stores; later groups add with the hardware
//      FP32 atomic, which saves the load of the old value: one lane owns each
//      value, so its adds reach the partial in program order and the result is
//      that of a read-modify-write in group order).
// The partial buffer pads every order by 32 rows, so whole tiles are written
// without bounds tests.  A final pass sums the slices in FP64 in fixed
// order and applies the output scale sigma_lm.  Every order is fixed, so
// results are reproducible.
#include "ptalm_internal.h"

namespace ptalm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_bits;

template <typename T>
using const_ptr = const T __attribute__((address_space(4))) *;

constexpr int kG = kMultiGroup;  // points per group = threads per workgroup
constexpr int kHalf = kG / 2;    // points of one half: the K range of one wavefront
constexpr int kLT = 32;          // l values per tile
constexpr int kRowA = kG + 8;    // padded LDS row of an A tile (bf16): rows land on different banks
constexpr int kRowB = kG + 4;    // padded LDS column of the staged B (floats)
constexpr int kLive = -512;                  // exponent from which the chain registers hold A itself
constexpr double kChainAbove = 0x1p+64 * 0x1p-512;   // 2^64 for the chain below kLive (scaled by 2^kLive)
static_assert(kLT == kMultiPad, "tiles must fit the padding of the partial buffer");

__device__ inline double ldexp_d(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
__device__ inline int frexp_exp_d(double x) { return __builtin_amdgcn_frexp_exp(x); }

__device__ inline void renorm(double &re, double &im, int &exponent) {
    const double mx = fmax(fabs(re), fabs(im));
    const int e = (mx != 0.0) ? frexp_exp_d(mx) : 0;
    re = ldexp_d(re, -e);
    im = ldexp_d(im, -e);
    exponent += e;
}

// An FP32 value the optimiser may not look through: the A operand is rounded to
// FP32 first and then split, and must not be re-derived from the FP64 value.
__device__ inline float opaque(float f) {
    asm("" : "+v"(f));
    return f;
}

// f_k = hi_k + lo_k + O(2^-17 |f_k|) for a pair (k = 0, 1), both parts rounded
// to nearest even by v_cvt_pk_bf16_f32; the parts come back packed, element 0
// in the low half.
__device__ inline void split_pair(float f0, float f1, unsigned &hi, unsigned &lo) {
    hi = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){f0, f1}, bf16x2));
    const float h0 = __builtin_bit_cast(float, hi << 16);
    const float h1 = __builtin_bit_cast(float, hi & 0xffff0000u);
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){f0 - h0, f1 - h1}, bf16x2));
}

__device__ inline bf16x8 load_frag(const bf16_bits *p) {
    // 8 consecutive bf16 (16 bytes, 16-byte aligned)
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

template <int NW>
__global__ __launch_bounds__(kG) __attribute__((amdgpu_waves_per_eu(2))) void alm_multi_kernel(MultiArgs a) {
    constexpr int NC = 2 * NW;          // columns of B (re, im per weight vector)
    constexpr int NT = NC / 16;         // 16-column N-tiles
    constexpr int NTW = NT / 2;         // N-tiles per wavefront (two wavefronts per M-tile and half)
    constexpr int KS = kHalf / 32;      // K-steps of one wavefront per tile
    constexpr int NV = 4 * NTW;         // D values per lane (value v = 4 n + r)
    constexpr int NOWN = NV / 2;        // of which this wavefront adds into the partial
    static_assert(NW % 16 == 0 && NW <= 32, "NW must be 16 or 32");
    // LDS: one region used first as the FP32 staging of B and x at a group's
    // start, then as the two A tiles (double buffer) x (hi, lo); after it the
    // D exchange [tile parity][wavefront][value][lane]
    constexpr int kStage = (NC * kRowB + kG) * 4;
    constexpr int kATile = kLT * kRowA;                 // bf16 elements of one A part
    constexpr int kABytes = 2 * 2 * kATile * 2;
    constexpr int kMain = kStage > kABytes ? kStage : kABytes;
    constexpr int kXch = 2 * (kG / 64) * NOWN * 64 * 4;
    __shared__ __attribute__((aligned(16))) unsigned char smem[kMain + kXch];
    float *Bs = reinterpret_cast<float *>(smem);        // [NC][kRowB]
    float *Xs = Bs + NC * kRowB;                        // [kG]
    bf16_bits *At = reinterpret_cast<bf16_bits *>(smem);  // [buffer][hi, lo][kLT][kRowA]
    float *xch = reinterpret_cast<float *>(smem + kMain);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lmax = a.lmax;
    const int s = blockIdx.x % a.n_slices;
    const int m = __builtin_amdgcn_readfirstlane(blockIdx.x / a.n_slices);
    const int L = lmax - m + 1;
    const int64_t g_a = (int64_t)s * a.groups / a.n_slices;
    const int64_t g_b = (int64_t)(s + 1) * a.groups / a.n_slices;
    const const_ptr<double> cm = (const_ptr<double>)a.coef + coef_segment(lmax, m);

    const int half = wave >> 2;          // point half of this wavefront (its K range)
    const int kbase = half * kHalf;
    const int mt = wave & 1;             // M-tile: 0 even l, 1 odd l
    const int nt0 = ((wave >> 1) & 1) * NTW;   // first N-tile
    const int partner = wave ^ 4;        // same D block, other point half
    const int frow = lane & 15;          // fragment row / column within a 16-tile
    const int fk = 8 * (lane >> 4);      // fragment k offset within a 32-step
    // this lane's D rows: tile row 4*(lane/16) + r holds l = jb + 2*(4*(lane/16) + r) + mt
    const int drow = 2 * (4 * (lane >> 4)) + mt;
    float *part = a.partial32 + ((int64_t)s * multi_rows(lmax) + multi_row_start(lmax, m)) * NC;
    // partial offset (within a tile) of the o-th value this lane adds: value v = half*NOWN + o
    auto own_offset = [&](int o) {
        const int v = half * NOWN + o, n = v >> 2, r = v & 3;
        return (drow + 2 * r) * NC + (nt0 + n) * 16 + frow;
    };

    for (int64_t g = g_a; g < g_b; ++g) {
        const bool first = (g == g_a);
        // ---- 1. point data; stage B = w Z (FP32) and x --------------------------
        const int64_t i = g * kG + tid;
        const bool valid = i < a.n;
        // every load issued at once from a clamped index (the tail's points get
        // weight 0 and a harmless position), so their latencies overlap
        const int64_t ic = valid ? i : a.n - 1;
        float wv[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v) wv[v] = a.w32[(int64_t)v * a.n + ic];
        double th = a.theta[ic], ph = a.phi[ic];
        if (!valid) {
            th = 1.5707963267948966;
            ph = 0.0;
        }
        double st, ct, sp, cp;
        sincos(th, &st, &ct);
        sincos(ph, &sp, &cp);
        const double x = ct, y = ct * ct;
        // Z = (s e^{-i phi})^m, mantissa + exponent, by binary powering
        double br = st * cp, bi = -st * sp;
        int be = 0;
        renorm(br, bi, be);
        double zr = 1.0, zi = 0.0;
        int ze = 0;
        for (int k = m; k; k >>= 1) {
            if (k & 1) {
                const double tr = zr * br - zi * bi, ti = zr * bi + zi * br;
                zr = tr;
                zi = ti;
                ze += be;
                renorm(zr, zi, ze);
            }
            if (k > 1) {
                const double tr = br * br - bi * bi, ti = 2.0 * br * bi;
                br = tr;
                bi = ti;
                be *= 2;
                renorm(br, bi, be);
            }
        }
        const float zr32 = (float)zr, zi32 = (float)zi;
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            const float wq = valid ? wv[v] : 0.f;
            Bs[(2 * v) * kRowB + tid] = wq * zr32;
            Bs[(2 * v + 1) * kRowB + tid] = wq * zi32;
        }
        Xs[tid] = (float)x;
        __syncthreads();
        // B fragments of this wavefront's points (x folded in for the odd-l
        // rows), kept for every l-tile of this group
        bf16x8 bh[NTW][KS], bl[NTW][KS];
#pragma unroll
        for (int n = 0; n < NTW; ++n)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k0 = kbase + ks * 32 + fk;
                const float *bp = Bs + ((nt0 + n) * 16 + frow) * kRowB + k0;
                const f32x4 b0 = *reinterpret_cast<const f32x4 *>(bp);
                const f32x4 b1 = *reinterpret_cast<const f32x4 *>(bp + 4);
                f32x4 x0 = *reinterpret_cast<const f32x4 *>(Xs + k0);
                f32x4 x1 = *reinterpret_cast<const f32x4 *>(Xs + k0 + 4);
                if (mt == 0) x0 = x1 = (f32x4){1.f, 1.f, 1.f, 1.f};
                const float f[8] = {b0[0] * x0[0], b0[1] * x0[1], b0[2] * x0[2], b0[3] * x0[3],
                                    b1[0] * x1[0], b1[1] * x1[1], b1[2] * x1[2], b1[3] * x1[3]};
                uint4 h, l;
                split_pair(f[0], f[1], h.x, l.x);
                split_pair(f[2], f[3], h.y, l.y);
                split_pair(f[4], f[5], h.z, l.z);
                split_pair(f[6], f[7], h.w, l.w);
                bh[n][ks] = __builtin_bit_cast(bf16x8, h);
                bl[n][ks] = __builtin_bit_cast(bf16x8, l);
            }
        __syncthreads();   // the staging region becomes the A tiles

        // ---- 2. l-tiles, software pipelined: the MFMAs of tile t read one A
        // buffer while the recurrence writes tile t+1 into the other ----------
        // The chain (E, O) of tables.hip times 2^q is A.  While q >= kLive the
        // registers hold that product itself (live: A is read off them, and its
        // values stay inside the FP32 range, so far inside FP64's); below, they
        // hold the chain times 2^kLive, small enough that every A rounds to 0 in
        // FP32 as it must (A < 2^(kLive + 192) there, the chain staying below
        // 2^192 between checks), yet normal in FP64, so the chain loses nothing.
        // Scaling by powers of two commutes with the rounding, so the A values
        // are those of a chain kept apart from its exponent.  A point exactly at
        // a pole has s^m = 0 for m > 0 and contributes nothing: it stays below.
        int q = (zr == 0.0 && zi == 0.0) ? -100000 : ze;
        double E = -ldexp_d(1.0, q < kLive ? kLive : q), O = 0.0;
        // one recurrence pair (steps k, k+1 with coefficients c0, c1): its two A
        // values, split, into rows k/2 (even l) and 16 + k/2 (odd l) of buffer b
        auto recur_pair = [&](double c0, double c1, int k, int b) {
            bf16_bits *ah = At + (2 * b) * kATile + tid;
            bf16_bits *al = ah + kATile;
            E = fma(c0 * y, O, -E);
            O = fma(c1, E, -O);
            unsigned hi, lo;
            split_pair(opaque((float)E), opaque((float)O), hi, lo);
            ah[(k >> 1) * kRowA] = (bf16_bits)hi;
            ah[(kLT / 2 + (k >> 1)) * kRowA] = (bf16_bits)(hi >> 16);
            al[(k >> 1) * kRowA] = (bf16_bits)lo;
            al[(kLT / 2 + (k >> 1)) * kRowA] = (bf16_bits)(lo >> 16);
        };
#pragma unroll
        for (int k = 0; k < kLT; k += 2) recur_pair(cm[k], cm[k + 1], k, 0);
        __syncthreads();
        const int ntiles = (L + kLT - 1) / kLT;
        constexpr int kUnits = NTW * KS;   // (K-step, N-tile) units of 3 MFMAs per tile
        for (int t = 0; t < ntiles; ++t) {
            const int jb = t * kLT;
            const int b = t & 1;
            float *pt = part + (int64_t)jb * NC;
            // step coefficients of the next tile (the tile after the last reads
            // the table's padding; steps past lmax-m land in padding rows)
            double cf[kLT];
#pragma unroll
            for (int k = 0; k < kLT; ++k) cf[k] = cm[jb + kLT + k];
            f32x4 d[NTW];
#pragma unroll
            for (int n = 0; n < NTW; ++n) d[n] = f32x4{0.f, 0.f, 0.f, 0.f};
            const bf16_bits *ah = At + (2 * b) * kATile + (mt * 16 + frow) * kRowA + kbase + fk;
            bf16x8 fa_h[KS], fa_l[KS];
            fa_h[0] = load_frag(ah);
            fa_l[0] = load_frag(ah + kATile);
            // The MFMAs of this tile interleaved with the recurrence of the next
            // one, in issue order fixed by scheduling fences, so one wavefront
            // keeps the matrix core and the vector ALU busy at the same time; each
            // K-step's A fragments are read one K-step ahead.
#pragma unroll
            for (int i = 0; i < kLT / 2; ++i) {
                // the MFMAs issue at raised wave priority, the recurrence at normal
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int u = i * kUnits / (kLT / 2); u < (i + 1) * kUnits / (kLT / 2); ++u) {
                    const int ks = u / NTW, n = u % NTW;
                    if (n == 0 && ks + 1 < KS) {
                        fa_h[ks + 1] = load_frag(ah + (ks + 1) * 32);
                        fa_l[ks + 1] = load_frag(ah + kATile + (ks + 1) * 32);
                    }
                    d[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa_h[ks], bh[n][ks], d[n], 0, 0, 0);
                    d[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa_h[ks], bl[n][ks], d[n], 0, 0, 0);
                    d[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa_l[ks], bh[n][ks], d[n], 0, 0, 0);
                }
                __builtin_amdgcn_s_setprio(0);
                recur_pair(cf[2 * i], cf[2 * i + 1], 2 * i, b ^ 1);
                __builtin_amdgcn_sched_barrier(0);
            }
            // below kLive, keep the chain (registers x 2^-kLive) under 2^64 (its
            // growth is < 2^255 per 64 steps), moving the excess into q, and go
            // live once q reaches kLive
            if (q < kLive) {
                const double mx = fmax(fabs(E), fabs(O));
                const int e = mx > kChainAbove ? frexp_exp_d(mx) - kLive : 0;
                q += e;
                const int sh = q < kLive ? -e : q - kLive - e;
                E = ldexp_d(E, sh);
                O = ldexp_d(O, sh);
            }
            // D[row][col]: row = 4*(lane/16) + r, col = lane % 16 (checked layout);
            // value v = 4 n + r.  Hand the values the partner adds to it.
            float dv[NV];
#pragma unroll
            for (int n = 0; n < NTW; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) dv[4 * n + r] = d[n][r];
            float *xw = xch + ((b * (kG / 64) + wave) * NOWN) * 64 + lane;
            const float *xr = xch + ((b * (kG / 64) + partner) * NOWN) * 64 + lane;
#pragma unroll
            for (int o = 0; o < NOWN; ++o) xw[o * 64] = half ? dv[o] : dv[NOWN + o];
            __syncthreads();
#pragma unroll
            for (int o = 0; o < NOWN; ++o) {
                const float mine = half ? dv[NOWN + o] : dv[o];
                const float val = mine + xr[o * 64];
                if (first)
                    pt[own_offset(o)] = 0.f + val;
                else
                    (void)unsafeAtomicAdd(pt + own_offset(o), val);
            }
        }
    }
}

// out[v][column_start(m) + j] = sigma * sum_s partial[s][row(m) + j][2v, 2v+1]
// (compensated FP64 sum in slice order); one workgroup per order m
__global__ void multi_finish_kernel(const float *__restrict__ partial, int n_slices, int nw,
                                    const double *__restrict__ sigma, int lmax, double *__restrict__ alm) {
    const int m = blockIdx.x;
    const int L = lmax - m + 1;
    const int64_t T = tri_size(lmax), rows = multi_rows(lmax);
    const int64_t c0 = column_start(lmax, m), r0 = multi_row_start(lmax, m);
    const int nc = 2 * nw;
    for (int e = threadIdx.x; e < L * nw; e += blockDim.x) {
        const int v = e / L, j = e - v * L;
        double re = 0.0, im = 0.0, cre = 0.0, cim = 0.0;
        for (int s = 0; s < n_slices; ++s) {
            const float2 p = *reinterpret_cast<const float2 *>(partial + ((int64_t)s * rows + r0 + j) * nc + 2 * v);
            neumaier_add(re, cre, (double)p.x);
            neumaier_add(im, cim, (double)p.y);
        }
        const double sg = sigma[c0 + j];
        reinterpret_cast<double2 *>(alm)[(int64_t)v * T + c0 + j] = make_double2(sg * (re + cre), sg * (im + cim));
    }
}

// weights FP64 -> FP32 copy (the B operand is formed in FP32 before its split)
__global__ void weights_to_f32_kernel(const double *__restrict__ w, int64_t count, float *__restrict__ w32) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
        w32[e] = (float)w[e];
}

unsigned grid_for(int64_t count, int threads) {
    int64_t b = (count + threads - 1) / threads;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

bool multi_nw_supported(int nw) { return nw == 16 || nw == 32; }

hipError_t launch_alm_multi(const MultiArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL(weights_to_f32_kernel, dim3(grid_for((int64_t)a.n_weights * a.n, 256)), dim3(256), 0, stream,
                       a.w, (int64_t)a.n_weights * a.n, a.w32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int blocks = (a.lmax + 1) * a.n_slices;
    if (a.n_weights == 32)
        hipLaunchKernelGGL(alm_multi_kernel<32>, dim3(blocks), dim3(kG), 0, stream, a);
    else
        hipLaunchKernelGGL(alm_multi_kernel<16>, dim3(blocks), dim3(kG), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_multi_finish(const MultiArgs &a, const double *sigma, double *alm, hipStream_t stream) {
    hipLaunchKernelGGL(multi_finish_kernel, dim3(a.lmax + 1), dim3(256), 0, stream,
                       a.partial32, a.n_slices, a.n_weights, sigma, a.lmax, alm);
    return hipGetLastError();
}

}  // namespace ptalm
