// Wavefront helpers shared by the direct-sum kernels (scalar and spin-weighted):
// constant-address-space table pointers, exponent-tracked complex
// renormalisation, chain range limits, and the fixed-order cross-lane
// reduction of per-lane l-block sums.  Device-only, with internal linkage
// (anonymous namespace): every kernel file that includes it gets its own copy.
#pragma once

#include <hip/hip_runtime.h>

namespace ptalm {
namespace {

// Read-only tables in the constant address space: uniform indices into them
// compile to scalar loads (s_load), so the step coefficients live in SGPRs.
template <typename T>
using const_ptr = const T __attribute__((address_space(4))) *;

__device__ inline double ldexp_t(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
__device__ inline float ldexp_t(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }
__device__ inline int frexp_exp_t(double x) { return __builtin_amdgcn_frexp_exp(x); }
__device__ inline int frexp_exp_t(float x) { return __builtin_amdgcn_frexp_expf(x); }

// (re, im) * 2^-e so that max(|re|, |im|) lies in [0.5, 1); exponent += e.
__device__ inline void renorm(double &re, double &im, int &exponent) {
    const double mx = fmax(fabs(re), fabs(im));
    const int e = (mx != 0.0) ? frexp_exp_t(mx) : 0;
    re = ldexp_t(re, -e);
    im = ldexp_t(im, -e);
    exponent += e;
}

// Chain range control.  The chain grows fastest right after its start next to
// a pole, where the step ratio is about x sqrt(2m / (l - m)): over 16 steps by
// less than 2^98 for any m <= 16383, over 128 steps by less than 2^446 for
// m ~ 3000 and 2^600 for any m <= 16383 (the normalised recurrence run on the
// host at x up to 1 - 1e-12).  FP64 chains are checked every 128 l against
// 2^64 (so they stay below 2^664), FP32 chains every 16 l against 2^16, so
// neither can overflow between checks.
template <typename RecT> struct ChainRange;
template <> struct ChainRange<double> {
    static constexpr int every_l = 128;
    static constexpr double above = 0x1p+64;
};
template <> struct ChainRange<float> {
    static constexpr int every_l = 16;
    static constexpr float above = 0x1p+16f;
};

// Cross-lane reduction of the per-lane l-block sums (V values per lane, value
// v = 2k + c for l = jb + k and c = re/im).  Optional register stage (SWAP = 1):
// v_permlane32_swap exchanges the upper half of value i with the lower half of
// value i + V/2, so after one add each lane holds V/2 values summed over two
// lanes.  The rest goes through LDS as a transpose: every lane writes its
// values, then P = 64/V lanes per value each add an interleaved share of the
// entries and combine by DPP.  All orders are fixed.
template <int V, int SWAP>
struct Red {
    static constexpr int ENTRIES = 64 >> SWAP;  // lanes contributing to each value in LDS
    static constexpr int P = 64 / V;            // lanes combining one value at the end
    static constexpr int ROW = ENTRIES + 1;     // padded LDS row (elements)
    static constexpr int BUF = V * ROW;         // elements per LDS buffer
};

// value from lane (lane ^ 1) or (lane ^ 2) within each quad (DPP quad_perm)
template <int XOR>
__device__ inline int dpp_xor_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, XOR == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false);
}
template <int XOR>
__device__ inline double dpp_xor(double x) {
    return __hiloint2double(dpp_xor_i<XOR>(__double2hiint(x)), dpp_xor_i<XOR>(__double2loint(x)));
}
template <int XOR>
__device__ inline float dpp_xor(float x) {
    return __int_as_float(dpp_xor_i<XOR>(__float_as_int(x)));
}

// Lanes 0-31 get value a summed over lanes j and j+32; lanes 32-63 get value b
// summed over lanes j-32 and j (v_permlane32_swap on each 32-bit half).
__device__ inline double swap32_add(double a, double b) {
    unsigned al = __double2loint(a), ah = __double2hiint(a), bl = __double2loint(b), bh = __double2hiint(b);
    auto lo = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ inline float swap32_add(float a, float b) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Orders LDS accesses of this wavefront (each workgroup is one wavefront, and
// one wavefront's LDS operations complete in order).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename AccT, int V, int SWAP>
__device__ inline void reduce_write(AccT *buf, const AccT (&vals)[V], int lane) {
    using R = Red<V, SWAP>;
    if constexpr (SWAP == 0) {
#pragma unroll
        for (int i = 0; i < V; ++i) buf[i * R::ROW + lane] = vals[i];
    } else {
        const int half = lane >> 5;
#pragma unroll
        for (int i = 0; i < V / 2; ++i) {
            const AccT u = swap32_add(vals[i], vals[i + V / 2]);
            buf[(i + half * (V / 2)) * R::ROW + (lane & 31)] = u;
        }
    }
}

template <typename AccT, int V, int SWAP>
__device__ inline AccT reduce_finish(const AccT *buf, int v, int h) {
    using R = Red<V, SWAP>;
    static_assert(R::P <= 4, "at most 4 lanes per value");
    AccT sum = buf[v * R::ROW + h];
#pragma unroll
    for (int k = 1; k < R::ENTRIES / R::P; ++k) sum += buf[v * R::ROW + h + k * R::P];
    if constexpr (R::P >= 2) sum += dpp_xor<1>(sum);
    if constexpr (R::P >= 4) sum += dpp_xor<2>(sum);
    return sum;
}

}  // namespace
}  // namespace ptalm
