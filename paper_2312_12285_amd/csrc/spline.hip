// Interpolated transform of App. A.2: cubic Hermite splines of y_lm(x) and
// y'_lm(x) on a node grid, the points summed into per-m binned weights per
// interval, and a sum over the nodes.  Points outside the spline region take
// the exact direct sum (the caller adds it).
//
// Nodes: n_nodes nodes uniform in theta over [theta_cut, pi - theta_cut],
// x_j = cos(pi - theta_cut - j h), ascending in x, h = (pi - 2 theta_cut)/(n_nodes - 1);
// interval j = [x_j, x_{j+1}).  With t = (x - x_j)/(x_{j+1} - x_j) and the basis
// c_0..c_3 of App. A.2,
//   v_ja^(m) = sum_{r in j} w_r e^{-i m phi_r} c_a(t_r),
//   a_lm = sum_j [v_j0 y(x_j) + v_j1 dx_j y'(x_j) + v_j2 y(x_{j+1}) + v_j3 dx_j y'(x_{j+1})],
// which per node n is a_lm = sum_n V_n y_lm(x_n) + D_n y'_lm(x_n) with
// V_n = v_n0 + v_{n-1,2}, D_n = dx_n v_n1 + dx_{n-1} v_{n-1,3}.  The derivative
// relation of App. A.1, for the orthonormal functions,
//   (1 - x^2) y'_l = -l x y_l + d_l y_{l-1},  d_l = sqrt((2l+1)/(2l-1) (l^2 - m^2)),
// turns the derivative part into two more plain sums over the nodes:
//   a_lm = A_l - l F_l + d_l G_{l-1},   A_l = sum_n V_n y_l(x_n),
//   F_l = sum_n D_n x_n/(1-x_n^2) y_l(x_n),  G_l = sum_n D_n/(1-x_n^2) y_l(x_n).
//
// Steps: count points per interval (polar points in an extra bucket), scan,
// scatter into interval order with the spline weights w c_a precomputed,
// binning (one wavefront per (interval, 8 orders)), node weights per (m, n),
// and the node sum as a direct sum over the nodes (the wavefront design of the
// direct kernels: nodes in lanes, the recurrence over l in registers, four
// sums per l reduced across lanes), then a_lm from its two sums per l.
#include <type_traits>

#include "ptalm_internal.h"
#include "wave_common.h"

namespace ptalm {

namespace {

constexpr double kPi = 3.141592653589793;
constexpr double kInv4Pi = 0.079577471545947667884441881686257181;
constexpr double kInv2Pi = 0.15915494309189533576888376337251436;
constexpr int kPointDoubles = 8;   // doubles per sorted point record

__device__ inline int interval_of(double th, double theta_cut, double h, int n_int) {
    if (th < theta_cut || th > kPi - theta_cut) return n_int;   // polar bucket
    const double u = (kPi - theta_cut - th) / h;
    const int j = (int)floor(u);
    return j < n_int - 1 ? j : n_int - 1;
}

__global__ void nodes_kernel(double theta_cut, double h, int n_nodes, double *__restrict__ xn,
                             double *__restrict__ thn) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_nodes) return;
    const double th = kPi - theta_cut - h * j;
    thn[j] = th;
    xn[j] = cos(th);
}

// Stable counting sort of the points by interval (polar points in the last
// bucket), so the order of the points inside an interval is their input order
// and the binning sums are reproducible bit for bit.  The points are cut into
// fixed chunks, one wavefront each:
//   chunk_hist_kernel   H[c][b] = points of chunk c in bucket b (LDS histogram);
//   bucket_total_kernel counts[b] = sum_c H[c][b];  scan_kernel: offsets;
//   bucket_start_kernel H[c][b] <- offsets[b] + sum_{c' < c} H[c'][b], the place
//                       of the first point of chunk c in bucket b;
//   stable_scatter_kernel each wavefront walks its chunk in input order, 64
//                       points per round; each lane compares its bucket with
//                       every other lane's (lane shuffles), which gives its rank
//                       among the lower lanes of the same bucket, so a point's
//                       place is its chunk's start in its bucket plus the points
//                       of that bucket before it in the chunk.
// Buckets are handled in windows of kHistMax (one LDS array per wavefront), one
// pass over the chunk per window.
constexpr int kHistMax = 16384;      // buckets per LDS window (64 KB)
constexpr int kSortChunksMax = 1024;
constexpr int64_t kSortChunkMin = 4096;

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__global__ __launch_bounds__(64) void chunk_hist_kernel(const double *__restrict__ theta, int64_t n, double theta_cut,
                                                        double h, int n_int, int64_t chunk,
                                                        unsigned *__restrict__ H) {
    extern __shared__ unsigned hist[];   // min(nb, kHistMax) counters (dynamic, so that small bucket counts
                                         // leave room for more wavefronts per CU)
    const int nb = n_int + 1;
    const int64_t c = blockIdx.x;
    const int64_t lo = c * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int w0 = 0; w0 < nb; w0 += kHistMax) {
        const int wn = nb - w0 < kHistMax ? nb - w0 : kHistMax;
        for (int b = threadIdx.x; b < wn; b += 64) hist[b] = 0u;
        wave_sync_lds();
        for (int64_t i = lo + threadIdx.x; i < hi; i += 64) {
            const int b = interval_of(theta[i], theta_cut, h, n_int) - w0;
            if (b >= 0 && b < wn) atomicAdd(&hist[b], 1u);   // a count: the order does not matter
        }
        wave_sync_lds();
        for (int b = threadIdx.x; b < wn; b += 64) H[c * nb + w0 + b] = hist[b];
        wave_sync_lds();
    }
}

__global__ void bucket_total_kernel(const unsigned *__restrict__ H, int n_chunks, int nb,
                                    unsigned *__restrict__ counts) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    unsigned s = 0u;
    for (int c = 0; c < n_chunks; ++c) s += H[(int64_t)c * nb + b];
    counts[b] = s;
}

// H[c][b] <- offsets[b] + sum_{c' < c} H[c'][b]; the polar count goes to *n_polar
__global__ void bucket_start_kernel(unsigned *__restrict__ H, int n_chunks, int nb,
                                    const int64_t *__restrict__ offsets, int64_t *__restrict__ n_polar) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    unsigned run = (unsigned)offsets[b];
    for (int c = 0; c < n_chunks; ++c) {
        const unsigned t = H[(int64_t)c * nb + b];
        H[(int64_t)c * nb + b] = run;
        run += t;
    }
    if (b == nb - 1) *n_polar = offsets[nb] - offsets[nb - 1];
}

// Points of the spline region in interval order, one 64-byte record each:
// (w c_0(t), w c_1(t), w c_2(t), w c_3(t), phi / (2 pi), cos phi, sin phi, 0);
// polar points (bucket n_int) to their own arrays, in input order as well.
__global__ __launch_bounds__(64) void stable_scatter_kernel(
    const double *__restrict__ theta, const double *__restrict__ phi, const double *__restrict__ w, int64_t n,
    double theta_cut, double h, int n_int, int64_t chunk, const double *__restrict__ xn,
    const int64_t *__restrict__ offsets, const unsigned *__restrict__ start, double *__restrict__ q,
    double *__restrict__ pth, double *__restrict__ pph, double *__restrict__ pw) {
    extern __shared__ unsigned cur[];   // min(nb, kHistMax) cursors (dynamic, as in chunk_hist_kernel)
    const int nb = n_int + 1;
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int64_t lo = c * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int w0 = 0; w0 < nb; w0 += kHistMax) {
        const int wn = nb - w0 < kHistMax ? nb - w0 : kHistMax;
        for (int b = lane; b < wn; b += 64) cur[b] = start[c * nb + w0 + b];
        wave_sync_lds();
        for (int64_t base = lo; base < hi; base += 64) {
            const int64_t i = base + lane;
            double th = 0.0;
            int j = -1;
            if (i < hi) {
                th = theta[i];
                j = interval_of(th, theta_cut, h, n_int);
            }
            const bool act = j >= w0 && j < w0 + wn;
            // rank among the lower lanes of the same bucket, and whether no higher
            // lane shares it: compared against every other lane's bucket (lane
            // lane - r after r steps), so the round needs no serial pass per bucket
            const int jm = act ? j : -1 - lane;   // inactive lanes match no one
            int lower = 0;
            bool last = true;
#pragma unroll 8
            for (int r = 1; r < 64; ++r) {
                const bool eq = __shfl(jm, (lane - r) & 63) == jm;
                lower += (eq && r <= lane) ? 1 : 0;
                last = last && !(eq && r > lane);
            }
            unsigned pos = 0u;
            if (act) pos = cur[j - w0] + (unsigned)lower;
            if (act && last) cur[j - w0] = pos + 1u;
            wave_sync_lds();
            if (!act) continue;
            const double ph = phi[i], wi = w[i];
            if (j == n_int) {
                const int64_t p = (int64_t)pos - offsets[n_int];
                pth[p] = th;
                pph[p] = ph;
                pw[p] = wi;
                continue;
            }
            const double x = cos(th);
            const double t = (x - xn[j]) / (xn[j + 1] - xn[j]);
            const double u = 1.0 - t;
            double sp, cp;
            sincos(ph, &sp, &cp);
            double2 *dst = (double2 *)(q + (int64_t)pos * kPointDoubles);
            dst[0] = make_double2(wi * ((2.0 * t + 1.0) * u * u), wi * (t * u * u));
            dst[1] = make_double2(wi * (t * t * (3.0 - 2.0 * t)), wi * (t * t * (t - 1.0)));
            dst[2] = make_double2(ph * kInv2Pi, cp);
            dst[3] = make_double2(sp, 0.0);
        }
        wave_sync_lds();
    }
}

// offsets[b] = sum_{b' < b} counts[b'] for b <= nb (nb buckets), one workgroup
__global__ __launch_bounds__(1024) void scan_kernel(const unsigned *__restrict__ counts, int nb,
                                                    int64_t *__restrict__ offsets) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int chunk = (nb + 1023) / 1024;
    const int lo = tid * chunk < nb ? tid * chunk : nb;
    const int hi = lo + chunk < nb ? lo + chunk : nb;
    int64_t s = 0;
    for (int b = lo; b < hi; ++b) s += counts[b];
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        int64_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    int64_t run = part[tid];
    for (int b = lo; b < hi; ++b) {
        offsets[b] = run;
        run += counts[b];
    }
    if (tid == 1023) offsets[nb] = run;
}

constexpr int kPhaseN = 1024;    // entries of the phase table e^{2 pi i k / kPhaseN}

__global__ void phase_table_kernel(double2 *__restrict__ tab) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kPhaseN) return;
    double s, c;
    sincospi(2.0 * k / kPhaseN, &s, &c);
    tab[k] = make_double2(c, s);
}

constexpr int kBinM = 8;         // orders per binning wave
constexpr int kBinThreads = 64;  // one wave per (interval, kBinM orders)
constexpr int kBinVals = kBinM * 8;   // sums per wave: 4 basis functions x (re, im) per order
constexpr int kBinPts = 2;       // points per lane per iteration

// v[((m n_int) + j) * 4 + a] (complex) for the orders [kBinM p, kBinM (p + 1)) of interval j,
// one wavefront each.  Workgroups go to the 8 XCDs round robin (blockIdx mod 8);
// interval j is given to XCD j mod 8 with all of its passes, so the passes
// reuse that XCD's L2 copy of the interval's points, while neighbouring
// intervals (whose point counts are alike: the mask and the sin(theta) area
// factor vary slowly) spread over all XCDs and keep their loads balanced.  Each
// lane sums a strided subset of the points (loading its next points while it
// sums the current ones); the 64 sums per lane are then added across the wave.
__global__ __launch_bounds__(kBinThreads, 2) void bin_kernel(const double *__restrict__ q, int64_t n_spline,
                                                          const int64_t *__restrict__ offsets, int n_int, int lmax,
                                                          int n_pass, const double2 *__restrict__ ptab,
                                                          double2 *__restrict__ v) {
    const int64_t k = blockIdx.x >> 3;   // position in this XCD's sequence
    const int64_t jj = (int64_t)(blockIdx.x & 7) + 8 * (k / n_pass);
    const int pass = (int)(k % n_pass);
    if (jj >= n_int) return;
    const int j = (int)jj;
    const int m0 = pass * kBinM;
    const int lane = threadIdx.x;
    double acc[kBinM][8];
#pragma unroll
    for (int mm = 0; mm < kBinM; ++mm)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[mm][c] = 0.0;
    const int64_t lo = offsets[j], hi = offsets[j + 1];
    if (hi <= lo) {   // empty interval: its sums are zero
        for (int flat = lane; flat < kBinVals; flat += 64) {
            const int mm = flat >> 3, c = flat & 7;
            if (m0 + mm <= lmax) ((double *)(v + ((int64_t)(m0 + mm) * n_int + j) * 4 + c / 2))[c & 1] = 0.0;
        }
        return;
    }
    // e^{-i m0 phi} from the reduced argument m0 phi / (2 pi) mod 1, taken exactly
    // (two-product of m0 and phi / (2 pi)), so sincospi sees a small argument.
    // Each lane takes kBinPts points per iteration (independent phase chains that
    // the scheduler interleaves); the next iteration's records are loaded
    // (unconditionally, at clamped indices) while the current ones are summed, and
    // a point past the end of the interval contributes with weight 0.
    const double2 *rec = (const double2 *)q;
    double2 nx[kBinPts][4];
    auto fetch = [&](int64_t r) {
#pragma unroll
        for (int b = 0; b < kBinPts; ++b) {
            const int64_t rb = r + b * kBinThreads;
            const int64_t rr = rb < hi ? rb : hi - 1;
#pragma unroll
            for (int a = 0; a < 4; ++a) nx[b][a] = rec[rr * 4 + a];
        }
    };
    // e^{2 pi i k / kPhaseN} in LDS for the phase of every point below
    __shared__ double2 stab[kPhaseN];
    for (int k = lane; k < kPhaseN; k += kBinThreads) stab[k] = ptab[k];
    wave_lds_sync();
    // Per point and pass: e^{-i m0 phi} and e^{-i (m0-1) phi}, then the orders
    // m0 .. m0+7 by the two-term recurrence z_{m+1} = 2 cos(phi) z_m - z_{m-1}
    // (two FMAs per order).  Iterations whose points all lie in the interval
    // skip the masking; the last one (per lane) gives points past the end weight 0.
    auto body = [&](int64_t r, auto tail) {
        double q0[kBinPts], q1[kBinPts], q2[kBinPts], q3[kBinPts], zr[kBinPts], zi[kBinPts], pr[kBinPts],
            pi[kBinPts], tc[kBinPts];
#pragma unroll
        for (int b = 0; b < kBinPts; ++b) {
            const double keep = (!decltype(tail)::value || r + b * kBinThreads < hi) ? 1.0 : 0.0;
            q0[b] = decltype(tail)::value ? keep * nx[b][0].x : nx[b][0].x;
            q1[b] = decltype(tail)::value ? keep * nx[b][0].y : nx[b][0].y;
            q2[b] = decltype(tail)::value ? keep * nx[b][1].x : nx[b][1].x;
            q3[b] = decltype(tail)::value ? keep * nx[b][1].y : nx[b][1].y;
            const double tph = nx[b][2].x, c1 = nx[b][2].y, s1 = nx[b][3].x;
            const double p = (double)m0 * tph;
            const double pe = fma((double)m0, tph, -p);
            const double fr = (p - floor(p)) + pe;      // m0 phi / (2 pi) mod 1, within 2^-52
            // e^{2 pi i fr} = table[k] e^{i eps}: k = floor(kPhaseN fr) (clamped: fr may leave
            // [0, 1) by an ulp), eps = 2 pi (fr - k / kPhaseN) formed from an exact difference,
            // |eps| <= 2 pi / kPhaseN, and cos/sin of eps by their Taylor series to eps^6 / eps^5
            // (the next terms are below 1e-19)
            const double f = fr * (double)kPhaseN;
            int k = (int)floor(f);
            k = k < 0 ? 0 : (k > kPhaseN - 1 ? kPhaseN - 1 : k);
            const double eps = (f - (double)k) * (6.283185307179586476925 / kPhaseN);
            const double e2 = eps * eps;
            const double ce = fma(e2, fma(e2, fma(e2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
            const double se = eps * fma(e2, fma(e2, 1.0 / 120.0, -1.0 / 6.0), 1.0);
            const double2 tk = stab[k];
            const double cm = fma(tk.x, ce, -tk.y * se);
            const double sm = fma(tk.x, se, tk.y * ce);
            zr[b] = cm;           // e^{-i m0 phi}
            zi[b] = -sm;
            // e^{-i (m0 - 1) phi} = (cm - i sm)(c1 + i s1)
            pr[b] = fma(cm, c1, sm * s1);
            pi[b] = fma(cm, s1, -sm * c1);
            tc[b] = 2.0 * c1;
        }
        fetch(r + kBinPts * kBinThreads);
#pragma unroll
        for (int mm = 0; mm < kBinM; ++mm) {
#pragma unroll
            for (int b = 0; b < kBinPts; ++b) {
                acc[mm][0] = fma(q0[b], zr[b], acc[mm][0]);
                acc[mm][1] = fma(q0[b], zi[b], acc[mm][1]);
                acc[mm][2] = fma(q1[b], zr[b], acc[mm][2]);
                acc[mm][3] = fma(q1[b], zi[b], acc[mm][3]);
                acc[mm][4] = fma(q2[b], zr[b], acc[mm][4]);
                acc[mm][5] = fma(q2[b], zi[b], acc[mm][5]);
                acc[mm][6] = fma(q3[b], zr[b], acc[mm][6]);
                acc[mm][7] = fma(q3[b], zi[b], acc[mm][7]);
                if (mm + 1 < kBinM) {
                    const double nr = fma(tc[b], zr[b], -pr[b]);
                    const double ni = fma(tc[b], zi[b], -pi[b]);
                    pr[b] = zr[b];
                    pi[b] = zi[b];
                    zr[b] = nr;
                    zi[b] = ni;
                }
            }
        }
        // Keep the prefetch one iteration ahead: without a use of the loaded
        // registers here the compiler moves the loads into the next iteration,
        // right before their use, and every point waits for L2.
#pragma unroll
        for (int b = 0; b < kBinPts; ++b)
#pragma unroll
            for (int a = 0; a < 4; ++a) asm volatile("" : "+v"(nx[b][a].x), "+v"(nx[b][a].y));
    };
    fetch(lo + lane);
    int64_t r = lo + lane;
    for (; r + (kBinPts - 1) * kBinThreads < hi; r += kBinPts * kBinThreads) body(r, std::false_type{});
    if (r < hi) body(r, std::true_type{});
    // reduce-scatter butterflies over the wave, 64 values at a time: at each step
    // a lane keeps one half of its values and adds its partner's copy of that
    // half; lane k ends with the total of value 64 g + k (= 8 mm + c), always
    // in the same order of additions
#pragma unroll
    for (int g = 0; g < kBinVals / 64; ++g) {
        double vals[64];
#pragma unroll
        for (int k = 0; k < 64; ++k) vals[k] = acc[(64 * g + k) >> 3][k & 7];
#pragma unroll
        for (int half = 32; half >= 1; half >>= 1) {
            const bool upper = (lane & half) != 0;
#pragma unroll
            for (int i = 0; i < half; ++i) {
                const double send = upper ? vals[i] : vals[half + i];
                const double keep = upper ? vals[half + i] : vals[i];
                vals[i] = keep + __shfl_xor(send, half);
            }
        }
        const int flat = 64 * g + lane;
        const int mm = flat >> 3, c = flat & 7;
        const int m = m0 + mm;
        if (m <= lmax) {
            double *dst = (double *)(v + ((int64_t)m * n_int + j) * 4 + c / 2);
            dst[c & 1] = vals[0];
        }
    }
}

// Node weights per (m, n): V_n, F_n = D_n x_n/(1-x_n^2), G_n = D_n/(1-x_n^2) (complex),
// wn[((m n_nodes) + n) * 3 + k]
__global__ void node_weights_kernel(const double2 *__restrict__ v, const double *__restrict__ xn, int n_nodes,
                                    int lmax, double2 *__restrict__ wn) {
    const int64_t total = (int64_t)(lmax + 1) * n_nodes;
    const int n_int = n_nodes - 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(e / n_nodes), n = (int)(e % n_nodes);
        double vr = 0.0, vi = 0.0, dr = 0.0, di = 0.0;
        if (n < n_int) {
            const double2 a0 = v[((int64_t)m * n_int + n) * 4 + 0];
            const double2 a1 = v[((int64_t)m * n_int + n) * 4 + 1];
            const double dx = xn[n + 1] - xn[n];
            vr += a0.x;
            vi += a0.y;
            dr += dx * a1.x;
            di += dx * a1.y;
        }
        if (n > 0) {
            const double2 a2 = v[((int64_t)m * n_int + n - 1) * 4 + 2];
            const double2 a3 = v[((int64_t)m * n_int + n - 1) * 4 + 3];
            const double dx = xn[n] - xn[n - 1];
            vr += a2.x;
            vi += a2.y;
            dr += dx * a3.x;
            di += dx * a3.y;
        }
        const double x = xn[n];
        const double inv = 1.0 / (1.0 - x * x);
        wn[e * 3 + 0] = make_double2(vr, vi);
        wn[e * 3 + 1] = make_double2(dr * x * inv, di * x * inv);
        wn[e * 3 + 2] = make_double2(dr * inv, di * inv);
    }
}

constexpr int kNsKP = 5;            // node sum: nodes per lane
constexpr int kNsLB = 8;            // node sum: degrees per register block
constexpr int kNsMaxSlices = 8;     // node sum: node slices (partial columns)
constexpr int kNsItems = 16384;     // node sum: target (slice, order range) items
// Node-sum tables, one thread per order m.  With y_l = c_m s^m kappa_l E_l
// (c_m = (-1)^m sqrt((2m+1)/4pi prod_{k<=m} (2k-1)/(2k)), the sectoral seed of
// App. A.1), kappa_m = kappa_{m+1} = 1 and kappa_l = b_l kappa_{l-2}, the
// three-term recurrence y_l = a_l x y_{l-1} - b_l y_{l-2} becomes
// E_l = alpha_l x E_{l-1} - E_{l-2} with alpha_l = a_l kappa_{l-1} / kappa_l.
// alpha at coef[segment(m) + l - m] (0 at l = m, where the kernel's general step
// turns its start state (0, -1) into E_m = 1; zero past lmax through the padding),
// scale c_m kappa_l at sig[column_start(m) + l - m].
__global__ void node_tables_kernel(int lmax, double *coef, double *sig) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m > lmax) return;
    double cm2 = (2.0 * m + 1.0) * kInv4Pi;
    for (int k = 1; k <= m; ++k) cm2 *= (2.0 * k - 1.0) / (2.0 * k);
    const double cm = sqrt(cm2) * ((m & 1) ? -1.0 : 1.0);
    double *seg = coef + coef_segment(lmax, m);
    const int64_t col = column_start(lmax, m);
    const int jmax = lmax - m;
    for (int j = 0; j <= jmax + kCoefPad; ++j) seg[j] = 0.0;
    sig[col] = cm;
    double kap2 = 1.0, kap1 = 1.0;   // kappa_{l-2}, kappa_{l-1}
    for (int l = m + 1; l <= lmax; ++l) {
        const double ll = l, mm = m;
        const double a = sqrt((4.0 * ll * ll - 1.0) / (ll * ll - mm * mm));
        double kap;
        if (l == m + 1) {
            kap = 1.0;
        } else {
            const double b = sqrt((2.0 * ll + 1.0) * ((ll - 1.0) * (ll - 1.0) - mm * mm) /
                                  ((2.0 * ll - 3.0) * (ll * ll - mm * mm)));
            kap = b * kap2;
        }
        seg[l - m] = a * kap1 / kap;
        sig[col + (l - m)] = cm * kap;
        kap2 = kap1;
        kap1 = kap;
    }
}

// The node sum as a direct sum over nodes: for order m and degree l,
//     P_l = sum_n s_n^m (V_n - l F_n) E_l(x_n),   Q_l = sum_n s_n^m G_n E_{l-1}(x_n),
// and a_lm = c_m kappa_l P_l + d_l c_m kappa_{l-1} Q_l (= A_l - l F_l + d_l G_{l-1}
// with the sums of the node weights against y_l).  Work decomposition of the
// direct kernels: groups of 64*KP nodes, S node slices, R order ranges, one
// wavefront per (slice, range); s^m as a mantissa with a binary exponent
// advanced by s per order; the chain rescaled every 128 l; the four sums per l
// reduced across lanes in a fixed order into the slice's partial column.
// Per (node, l, m): 8 FP64 operations (chain 2, V - l F 2, P 2, Q 2).
template <int KP, int LB>
__global__ __launch_bounds__(64) void node_sum_wave_kernel(NodeSumArgs a) {
    static_assert(LB % 2 == 0 && 64 % (4 * LB) == 0, "4*LB must divide 64");
    constexpr int V = 4 * LB;
    using R = Red<V, 1>;
    constexpr int P = R::P;
    constexpr int RESCALE_EVERY = ChainRange<double>::every_l / LB;
    constexpr double kAbove = ChainRange<double>::above;

    __shared__ double red[2 * R::BUF];

    const int lane = threadIdx.x;
    const int lmax = a.lmax;
    const int r = blockIdx.x % a.n_ranges;
    const int s = blockIdx.x / a.n_ranges;
    const int m_a = __builtin_amdgcn_readfirstlane(a.range_m[r]);
    const int m_b = __builtin_amdgcn_readfirstlane(a.range_m[r + 1]);
    const const_ptr<double> coef = (const_ptr<double>)(const void *)a.coef;
    const int64_t g_a = (int64_t)s * a.groups / a.n_slices;
    const int64_t g_b = (int64_t)(s + 1) * a.groups / a.n_slices;
    double *part = a.partial + (int64_t)s * 4 * tri_size(lmax);
    const int v = lane / P;
    const int h = lane % P;

    for (int64_t g = g_a; g < g_b; ++g) {
        const bool first = (g == g_a);
        double x[KP], sn[KP], Z[KP];
        int Ze[KP];
        bool live[KP];
#pragma unroll
        for (int t = 0; t < KP; ++t) {
            const int64_t n = g * (64 * KP) + t * 64 + lane;
            live[t] = n < a.n_nodes;
            x[t] = live[t] ? a.xn[n] : 0.0;
            sn[t] = live[t] ? sin(a.thn[n]) : 0.0;
            // s^{m_a} by binary powering with renormalisation
            int eb = 0, e = 0, tt;
            double b = frexp(sn[t], &eb), rr = 1.0;
            for (int k = m_a; k > 0; k >>= 1) {
                if (k & 1) {
                    rr = frexp(rr * b, &tt);
                    e += tt + eb;
                }
                b = frexp(b * b, &tt);
                eb = 2 * eb + tt;
            }
            Z[t] = live[t] ? rr : 0.0;
            Ze[t] = e;
        }
        for (int m = m_a; m < m_b; ++m) {
            const int L = lmax - m + 1;
            const const_ptr<double> cm = coef + coef_segment(lmax, m);
            double *pm = part + 4 * column_start(lmax, m);
            double E[KP], Ep[KP], WVr[KP], WVi[KP], WFr[KP], WFi[KP], WGr[KP], WGi[KP];
            int q[KP];
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                const int64_t n = g * (64 * KP) + t * 64 + lane;
                double2 wv = make_double2(0.0, 0.0), wf = wv, wg = wv;
                if (live[t]) {
                    const double2 *src = a.wn + ((int64_t)m * a.n_nodes + n) * 3;
                    wv = src[0];
                    wf = src[1];
                    wg = src[2];
                }
                q[t] = Ze[t];
                const double z = ldexp_t(Z[t], q[t]);
                WVr[t] = z * wv.x;
                WVi[t] = z * wv.y;
                WFr[t] = z * wf.x;
                WFi[t] = z * wf.y;
                WGr[t] = z * wg.x;
                WGi[t] = z * wg.y;
                E[t] = 0.0;
                Ep[t] = -1.0;
            }
            bool pending = false;
            bool p_owner = false;
            double *p_dst = pm;
            double p_prev = 0.0;
            int cur = 0;
            int blk = 0;
            for (int jb = 0; jb < L; jb += LB, ++blk) {
                const bool owner = (h == 0) && (jb + (v >> 2) < L);
                double *dst = pm + 4 * jb + v;
                double prev = 0.0;
                if (owner && !first) prev = *dst;
                double al[LB];
#pragma unroll
                for (int k = 0; k < LB; ++k) al[k] = cm[jb + k];
                double vals[V];
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    const double ml = -(double)(m + jb + k);
                    double pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0;
#pragma unroll
                    for (int t = 0; t < KP; ++t) {
                        const double en = fma(al[k] * x[t], E[t], -Ep[t]);
                        const double tr = fma(ml, WFr[t], WVr[t]);
                        const double ti = fma(ml, WFi[t], WVi[t]);
                        pr = fma(tr, en, pr);
                        pi = fma(ti, en, pi);
                        qr = fma(WGr[t], E[t], qr);
                        qi = fma(WGi[t], E[t], qi);
                        Ep[t] = E[t];
                        E[t] = en;
                    }
                    vals[4 * k] = pr;
                    vals[4 * k + 1] = pi;
                    vals[4 * k + 2] = qr;
                    vals[4 * k + 3] = qi;
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
                            const int64_t n = g * (64 * KP) + t * 64 + lane;
                            double2 wv = make_double2(0.0, 0.0), wf = wv, wg = wv;
                            if (live[t]) {   // the weights again (re-read: they are not kept)
                                const double2 *src = a.wn + ((int64_t)m * a.n_nodes + n) * 3;
                                wv = src[0];
                                wf = src[1];
                                wg = src[2];
                            }
                            const double z = ldexp_t(Z[t], q[t]);
                            WVr[t] = z * wv.x;
                            WVi[t] = z * wv.y;
                            WFr[t] = z * wf.x;
                            WFi[t] = z * wf.y;
                            WGr[t] = z * wg.x;
                            WGi[t] = z * wg.y;
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
            // next order: Z <- Z s
#pragma unroll
            for (int t = 0; t < KP; ++t) {
                int tt;
                Z[t] = frexp(Z[t] * sn[t], &tt);
                Ze[t] += tt;
            }
        }
    }
}

// a_lm = sig_l P_l + d_l sig_{l-1} Q_l with the compensated slice sums in slice order; one
// workgroup per order m.
__global__ void node_finish_kernel(const double *__restrict__ partial, int n_slices, const double *__restrict__ sig,
                                   int lmax, double *__restrict__ alm) {
    const int m = blockIdx.x;
    const int64_t T = tri_size(lmax);
    const int64_t col = column_start(lmax, m);
    for (int l = m + threadIdx.x; l <= lmax; l += blockDim.x) {
        const int64_t k = col + (l - m);
        double pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0, cpr = 0.0, cpi = 0.0, cqr = 0.0, cqi = 0.0;
        for (int s = 0; s < n_slices; ++s) {
            const double4 v = reinterpret_cast<const double4 *>(partial + (int64_t)s * 4 * T)[k];
            neumaier_add(pr, cpr, v.x);
            neumaier_add(pi, cpi, v.y);
            neumaier_add(qr, cqr, v.z);
            neumaier_add(qi, cqi, v.w);
        }
        pr += cpr;
        pi += cpi;
        qr += cqr;
        qi += cqi;
        double re = sig[k] * pr, im = sig[k] * pi;
        if (l > m) {
            const double ll = l, mm = m;
            const double d = sqrt((2.0 * ll + 1.0) / (2.0 * ll - 1.0) * (ll * ll - mm * mm)) * sig[k - 1];
            re = fma(d, qr, re);
            im = fma(d, qi, im);
        }
        alm[2 * k] = re;
        alm[2 * k + 1] = im;
    }
}

unsigned grid_for(int64_t count, int threads, int64_t cap) {
    int64_t b = (count + threads - 1) / threads;
    if (b < 1) b = 1;
    return (unsigned)(b > cap ? cap : b);
}

}  // namespace

SplinePlan spline_plan(int64_t n, int lmax, int n_nodes) {
    SplinePlan p;
    p.n_int = n_nodes - 1;
    p.n_pass = (lmax + kBinM) / kBinM;
    p.v_doubles = (size_t)(lmax + 1) * p.n_int * 8;
    p.wn_doubles = (size_t)(lmax + 1) * n_nodes * 6;
    p.ns_groups = (n_nodes + 64 * kNsKP - 1) / (64 * kNsKP);
    p.ns_slices = (int)(p.ns_groups < kNsMaxSlices ? p.ns_groups : kNsMaxSlices);
    const int want = kNsItems / p.ns_slices;
    p.ns_ranges = want < lmax + 1 ? (want > 0 ? want : 1) : lmax + 1;
    // node-sum partials (4 per (l, m) and slice), alpha table, scale table
    p.state_doubles = (size_t)p.ns_slices * 4 * (size_t)tri_size(lmax) + (size_t)coef_table_size(lmax) +
                      (size_t)tri_size(lmax) + 2 * (size_t)kPhaseN;   // + the phase table
    // stable sort: chunks of at least kSortChunkMin points, at most kSortChunksMax of them
    int64_t chunks = (n + kSortChunkMin - 1) / kSortChunkMin;
    chunks = chunks < 1 ? 1 : (chunks > kSortChunksMax ? kSortChunksMax : chunks);
    p.sort_chunk = n > 0 ? (n + chunks - 1) / chunks : 1;
    p.sort_chunks = n > 0 ? (int)((n + p.sort_chunk - 1) / p.sort_chunk) : 1;
    return p;
}

hipError_t launch_spline_sort(const double *theta, const double *phi, const double *w, int64_t n, double theta_cut,
                              double h, int n_nodes, const SplinePlan &p, double *xn, double *thn, unsigned *H,
                              unsigned *counts, int64_t *offsets, int64_t *n_polar, double *q, double *pth, double *pph,
                              double *pw, hipStream_t stream) {
    const int nb = n_nodes;   // n_int intervals + the polar bucket
    hipLaunchKernelGGL(nodes_kernel, dim3((n_nodes + 255) / 256), dim3(256), 0, stream, theta_cut, h, n_nodes, xn, thn);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t win_bytes = sizeof(unsigned) * (size_t)(nb < kHistMax ? nb : kHistMax);
    hipLaunchKernelGGL(chunk_hist_kernel, dim3(p.sort_chunks), dim3(64), win_bytes, stream, theta, n, theta_cut, h, nb - 1,
                       p.sort_chunk, H);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(bucket_total_kernel, dim3((nb + 255) / 256), dim3(256), 0, stream, (const unsigned *)H,
                       p.sort_chunks, nb, counts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, stream, (const unsigned *)counts, nb, offsets);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(bucket_start_kernel, dim3((nb + 255) / 256), dim3(256), 0, stream, H, p.sort_chunks, nb,
                       (const int64_t *)offsets, n_polar);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(stable_scatter_kernel, dim3(p.sort_chunks), dim3(64), win_bytes, stream, theta, phi, w, n, theta_cut, h,
                       nb - 1, p.sort_chunk, (const double *)xn, (const int64_t *)offsets, (const unsigned *)H, q, pth,
                       pph, pw);
    return hipGetLastError();
}

hipError_t launch_spline_transform(const SplinePlan &p, const double *q, int64_t n_spline, const int64_t *offsets,
                                   const double *xn, const double *thn, int n_nodes, int lmax, double2 *v,
                                   double2 *wn, double *state, const int *ranges, double *alm, hipStream_t stream,
                                   hipEvent_t bin_start, hipEvent_t bin_stop) {
    double *partial = state;
    double *coef = partial + (size_t)p.ns_slices * 4 * (size_t)tri_size(lmax);
    double *sig = coef + coef_table_size(lmax);
    double *ptab = sig + tri_size(lmax);
    hipLaunchKernelGGL(phase_table_kernel, dim3(kPhaseN / 256), dim3(256), 0, stream, (double2 *)ptab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t per_xcd = (int64_t)((p.n_int + 7) / 8) * p.n_pass;   // units per XCD
    if (bin_start && (e = hipEventRecord(bin_start, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(bin_kernel, dim3((unsigned)(per_xcd * 8)), dim3(kBinThreads), 0, stream, q, n_spline, offsets,
                       p.n_int, lmax, p.n_pass, (const double2 *)ptab, v);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (bin_stop && (e = hipEventRecord(bin_stop, stream)) != hipSuccess) return e;
    const int64_t total = (int64_t)(lmax + 1) * n_nodes;
    hipLaunchKernelGGL(node_weights_kernel, dim3(grid_for(total, 256, 65536)), dim3(256), 0, stream,
                       (const double2 *)v, xn, n_nodes, lmax, wn);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(node_tables_kernel, dim3((lmax + 64) / 64), dim3(64), 0, stream, lmax, coef, sig);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    NodeSumArgs a;
    a.xn = xn;
    a.thn = thn;
    a.n_nodes = n_nodes;
    a.lmax = lmax;
    a.n_ranges = p.ns_ranges;
    a.n_slices = p.ns_slices;
    a.groups = p.ns_groups;
    a.range_m = ranges;
    a.coef = coef;
    a.wn = wn;
    a.partial = partial;
    hipLaunchKernelGGL((node_sum_wave_kernel<kNsKP, kNsLB>), dim3((unsigned)(p.ns_ranges * p.ns_slices)), dim3(64), 0,
                       stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(node_finish_kernel, dim3(lmax + 1), dim3(256), 0, stream, (const double *)partial, p.ns_slices,
                       (const double *)sig, lmax, alm);
    return hipGetLastError();
}

}  // namespace ptalm
