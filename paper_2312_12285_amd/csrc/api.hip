// C ABI of the ptalm library: validation, work plans, scratch, launches.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "ptalm.h"
#include "ptalm_internal.h"

namespace {

thread_local std::string g_error;

// Events of the last timed transform on this thread (created on first use).
struct TimingEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool valid = false;
};
thread_local TimingEvents g_timing;

int fail(int code, const std::string &msg) {
    g_error = msg;
    return code;
}

int fail_hip(hipError_t e, const char *what) {
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return (e == hipErrorOutOfMemory) ? PTALM_ENOMEM : PTALM_EDEVICE;
}

bool lmax_ok(int lmax) { return lmax >= 0 && lmax <= PTALM_LMAX_MAX; }

// ---------------------------------------------------------------------------
// Per-device caches: coefficient tables per lmax, m-range tables per (lmax, R).
// Entries are built synchronously on a private stream and never modified
// afterwards, so any stream may read them.
// ---------------------------------------------------------------------------
std::mutex g_mu;
std::map<std::pair<int, int>, ptalm::Tables> g_tables;          // (device, lmax)
std::map<std::tuple<int, int, int>, int *> g_ranges;            // (device, lmax, R)

std::map<std::pair<int, int>, ptalm::SpinTables> g_spin_tables;  // (device, lmax)

// Kernel choices found by ptalm_autotune, per (device, precision, n_weights,
// lmax); used for every option left at 0 in later calls.
struct Tuned {
    int kp = 0, lb = 0, mode = 0, slices = 0;
};
std::map<std::tuple<int, int, int, int>, Tuned> g_tuned;

int current_device(int *dev) {
    hipError_t e = hipGetDevice(dev);
    return e == hipSuccess ? PTALM_OK : fail_hip(e, "hipGetDevice");
}

int get_tables(int lmax, const ptalm::Tables **out, bool may_build = true) {
    int dev;
    int rc = current_device(&dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_tables.find({dev, lmax});
    if (it != g_tables.end()) {
        *out = &it->second;
        return PTALM_OK;
    }
    if (!may_build) return fail(PTALM_EBUSY, "coefficient tables not prepared (call ptalm_prepare_call before capture)");
    ptalm::Tables t;
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return fail_hip(e, "hipStreamCreate");
    e = ptalm::build_tables(lmax, &t, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    const hipError_t ed = hipStreamDestroy(s);
    if (e == hipSuccess) e = ed;
    if (e != hipSuccess) {
        (void)hipFree(t.coef);
        (void)hipFree(t.coef32);
        (void)hipFree(t.sigma);
        return fail_hip(e, "building coefficient tables");
    }
    auto res = g_tables.emplace(std::make_pair(dev, lmax), t);
    *out = &res.first->second;
    return PTALM_OK;
}

}  // namespace

// Boundaries of R contiguous m ranges of about equal work sum_m (lmax-m+1 + c):
// range r is [b[r], b[r+1]).  Exposed for the host tests (bit-exact coverage).
extern "C" int ptalm_plan_m_ranges(int lmax, int R, int *bounds) {
    if (!lmax_ok(lmax) || R < 1 || R > lmax + 1 || bounds == nullptr) return PTALM_EINVAL;
    const double setup = 8.0;  // per-order cost of forming weights, in l-steps
    std::vector<double> cum(lmax + 2, 0.0);
    for (int m = 0; m <= lmax; ++m) cum[m + 1] = cum[m] + (double)(lmax - m + 1) + setup;
    const double total = cum[lmax + 1];
    bounds[0] = 0;
    int m = 0;
    for (int r = 1; r < R; ++r) {
        const double target = total * r / R;
        while (m < lmax + 1 && cum[m] < target) ++m;
        // at least one order per range: ranges never empty while R <= lmax+1
        int lo = bounds[r - 1] + 1, hi = lmax + 1 - (R - r);
        bounds[r] = std::min(std::max(m, lo), hi);
        m = bounds[r];
    }
    bounds[R] = lmax + 1;
    return PTALM_OK;
}

namespace {

int get_ranges(int lmax, int R, const int **out, bool may_build = true) {
    int dev;
    int rc = current_device(&dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    auto key = std::make_tuple(dev, lmax, R);
    auto it = g_ranges.find(key);
    if (it != g_ranges.end()) {
        *out = it->second;
        return PTALM_OK;
    }
    if (!may_build) return fail(PTALM_EBUSY, "m-range table not prepared (call ptalm_prepare_call before capture)");
    std::vector<int> b(R + 1);
    ptalm_plan_m_ranges(lmax, R, b.data());
    int *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(int) * (R + 1));
    if (e != hipSuccess) return fail_hip(e, "hipMalloc(ranges)");
    e = hipMemcpy(d, b.data(), sizeof(int) * (R + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail_hip(e, "hipMemcpy(ranges)");
    }
    g_ranges[key] = d;
    *out = d;
    return PTALM_OK;
}

// Default kernel variant and decomposition.
constexpr int kDefaultKP = 6;
constexpr int kDefaultLB = 16;
constexpr int kDefaultMode = 3;  // register butterfly stage + pipelined reduction
constexpr int kMixedKP = 8;   // 238 VGPRs: two wavefronts per SIMD
constexpr int kFp32KP = 10;
constexpr int kTargetItems = 65536;  // (slice, range) items: ~32 per resident wavefront (finer items shorten the tail)
constexpr int kMaxSlices = 32;
constexpr int64_t kMaxItems = int64_t(1) << 22;   // workgroups of one launch (x 512 threads < 2^32)

struct Resolved {
    int precision, n_weights, kp, lb, mode, S, R;
    int64_t groups;
};

// Tuned entry for the current device, if ptalm_autotune stored one (no device
// query while the table is empty, so host-only callers never touch HIP).
bool tuned_lookup(int precision, int nw, int lmax, Tuned *t) {
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (g_tuned.empty()) return false;
    }
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_tuned.find(std::make_tuple(dev, precision, nw, lmax));
    if (it == g_tuned.end()) return false;
    *t = it->second;
    return true;
}

int resolve(int64_t n, int lmax, const ptalm_opts *o, Resolved *r) {
    ptalm_opts d;
    memset(&d, 0, sizeof d);
    if (!o) o = &d;
    r->precision = o->precision;
    r->n_weights = o->n_weights > 0 ? o->n_weights : 1;
    if (o->precision != PTALM_FP64 && o->precision != PTALM_MIXED && o->precision != PTALM_FP32 &&
        o->precision != PTALM_BF16X3)
        return fail(PTALM_EINVAL, "bad precision");
    if (o->n_weights < 0 || o->points_per_lane < 0 || o->l_block < 0 || o->n_slices < 0 || o->m_ranges < 0 ||
        o->reduction < 0 || o->reduction > 4)
        return fail(PTALM_EINVAL, "option out of range");
    if (o->n_slices > 65536) return fail(PTALM_EINVAL, "n_slices > 65536");
    if (o->precision == PTALM_BF16X3) {
        if (!ptalm::multi_nw_supported(r->n_weights))
            return fail(PTALM_ENOTSUP, "the split-bf16 MFMA form needs n_weights 16 or 32");
        r->kp = 0;
        r->lb = 0;
        r->mode = 0;
        r->groups = (n + ptalm::kMultiGroup - 1) / ptalm::kMultiGroup;
        Tuned tu;
        const bool tuned = o->n_slices == 0 && tuned_lookup(PTALM_BF16X3, r->n_weights, lmax, &tu);
        const int64_t want = tuned ? tu.slices : (512 + lmax) / (lmax + 1);
        int64_t S = o->n_slices ? o->n_slices : want;
        if (S > std::max<int64_t>(1, r->groups)) S = std::max<int64_t>(1, r->groups);
        if (S * (lmax + 1) > kMaxItems) return fail(PTALM_EINVAL, "n_slices x (lmax+1) work items exceed 2^22");
        r->S = (int)S;
        r->R = lmax + 1;
        return PTALM_OK;
    }
    int def_kp = r->precision == PTALM_FP64 ? kDefaultKP : (r->precision == PTALM_MIXED ? kMixedKP : kFp32KP);
    int def_lb = kDefaultLB, def_mode = kDefaultMode;
    Tuned tu;
    if ((o->points_per_lane == 0 || o->l_block == 0 || o->reduction == 0) &&
        tuned_lookup(r->precision, r->n_weights, lmax, &tu)) {
        def_kp = tu.kp;
        def_lb = tu.lb;
        def_mode = tu.mode;
    }
    r->kp = o->points_per_lane ? o->points_per_lane : def_kp;
    r->lb = o->l_block ? o->l_block : def_lb;
    r->mode = o->reduction ? o->reduction - 1 : def_mode;
    const bool have = r->precision == PTALM_FP64    ? ptalm::fp64_variant_exists(r->kp, r->lb, r->mode)
                      : r->precision == PTALM_MIXED ? ptalm::mixed_variant_exists(r->kp, r->lb, r->mode)
                                                    : ptalm::fp32_variant_exists(r->kp, r->lb, r->mode);
    if (!have) return fail(PTALM_ENOTSUP, "no kernel variant with these points_per_lane / l_block / reduction");
    r->groups = (n + 64 * r->kp - 1) / (64 * r->kp);
    int64_t S = o->n_slices ? o->n_slices : std::min<int64_t>(kMaxSlices, std::max<int64_t>(1, r->groups));
    if (S > std::max<int64_t>(1, r->groups)) S = std::max<int64_t>(1, r->groups);
    r->S = (int)S;
    int R = o->m_ranges ? o->m_ranges : (int)std::max<int64_t>(1, kTargetItems / S);
    if (R > lmax + 1) R = lmax + 1;
    if ((int64_t)S * R > kMaxItems) return fail(PTALM_EINVAL, "n_slices x m_ranges work items exceed 2^22");
    r->R = R;
    return PTALM_OK;
}

// Plan of the no-allocation transform: the default FP64 kernel variant, m ranges
// fixed by lmax alone (one range table per lmax, built by ptalm_prepare), and as
// many point slices (up to kMaxSlices) as the static scratch holds.
int noalloc_ranges(int lmax) { return std::min(lmax + 1, 2048); }

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t partial_bytes(const Resolved &r, int lmax) {
    return sizeof(double) * 2 * (size_t)ptalm::tri_size(lmax) * (size_t)r.S;
}

// multi-weight MFMA scratch: FP32 partials [S][rows][2 NW], then the FP32 weight copy
size_t multi_partial_bytes(const Resolved &r, int lmax) {
    return align256(sizeof(float) * 2 * (size_t)ptalm::multi_rows(lmax) * (size_t)r.n_weights * (size_t)r.S);
}
size_t multi_bytes(const Resolved &r, int64_t n, int lmax) {
    return multi_partial_bytes(r, lmax) + align256(sizeof(float) * (size_t)n * (size_t)r.n_weights);
}

// True when the n1 doubles at a and the n2 doubles at b share memory.
bool overlaps(const double *a, int64_t n1, const double *b, int64_t n2) {
    const uintptr_t a0 = (uintptr_t)a, a1 = a0 + sizeof(double) * (uintptr_t)n1;
    const uintptr_t b0 = (uintptr_t)b, b1 = b0 + sizeof(double) * (uintptr_t)n2;
    return a0 < b1 && b0 < a1;
}

}  // namespace

extern "C" {

int64_t ptalm_alm_size(int lmax) { return lmax_ok(lmax) ? ptalm::tri_size(lmax) : 0; }

int64_t ptalm_alm_index(int lmax, int l, int m) {
    if (!lmax_ok(lmax) || m < 0 || l < m || l > lmax) return -1;
    return ptalm::hp_index(lmax, l, m);
}

const char *ptalm_last_error(void) { return g_error.c_str(); }

int ptalm_last_timing(double *transform_ms) {
    if (transform_ms == nullptr || !g_timing.valid) return fail(PTALM_EINVAL, "no timed call on this thread");
    hipError_t e = hipEventSynchronize(g_timing.stop);
    if (e != hipSuccess) return fail_hip(e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, g_timing.start, g_timing.stop);
    if (e != hipSuccess) return fail_hip(e, "hipEventElapsedTime");
    *transform_ms = ms;
    return PTALM_OK;
}

size_t ptalm_workspace_bytes(int64_t n, int lmax, const ptalm_opts *opts) {
    if (n < 0 || !lmax_ok(lmax)) return 0;
    Resolved r;
    if (resolve(n, lmax, opts, &r)) return 0;
    return r.precision == PTALM_BF16X3 ? multi_bytes(r, n, lmax) : partial_bytes(r, lmax);
}

int ptalm_alm_from_points_ex(const double *theta, const double *phi, const double *w, int64_t n, int lmax,
                             double *alm, const ptalm_opts *opts, void *workspace, size_t ws_bytes,
                             void *stream_) {
    g_error.clear();
    if (n < 0) return fail(PTALM_EINVAL, "n < 0");
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    if (alm == nullptr) return fail(PTALM_EINVAL, "alm is NULL");
    if (n > 0 && (theta == nullptr || phi == nullptr || w == nullptr)) return fail(PTALM_EINVAL, "NULL input");
    Resolved r;
    int rc = resolve(n, lmax, opts, &r);
    if (rc) return rc;
    const size_t need = r.precision == PTALM_BF16X3 ? multi_bytes(r, n, lmax) : partial_bytes(r, lmax);
    if (n > 0 && workspace != nullptr && ws_bytes < need) return fail(PTALM_EINVAL, "workspace too small");
    if (((uintptr_t)workspace & 255) != 0) return fail(PTALM_EINVAL, "workspace not 256-byte aligned");
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t T = ptalm::tri_size(lmax);
    const bool timed = opts != nullptr && opts->timing != 0;
    // Under stream capture nothing may allocate or synchronize: the tables must
    // exist already and the caller must bring the workspace.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cap);
    if (e != hipSuccess) return fail_hip(e, "hipStreamIsCapturing");
    const bool capturing = cap != hipStreamCaptureStatusNone;
    if (capturing && timed) return fail(PTALM_EINVAL, "timing is not available under stream capture");
    if (capturing && n > 0 && workspace == nullptr) return fail(PTALM_EINVAL, "stream capture needs a caller workspace");
    if (n == 0) {
        e = ptalm::launch_zero(alm, 2 * T * r.n_weights, stream);
        return e == hipSuccess ? PTALM_OK : fail_hip(e, "zero kernel launch");
    }
    const ptalm::Tables *tab;
    if ((rc = get_tables(lmax, &tab, !capturing))) return rc;
    const int *ranges = nullptr;
    if (r.precision != PTALM_BF16X3 && (rc = get_ranges(lmax, r.R, &ranges, !capturing))) return rc;

    if (timed) {
        g_timing.valid = false;
        if (!g_timing.start && (e = hipEventCreate(&g_timing.start)) != hipSuccess) return fail_hip(e, "hipEventCreate");
        if (!g_timing.stop && (e = hipEventCreate(&g_timing.stop)) != hipSuccess) return fail_hip(e, "hipEventCreate");
    }
    double *partial = (double *)workspace;
    bool own = false;
    if (partial == nullptr) {
        e = hipMallocAsync((void **)&partial, need, stream);
        if (e != hipSuccess) return fail_hip(e, "hipMallocAsync(scratch)");
        own = true;
    }
    if (r.precision == PTALM_BF16X3) {
        ptalm::MultiArgs ma;
        ma.theta = theta;
        ma.phi = phi;
        ma.w = w;
        ma.partial32 = (float *)partial;
        ma.w32 = (float *)((char *)partial + multi_partial_bytes(r, lmax));
        ma.n = n;
        ma.lmax = lmax;
        ma.n_weights = r.n_weights;
        ma.n_slices = r.S;
        ma.groups = r.groups;
        ma.coef = tab->coef;
        if (timed && (e = hipEventRecord(g_timing.start, stream)) != hipSuccess) rc = fail_hip(e, "hipEventRecord");
        if (rc == PTALM_OK && (e = ptalm::launch_alm_multi(ma, stream)) != hipSuccess)
            rc = fail_hip(e, "multi-weight kernel launch");
        if (rc == PTALM_OK && timed) {
            if ((e = hipEventRecord(g_timing.stop, stream)) != hipSuccess) rc = fail_hip(e, "hipEventRecord");
            else g_timing.valid = true;
        }
        if (rc == PTALM_OK && (e = ptalm::launch_multi_finish(ma, tab->sigma, alm, stream)) != hipSuccess)
            rc = fail_hip(e, "multi-weight finish launch");
        if (own) {
            e = hipFreeAsync(partial, stream);
            if (e != hipSuccess && rc == PTALM_OK) rc = fail_hip(e, "hipFreeAsync(scratch)");
        }
        return rc;
    }
    for (int v = 0; v < r.n_weights && rc == PTALM_OK; ++v) {
        ptalm::AlmArgs a;
        a.theta = theta;
        a.phi = phi;
        a.w = w + (int64_t)v * n;
        a.n = n;
        a.lmax = lmax;
        a.n_ranges = r.R;
        a.n_slices = r.S;
        a.groups = r.groups;
        a.range_m = ranges;
        a.coef = tab->coef;
        a.coef32 = tab->coef32;
        a.partial = partial;
        a.w_stride = n;
        a.n_weights = 1;
        bool supported = true;
        if (timed && v == 0 && (e = hipEventRecord(g_timing.start, stream)) != hipSuccess) {
            rc = fail_hip(e, "hipEventRecord");
            break;
        }
        e = r.precision == PTALM_FP64    ? ptalm::launch_alm_fp64(a, r.kp, r.lb, r.mode, stream, &supported)
            : r.precision == PTALM_MIXED ? ptalm::launch_alm_mixed(a, r.kp, r.lb, r.mode, stream, &supported)
                                         : ptalm::launch_alm_fp32(a, r.kp, r.lb, r.mode, stream, &supported);
        if (timed && v == r.n_weights - 1 && e == hipSuccess && supported) {
            hipError_t e2 = hipEventRecord(g_timing.stop, stream);
            if (e2 != hipSuccess) e = e2;
            else g_timing.valid = true;
        }
        if (!supported) rc = fail(PTALM_ENOTSUP, "kernel variant not compiled");
        else if (e != hipSuccess) rc = fail_hip(e, "transform kernel launch");
        else if ((e = ptalm::launch_reduce_partials(partial, r.S, tab->sigma, lmax, alm + (int64_t)v * 2 * T, stream)) !=
                 hipSuccess)
            rc = fail_hip(e, "reduce kernel launch");
    }
    if (own) {
        e = hipFreeAsync(partial, stream);
        if (e != hipSuccess && rc == PTALM_OK) rc = fail_hip(e, "hipFreeAsync(partial)");
    }
    return rc;
}

int ptalm_alm_from_points(const double *theta, const double *phi, const double *w, int64_t n, int lmax,
                          double *alm, void *stream) {
    return ptalm_alm_from_points_ex(theta, phi, w, n, lmax, alm, nullptr, nullptr, 0, stream);
}

int ptalm_cl_from_alm(const double *alm, int lmax, double *cl, void *stream) {
    g_error.clear();
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    if (alm == nullptr || cl == nullptr) return fail(PTALM_EINVAL, "NULL pointer");
    if (overlaps(cl, lmax + 1, alm, 2 * ptalm::tri_size(lmax))) return fail(PTALM_EINVAL, "cl overlaps alm");
    hipError_t e = ptalm::launch_cl(alm, nullptr, lmax, cl, (hipStream_t)stream);
    return e == hipSuccess ? PTALM_OK : fail_hip(e, "cl kernel launch");
}

int ptalm_cross_cl(const double *alm1, const double *alm2, int lmax, double *cl, void *stream) {
    g_error.clear();
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    if (alm1 == nullptr || alm2 == nullptr || cl == nullptr) return fail(PTALM_EINVAL, "NULL pointer");
    if (overlaps(cl, lmax + 1, alm1, 2 * ptalm::tri_size(lmax)) || overlaps(cl, lmax + 1, alm2, 2 * ptalm::tri_size(lmax)))
        return fail(PTALM_EINVAL, "cl overlaps an input");
    hipError_t e = ptalm::launch_cl(alm1, alm2, lmax, cl, (hipStream_t)stream);
    return e == hipSuccess ? PTALM_OK : fail_hip(e, "cross_cl kernel launch");
}

int ptalm_alm_axpy(double alpha, const double *x, double *y, int lmax, void *stream) {
    g_error.clear();
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    if (x == nullptr || y == nullptr) return fail(PTALM_EINVAL, "NULL pointer");
    if (x != y && overlaps(x, 2 * ptalm::tri_size(lmax), y, 2 * ptalm::tri_size(lmax)))
        return fail(PTALM_EINVAL, "x and y overlap without being the same array");
    hipError_t e = ptalm::launch_axpy(alpha, x, y, 2 * ptalm::tri_size(lmax), (hipStream_t)stream);
    return e == hipSuccess ? PTALM_OK : fail_hip(e, "axpy kernel launch");
}

int ptalm_fkp_fields(const double *alm_data, const double *alm_randoms, int lmax, double *delta, double *window,
                     double *alpha_out, void *stream) {
    g_error.clear();
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    if (alm_data == nullptr || alm_randoms == nullptr) return fail(PTALM_EINVAL, "NULL input");
    const void *outs[3] = {delta, window, alpha_out};
    for (const void *p : outs)
        if (p != nullptr && (p == alm_data || p == alm_randoms)) return fail(PTALM_EINVAL, "output aliases an input");
    hipError_t e = ptalm::launch_fkp(alm_data, alm_randoms, lmax, delta, window, alpha_out, (hipStream_t)stream);
    return e == hipSuccess ? PTALM_OK : fail_hip(e, "fkp kernel launch");
}

int ptalm_window_shot_noise(const double *w, int64_t n, const double *alpha, double *out, void *stream) {
    g_error.clear();
    if (n < 0) return fail(PTALM_EINVAL, "n < 0");
    if (out == nullptr || (n > 0 && w == nullptr)) return fail(PTALM_EINVAL, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    double *partial = nullptr;
    hipError_t e = hipMallocAsync((void **)&partial, sizeof(double) * ptalm::shot_noise_scratch_doubles(), st);
    if (e != hipSuccess) return fail_hip(e, "hipMallocAsync");
    e = ptalm::launch_shot_noise(w, n, alpha, out, partial, st);
    int rc = e == hipSuccess ? PTALM_OK : fail_hip(e, "shot-noise kernel launch");
    e = hipFreeAsync(partial, st);
    if (rc == PTALM_OK && e != hipSuccess) rc = fail_hip(e, "hipFreeAsync");
    return rc;
}

int ptalm_coupling_matrix(const double *Wl, int lmax_w, const double *shot, int lmax, double *M, void *stream_) {
    g_error.clear();
    if (!lmax_ok(lmax) || lmax_w < 0 || lmax_w > 2 * PTALM_LMAX_MAX + 1) return fail(PTALM_EINVAL, "lmax out of range");
    if (Wl == nullptr || M == nullptr) return fail(PTALM_EINVAL, "NULL pointer");
    hipStream_t stream = (hipStream_t)stream_;
    double *scratch = nullptr;
    hipError_t e = hipMallocAsync((void **)&scratch, sizeof(double) * ptalm::coupling_scratch_doubles(lmax), stream);
    if (e != hipSuccess) return fail_hip(e, "hipMallocAsync");
    e = ptalm::launch_coupling(Wl, lmax_w, shot, scratch, lmax, M, stream);
    int rc = e == hipSuccess ? PTALM_OK : fail_hip(e, "coupling kernel launch");
    e = hipFreeAsync(scratch, stream);
    if (rc == PTALM_OK && e != hipSuccess) rc = fail_hip(e, "hipFreeAsync");
    return rc;
}

int ptalm_bandpower_count(int lmax, int lmin, int delta_l) {
    if (!lmax_ok(lmax)) return 0;
    return ptalm::bandpower_count(lmax, lmin, delta_l);
}

int ptalm_bandpowers(const double *cl_hat, const double *M, const double *Wl, int lmax_w, int lmax, int lmin,
                     int delta_l, int mode, double *cb, double *window, void *stream_) {
    g_error.clear();
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    const int nb = ptalm::bandpower_count(lmax, lmin, delta_l);
    if (nb < 1) return fail(PTALM_EINVAL, "no complete bin: need 0 <= lmin <= lmax and delta_l >= 1 within lmax");
    if (nb > 1024) return fail(PTALM_EINVAL, "more than 1024 bins");
    if (mode != 0 && mode != 1) return fail(PTALM_EINVAL, "mode must be 0 (decoupled) or 1 (normalised)");
    if (cl_hat == nullptr || M == nullptr || cb == nullptr) return fail(PTALM_EINVAL, "NULL pointer");
    if (mode == 1 && (Wl == nullptr || lmax_w < 0)) return fail(PTALM_EINVAL, "the normalised convention needs W_l");
    hipStream_t stream = (hipStream_t)stream_;
    double *scratch = nullptr;
    hipError_t e = hipMallocAsync((void **)&scratch, sizeof(double) * ptalm::bandpower_scratch_doubles(lmax, nb), stream);
    if (e != hipSuccess) return fail_hip(e, "hipMallocAsync");
    e = ptalm::launch_bandpowers(cl_hat, M, Wl, lmax_w, lmax, lmin, delta_l, nb, mode, cb, window, scratch, stream);
    int rc = e == hipSuccess ? PTALM_OK : fail_hip(e, "bandpower kernel launch");
    e = hipFreeAsync(scratch, stream);
    if (rc == PTALM_OK && e != hipSuccess) rc = fail_hip(e, "hipFreeAsync");
    return rc;
}

namespace {

// stream-ordered allocations released together (in reverse order) at scope end
struct AsyncAllocs {
    hipStream_t stream;
    std::vector<void *> ptrs;
    explicit AsyncAllocs(hipStream_t s) : stream(s) {}
    hipError_t get(void **p, size_t bytes) {
        *p = nullptr;
        hipError_t e = hipMallocAsync(p, bytes < 256 ? 256 : bytes, stream);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    hipError_t release() {
        hipError_t first = hipSuccess;
        for (auto it = ptrs.rbegin(); it != ptrs.rend(); ++it) {
            hipError_t e = hipFreeAsync(*it, stream);
            if (first == hipSuccess) first = e;
        }
        ptrs.clear();
        return first;
    }
    ~AsyncAllocs() { (void)release(); }   // errors of a late release have no caller to go to
};

}  // namespace

}  // extern "C"

namespace {

// Scratch of the interpolated transform: one buffer cut into 256-byte aligned
// parts (sizes from the upper bound n on both the spline and the polar counts,
// so nothing depends on the device-side split and nothing is read back).
struct SplineScratch {
    size_t xn, thn, H, counts, offsets, npolar, q, pth, pph, pw, v, wn, state, ppart, ptmp, total;
    ptalm::SplinePlan plan;
    Resolved polar;   // plan of the exact sum over the polar points (for n of them at most)
};

int spline_scratch(int64_t n, int lmax, int n_nodes, SplineScratch *s) {
    s->plan = ptalm::spline_plan(n, lmax, n_nodes);
    int rc = resolve(std::max<int64_t>(n, 1), lmax, nullptr, &s->polar);
    if (rc) return rc;
    const int64_t T = ptalm::tri_size(lmax);
    const int nb = n_nodes;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align256(bytes < 256 ? 256 : bytes);
        return at;
    };
    s->xn = take(sizeof(double) * n_nodes);
    s->thn = take(sizeof(double) * n_nodes);
    s->H = take(sizeof(unsigned) * (size_t)s->plan.sort_chunks * nb);
    s->counts = take(sizeof(unsigned) * nb);
    s->offsets = take(sizeof(int64_t) * (nb + 1));
    s->npolar = take(sizeof(int64_t));
    s->q = take(sizeof(double) * 8 * (size_t)n);
    s->pth = take(sizeof(double) * (size_t)n);
    s->pph = take(sizeof(double) * (size_t)n);
    s->pw = take(sizeof(double) * (size_t)n);
    s->v = take(sizeof(double) * s->plan.v_doubles);
    s->wn = take(sizeof(double) * s->plan.wn_doubles);
    s->state = take(sizeof(double) * s->plan.state_doubles);
    s->ppart = take(partial_bytes(s->polar, lmax));
    s->ptmp = take(sizeof(double) * 2 * (size_t)T);
    s->total = off;
    return PTALM_OK;
}

int spline_args_ok(int64_t n, int lmax, int n_nodes) {
    if (n < 0) return fail(PTALM_EINVAL, "n < 0");
    if (n > PTALM_SPLINE_N_MAX) return fail(PTALM_EINVAL, "n above PTALM_SPLINE_N_MAX (32-bit per-interval counters)");
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    if (n_nodes < 2 || n_nodes > PTALM_SPLINE_NODES_MAX) return fail(PTALM_EINVAL, "n_nodes out of range");
    return PTALM_OK;
}

}  // namespace

extern "C" {

size_t ptalm_spline_workspace_bytes(int64_t n, int lmax, int n_nodes) {
    if (n < 0 || n > PTALM_SPLINE_N_MAX || !lmax_ok(lmax) || n_nodes < 2 || n_nodes > PTALM_SPLINE_NODES_MAX) return 0;
    SplineScratch s;
    if (spline_scratch(n, lmax, n_nodes, &s)) return 0;
    return s.total;
}

int ptalm_prepare_spline_call(int64_t n, int lmax, int n_nodes) {
    g_error.clear();
    int rc = spline_args_ok(n, lmax, n_nodes);
    if (rc) return rc;
    SplineScratch s;
    if ((rc = spline_scratch(n, lmax, n_nodes, &s))) return rc;
    const ptalm::Tables *tab;
    const int *ranges;
    if ((rc = get_tables(lmax, &tab))) return rc;
    if ((rc = get_ranges(lmax, s.plan.ns_ranges, &ranges))) return rc;
    return get_ranges(lmax, s.polar.R, &ranges);
}

int ptalm_alm_from_points_spline(const double *theta, const double *phi, const double *w, int64_t n, int lmax,
                                 int n_nodes, double theta_cut, double *alm, const ptalm_opts *opts, void *workspace,
                                 size_t ws_bytes, void *stream_) {
    g_error.clear();
    int rc = spline_args_ok(n, lmax, n_nodes);
    if (rc) return rc;
    if (alm == nullptr || (n > 0 && (theta == nullptr || phi == nullptr || w == nullptr)))
        return fail(PTALM_EINVAL, "NULL pointer");
    const double kPi = 3.141592653589793;
    if (!(theta_cut > 0.0 && theta_cut < 0.5 * kPi)) return fail(PTALM_EINVAL, "theta_cut must be in (0, pi/2)");
    SplineScratch sc;
    if ((rc = spline_scratch(n, lmax, n_nodes, &sc))) return rc;
    if (workspace != nullptr && ws_bytes < sc.total) return fail(PTALM_EINVAL, "workspace too small");
    if (((uintptr_t)workspace & 255) != 0) return fail(PTALM_EINVAL, "workspace not 256-byte aligned");
    hipStream_t stream = (hipStream_t)stream_;
    const bool timed = opts != nullptr && opts->timing != 0;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cap);
    if (e != hipSuccess) return fail_hip(e, "hipStreamIsCapturing");
    const bool capturing = cap != hipStreamCaptureStatusNone;
    if (capturing && timed) return fail(PTALM_EINVAL, "timing is not available under stream capture");
    if (capturing && workspace == nullptr) return fail(PTALM_EINVAL, "stream capture needs a caller workspace");
    const ptalm::Tables *tab;
    const int *ns_ranges, *polar_ranges;
    if ((rc = get_tables(lmax, &tab, !capturing)) || (rc = get_ranges(lmax, sc.plan.ns_ranges, &ns_ranges, !capturing)) ||
        (rc = get_ranges(lmax, sc.polar.R, &polar_ranges, !capturing)))
        return rc;
    if (timed) {
        g_timing.valid = false;
        if (!g_timing.start && (e = hipEventCreate(&g_timing.start)) != hipSuccess) return fail_hip(e, "hipEventCreate");
        if (!g_timing.stop && (e = hipEventCreate(&g_timing.stop)) != hipSuccess) return fail_hip(e, "hipEventCreate");
    }
    char *base = (char *)workspace;
    bool own = false;
    if (base == nullptr) {
        if ((e = hipMallocAsync((void **)&base, sc.total, stream)) != hipSuccess)
            return fail_hip(e, "hipMallocAsync(scratch)");
        own = true;
    }
    const double h = (kPi - 2.0 * theta_cut) / (n_nodes - 1);
    const int64_t T = ptalm::tri_size(lmax);
    double *xn = (double *)(base + sc.xn), *thn = (double *)(base + sc.thn);
    int64_t *offsets = (int64_t *)(base + sc.offsets), *n_polar = (int64_t *)(base + sc.npolar);
    double *q = (double *)(base + sc.q);
    double *pth = (double *)(base + sc.pth), *pph = (double *)(base + sc.pph), *pw = (double *)(base + sc.pw);
    double *ptmp = (double *)(base + sc.ptmp);
    // points in interval order (stable), polar points apart; the polar count stays on the device
    e = ptalm::launch_spline_sort(theta, phi, w, n, theta_cut, h, n_nodes, sc.plan, xn, thn, (unsigned *)(base + sc.H),
                                  (unsigned *)(base + sc.counts), offsets, n_polar, q, pth, pph, pw, stream);
    if (e != hipSuccess) rc = fail_hip(e, "spline sort kernels");
    if (rc == PTALM_OK &&
        (e = ptalm::launch_spline_transform(sc.plan, q, n, offsets, xn, thn, n_nodes, lmax, (double2 *)(base + sc.v),
                                            (double2 *)(base + sc.wn), (double *)(base + sc.state), ns_ranges, alm,
                                            stream, timed ? g_timing.start : nullptr,
                                            timed ? g_timing.stop : nullptr)) != hipSuccess)
        rc = fail_hip(e, "spline transform kernels");
    if (rc == PTALM_OK && timed) g_timing.valid = true;
    if (rc == PTALM_OK && n > 0) {
        // the polar caps by the exact sum over the device-side count of polar points
        // (planned for n of them), added to the interpolated part
        ptalm::AlmArgs a;
        a.theta = pth;
        a.phi = pph;
        a.w = pw;
        a.n = n;
        a.lmax = lmax;
        a.n_ranges = sc.polar.R;
        a.n_slices = sc.polar.S;
        a.groups = sc.polar.groups;
        a.range_m = polar_ranges;
        a.coef = tab->coef;
        a.coef32 = tab->coef32;
        a.partial = (double *)(base + sc.ppart);
        a.w_stride = n;
        a.n_weights = 1;
        a.n_dev = n_polar;
        bool supported = true;
        e = ptalm::launch_alm_fp64(a, sc.polar.kp, sc.polar.lb, sc.polar.mode, stream, &supported);
        if (!supported) rc = fail(PTALM_ENOTSUP, "kernel variant not compiled");
        else if (e != hipSuccess) rc = fail_hip(e, "polar transform launch");
        else if ((e = ptalm::launch_reduce_partials(a.partial, sc.polar.S, tab->sigma, lmax, ptmp, stream)) != hipSuccess)
            rc = fail_hip(e, "polar reduce launch");
        else if ((e = ptalm::launch_axpy(1.0, ptmp, alm, 2 * T, stream)) != hipSuccess)
            rc = fail_hip(e, "axpy");
    }
    if (own) {
        e = hipFreeAsync(base, stream);
        if (rc == PTALM_OK && e != hipSuccess) rc = fail_hip(e, "hipFreeAsync(scratch)");
    }
    return rc;
}

namespace {

int get_spin_tables(int lmax, const ptalm::SpinTables **out) {
    int dev;
    int rc = current_device(&dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_spin_tables.find({dev, lmax});
    if (it != g_spin_tables.end()) {
        *out = &it->second;
        return PTALM_OK;
    }
    ptalm::SpinTables t;
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return fail_hip(e, "hipStreamCreate");
    e = ptalm::build_spin_tables(lmax, &t, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    const hipError_t ed = hipStreamDestroy(s);
    if (e == hipSuccess) e = ed;
    if (e != hipSuccess) {
        (void)hipFree(t.coef);
        (void)hipFree(t.sigma);
        return fail_hip(e, "building spin tables");
    }
    auto res = g_spin_tables.emplace(std::make_pair(dev, lmax), t);
    *out = &res.first->second;
    return PTALM_OK;
}

// Default spin kernels: two spins per wavefront (reduction option 1) and one spin per
// wavefront (option 2); kSpinSingle picks the default form.
constexpr int kSpinKP = 4;
constexpr int kSpinLB = 8;
constexpr int kSpinSingleKP = 6;
constexpr int kSpinSingleLB = 8;
constexpr bool kSpinSingle = false;

struct SpinResolved {
    int kp, lb, S, R;
    bool single;
    int64_t groups;
};

int spin_resolve(int64_t n, int lmax, const ptalm_opts *o, SpinResolved *r) {
    ptalm_opts d;
    memset(&d, 0, sizeof d);
    if (!o) o = &d;
    if (o->n_weights < 0 || o->points_per_lane < 0 || o->l_block < 0 || o->n_slices < 0 || o->m_ranges < 0)
        return fail(PTALM_EINVAL, "option out of range");
    if (o->precision != PTALM_FP64) return fail(PTALM_ENOTSUP, "the shear transform is FP64 only");
    if (o->n_weights > 1) return fail(PTALM_ENOTSUP, "the shear transform takes one weight vector");
    if (o->n_slices > 65536) return fail(PTALM_EINVAL, "n_slices > 65536");
    if (o->reduction < 0 || o->reduction > 2) return fail(PTALM_EINVAL, "shear reduction option must be 0, 1 or 2");
    r->single = o->reduction ? o->reduction == 2 : kSpinSingle;
    r->kp = o->points_per_lane ? o->points_per_lane : (r->single ? kSpinSingleKP : kSpinKP);
    r->lb = o->l_block ? o->l_block : (r->single ? kSpinSingleLB : kSpinLB);
    if (!ptalm::spin_variant_exists(r->kp, r->lb, r->single))
        return fail(PTALM_ENOTSUP, "no spin kernel variant with these points_per_lane / l_block");
    r->groups = (n + 64 * r->kp - 1) / (64 * r->kp);
    const int64_t gmax = std::max<int64_t>(1, r->groups);
    int64_t S = o->n_slices ? o->n_slices : std::min<int64_t>(kMaxSlices, gmax);
    if (S > gmax) S = gmax;  // every slice holds at least one group, so every partial is written
    r->S = (int)S;
    int R = o->m_ranges ? o->m_ranges : (int)std::max<int64_t>(1, kTargetItems / S);
    if (R > lmax + 1) R = lmax + 1;
    if ((int64_t)S * R > kMaxItems) return fail(PTALM_EINVAL, "n_slices x m_ranges work items exceed 2^22");
    r->R = R;
    return PTALM_OK;
}

}  // namespace

size_t ptalm_shear_workspace_bytes(int64_t n, int lmax, const ptalm_opts *opts) {
    if (n < 0 || !lmax_ok(lmax)) return 0;
    SpinResolved r;
    if (spin_resolve(n, lmax, opts, &r)) return 0;
    return sizeof(double) * 4 * (size_t)ptalm::tri_size(lmax) * (size_t)r.S;
}

int ptalm_shear_alm_from_points(const double *theta, const double *phi, const double *w, const double *g1,
                                const double *g2, int64_t n, int lmax, double *alm_E, double *alm_B,
                                const ptalm_opts *opts, void *stream_) {
    g_error.clear();
    if (n < 0) return fail(PTALM_EINVAL, "n < 0");
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    if (alm_E == nullptr || alm_B == nullptr) return fail(PTALM_EINVAL, "alm_E or alm_B is NULL");
    if (n > 0 && (theta == nullptr || phi == nullptr || w == nullptr || g1 == nullptr || g2 == nullptr))
        return fail(PTALM_EINVAL, "NULL input");
    SpinResolved r;
    int rc = spin_resolve(n, lmax, opts, &r);
    if (rc) return rc;
    hipStream_t stream = (hipStream_t)stream_;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cap);
    if (e != hipSuccess) return fail_hip(e, "hipStreamIsCapturing");
    if (cap != hipStreamCaptureStatusNone) return fail(PTALM_EINVAL, "the shear transform is not capturable");
    const int64_t T = ptalm::tri_size(lmax);
    if (n == 0) {
        if ((e = ptalm::launch_zero(alm_E, 2 * T, stream)) != hipSuccess ||
            (e = ptalm::launch_zero(alm_B, 2 * T, stream)) != hipSuccess)
            return fail_hip(e, "zero kernel launch");
        return PTALM_OK;
    }
    const ptalm::SpinTables *tab;
    if ((rc = get_spin_tables(lmax, &tab))) return rc;
    const int *ranges;
    if ((rc = get_ranges(lmax, r.R, &ranges))) return rc;
    const bool timed = opts != nullptr && opts->timing != 0;
    if (timed) {
        g_timing.valid = false;
        if (!g_timing.start && (e = hipEventCreate(&g_timing.start)) != hipSuccess) return fail_hip(e, "hipEventCreate");
        if (!g_timing.stop && (e = hipEventCreate(&g_timing.stop)) != hipSuccess) return fail_hip(e, "hipEventCreate");
    }
    AsyncAllocs mem(stream);
    double *partial;
    if ((e = mem.get((void **)&partial, sizeof(double) * 4 * (size_t)T * (size_t)r.S)) != hipSuccess)
        return fail_hip(e, "hipMallocAsync(partial)");
    ptalm::SpinArgs a;
    a.theta = theta;
    a.phi = phi;
    a.w = w;
    a.g1 = g1;
    a.g2 = g2;
    a.n = n;
    a.lmax = lmax;
    a.n_ranges = r.R;
    a.n_slices = r.S;
    a.groups = r.groups;
    a.range_m = ranges;
    a.coef = tab->coef;
    a.partial = partial;
    bool supported = true;
    if (timed && (e = hipEventRecord(g_timing.start, stream)) != hipSuccess) return fail_hip(e, "hipEventRecord");
    if ((e = ptalm::launch_spin(a, r.kp, r.lb, r.single, stream, &supported)) != hipSuccess) return fail_hip(e, "spin kernel launch");
    if (!supported) return fail(PTALM_ENOTSUP, "spin kernel variant not compiled");
    if (timed) {
        if ((e = hipEventRecord(g_timing.stop, stream)) != hipSuccess) return fail_hip(e, "hipEventRecord");
        g_timing.valid = true;
    }
    if ((e = ptalm::launch_spin_finish(partial, r.S, tab->sigma, lmax, alm_E, alm_B, stream)) != hipSuccess)
        return fail_hip(e, "spin finish launch");
    if ((e = mem.release()) != hipSuccess) return fail_hip(e, "hipFreeAsync");
    return PTALM_OK;
}

int ptalm_prepare(int lmax) {
    g_error.clear();
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    const ptalm::Tables *tab;
    int rc = get_tables(lmax, &tab);
    if (rc || lmax > PTALM_NOALLOC_LMAX_MAX) return rc;
    // set-up of the no-allocation form: its range table and its scratch address
    const int *ranges;
    if ((rc = get_ranges(lmax, noalloc_ranges(lmax), &ranges))) return rc;
    void *sp;
    hipError_t e = ptalm::noalloc_scratch(&sp);
    return e == hipSuccess ? PTALM_OK : fail_hip(e, "hipGetSymbolAddress(scratch)");
}

int ptalm_alm_from_points_noalloc(const double *theta, const double *phi, const double *w, int64_t n, int lmax,
                                  double *alm, void *stream_) {
    g_error.clear();
    if (n < 0) return fail(PTALM_EINVAL, "n < 0");
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    if (lmax > PTALM_NOALLOC_LMAX_MAX)
        return fail(PTALM_EINVAL, "lmax above PTALM_NOALLOC_LMAX_MAX (4094): one slice of partials, 16*T bytes, "
                                  "must fit the 128 MiB static scratch");
    if (alm == nullptr) return fail(PTALM_EINVAL, "alm is NULL");
    if (n > 0 && (theta == nullptr || phi == nullptr || w == nullptr)) return fail(PTALM_EINVAL, "NULL input");
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t T = ptalm::tri_size(lmax);
    hipError_t e;
    if (n == 0) {
        e = ptalm::launch_zero(alm, 2 * T, stream);
        return e == hipSuccess ? PTALM_OK : fail_hip(e, "zero kernel launch");
    }
    const ptalm::Tables *tab;
    const int *ranges;
    const int R = noalloc_ranges(lmax);
    if (get_tables(lmax, &tab, false) != PTALM_OK || get_ranges(lmax, R, &ranges, false) != PTALM_OK)
        return fail(PTALM_EBUSY, "not set up for this lmax on this device: call ptalm_prepare(lmax) first");
    void *sp = nullptr;
    if ((e = ptalm::noalloc_scratch(&sp)) != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    const int64_t groups = (n + 64 * kDefaultKP - 1) / (64 * kDefaultKP);
    const int64_t fit = (int64_t)(PTALM_NOALLOC_SCRATCH_BYTES / (sizeof(double) * 2 * (size_t)T));
    const int S = (int)std::min<int64_t>(std::min<int64_t>(kMaxSlices, groups), fit);
    ptalm::AlmArgs a;
    a.theta = theta;
    a.phi = phi;
    a.w = w;
    a.n = n;
    a.lmax = lmax;
    a.n_ranges = R;
    a.n_slices = S;
    a.groups = groups;
    a.range_m = ranges;
    a.coef = tab->coef;
    a.coef32 = tab->coef32;
    a.partial = (double *)sp;   // the static scratch: S x 2T doubles, every one written before it is read
    a.w_stride = n;
    a.n_weights = 1;
    bool supported = true;
    e = ptalm::launch_alm_fp64(a, kDefaultKP, kDefaultLB, kDefaultMode, stream, &supported);
    if (!supported) return fail(PTALM_ENOTSUP, "default kernel variant not compiled");
    if (e != hipSuccess) return fail_hip(e, "transform kernel launch");
    e = ptalm::launch_reduce_partials(a.partial, S, tab->sigma, lmax, alm, stream);
    return e == hipSuccess ? PTALM_OK : fail_hip(e, "reduce kernel launch");
}

int ptalm_prepare_call(int64_t n, int lmax, const ptalm_opts *opts) {
    g_error.clear();
    if (n < 0) return fail(PTALM_EINVAL, "n < 0");
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    Resolved r;
    int rc = resolve(n, lmax, opts, &r);
    if (rc) return rc;
    const ptalm::Tables *tab;
    if ((rc = get_tables(lmax, &tab))) return rc;
    const int *ranges;
    if (r.precision != PTALM_BF16X3 && (rc = get_ranges(lmax, r.R, &ranges))) return rc;
    return PTALM_OK;
}

int ptalm_autotune(const double *theta, const double *phi, const double *w, int64_t n, int lmax, int precision,
                   int n_weights, ptalm_opts *best, void *stream_) {
    g_error.clear();
    if (n <= 0) return fail(PTALM_EINVAL, "autotune needs n > 0");
    if (!lmax_ok(lmax)) return fail(PTALM_EINVAL, "lmax out of range");
    if (theta == nullptr || phi == nullptr || w == nullptr || best == nullptr) return fail(PTALM_EINVAL, "NULL pointer");
    if (precision < PTALM_FP64 || precision > PTALM_BF16X3) return fail(PTALM_EINVAL, "bad precision");
    if (n_weights < 1) return fail(PTALM_EINVAL, "n_weights < 1");
    hipStream_t stream = (hipStream_t)stream_;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cap);
    if (e != hipSuccess) return fail_hip(e, "hipStreamIsCapturing");
    if (cap != hipStreamCaptureStatusNone) return fail(PTALM_EINVAL, "autotune cannot run under stream capture");

    // candidates: every compiled kernel variant (VALU forms) or slice count (MFMA form)
    std::vector<ptalm_opts> cands;
    std::vector<int> seen_slices;
    auto base = [&]() {
        ptalm_opts o;
        memset(&o, 0, sizeof o);
        o.precision = precision;
        o.n_weights = n_weights;
        return o;
    };
    if (precision == PTALM_BF16X3) {
        for (int S : {1, 2, 4, 8}) {
            ptalm_opts o = base();
            o.n_slices = S;
            Resolved r;
            int rc = resolve(n, lmax, &o, &r);
            if (rc) return rc;
            if (std::find(seen_slices.begin(), seen_slices.end(), r.S) != seen_slices.end()) continue;
            seen_slices.push_back(r.S);
            o.n_slices = r.S;
            cands.push_back(o);
        }
    } else {
        int v[64][3];
        const int k = std::min(64, ptalm::list_variants(precision, v, 64));
        for (int i = 0; i < k; ++i) {
            ptalm_opts o = base();
            o.points_per_lane = v[i][0];
            o.l_block = v[i][1];
            o.reduction = v[i][2] + 1;
            cands.push_back(o);
        }
    }
    size_t ws = 0;
    for (const ptalm_opts &o : cands) {
        Resolved r;
        int rc = resolve(n, lmax, &o, &r);
        if (rc) return rc;
        ws = std::max(ws, r.precision == PTALM_BF16X3 ? multi_bytes(r, n, lmax) : partial_bytes(r, lmax));
    }
    const size_t out_bytes = sizeof(double) * 2 * (size_t)ptalm::tri_size(lmax) * (size_t)n_weights;
    void *buf = nullptr;
    if ((e = hipMallocAsync(&buf, align256(out_bytes) + ws, stream)) != hipSuccess) return fail_hip(e, "hipMallocAsync");
    double *out = (double *)buf;
    void *wsp = (char *)buf + align256(out_bytes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PTALM_OK;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) rc = fail_hip(e, "hipEventCreate");
    float best_ms = -1.f;
    ptalm_opts pick = cands.empty() ? base() : cands[0];
    for (size_t c = 0; c < cands.size() && rc == PTALM_OK; ++c) {
        // one untimed call (first touch of code and tables), then one timed call
        rc = ptalm_alm_from_points_ex(theta, phi, w, n, lmax, out, &cands[c], wsp, ws, stream);
        if (rc) break;
        if ((e = hipEventRecord(e0, stream)) != hipSuccess) { rc = fail_hip(e, "hipEventRecord"); break; }
        rc = ptalm_alm_from_points_ex(theta, phi, w, n, lmax, out, &cands[c], wsp, ws, stream);
        if (rc) break;
        if ((e = hipEventRecord(e1, stream)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
            rc = fail_hip(e, "timing event");
            break;
        }
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { rc = fail_hip(e, "hipEventElapsedTime"); break; }
        if (best_ms < 0.f || ms < best_ms) {
            best_ms = ms;
            pick = cands[c];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    e = hipFreeAsync(buf, stream);
    if (rc == PTALM_OK && e != hipSuccess) rc = fail_hip(e, "hipFreeAsync");
    if (rc) return rc;
    int dev;
    if ((rc = current_device(&dev))) return rc;
    Tuned t;
    t.kp = pick.points_per_lane;
    t.lb = pick.l_block;
    t.mode = pick.reduction > 0 ? pick.reduction - 1 : 0;
    t.slices = pick.n_slices;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_tuned[std::make_tuple(dev, precision, n_weights, lmax)] = t;
    }
    *best = pick;
    return PTALM_OK;
}

int ptalm_release_cache(void) {
    g_error.clear();
    std::lock_guard<std::mutex> lock(g_mu);
    hipError_t first = hipSuccess;
    auto release = [&](void *p) {
        const hipError_t e = hipFree(p);
        if (first == hipSuccess) first = e;
    };
    for (auto &kv : g_tables) {
        release(kv.second.coef);
        release(kv.second.coef32);
        release(kv.second.sigma);
    }
    g_tables.clear();
    for (auto &kv : g_spin_tables) {
        release(kv.second.coef);
        release(kv.second.sigma);
    }
    g_spin_tables.clear();
    for (auto &kv : g_ranges) release(kv.second);
    g_ranges.clear();
    g_tuned.clear();
    const hipError_t ec = ptalm::release_coupling_tables();
    if (first == hipSuccess) first = ec;
    return first == hipSuccess ? PTALM_OK : fail_hip(first, "hipFree (release_cache)");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Request-server support: one transform planned exactly as
// ptalm_alm_from_points_ex(opts = {precision}) plans it, launched in chunks of
// point slices and then the second pass.  A slice's partial is computed by the
// same work items whichever launch runs them, so the result is bitwise that of
// the single call.
// ---------------------------------------------------------------------------
namespace ptalm {

int sliced_slice_count(int64_t n, int lmax, int precision) {
    if (n < 0 || !lmax_ok(lmax)) return fail(PTALM_EINVAL, "bad n or lmax");
    ptalm_opts o;
    memset(&o, 0, sizeof o);
    o.precision = precision;
    o.n_weights = 1;
    Resolved r;
    const int rc = resolve(n, lmax, &o, &r);
    return rc ? rc : r.S;
}

int plan_sliced(const double *theta, const double *phi, const double *w, int64_t n, int lmax, int precision,
                double *partial, SlicedCall *c) {
    g_error.clear();
    if (n <= 0 || !lmax_ok(lmax)) return fail(PTALM_EINVAL, "bad n or lmax");
    if (precision != PTALM_FP64 && precision != PTALM_MIXED && precision != PTALM_FP32)
        return fail(PTALM_EINVAL, "sliced calls take the vector forms");
    ptalm_opts o;
    memset(&o, 0, sizeof o);
    o.precision = precision;
    o.n_weights = 1;
    Resolved r;
    int rc = resolve(n, lmax, &o, &r);
    if (rc) return rc;
    const Tables *tab;
    const int *ranges;
    if ((rc = get_tables(lmax, &tab)) || (rc = get_ranges(lmax, r.R, &ranges))) return rc;
    AlmArgs &a = c->a;
    a = AlmArgs();
    a.theta = theta;
    a.phi = phi;
    a.w = w;
    a.n = n;
    a.lmax = lmax;
    a.n_ranges = r.R;
    a.n_slices = r.S;
    a.groups = r.groups;
    a.range_m = ranges;
    a.coef = tab->coef;
    a.coef32 = tab->coef32;
    a.partial = partial;
    a.w_stride = n;
    a.n_weights = 1;
    c->precision = precision;
    c->kp = r.kp;
    c->lb = r.lb;
    c->mode = r.mode;
    c->sigma = tab->sigma;
    return PTALM_OK;
}

hipError_t launch_sliced(const SlicedCall &c, int s0, int s1, hipStream_t stream) {
    if (s0 < 0 || s1 > c.a.n_slices || s0 >= s1) return hipErrorInvalidValue;
    AlmArgs a = c.a;
    a.slice_base = s0;
    a.slice_count = s1 - s0;
    bool supported = true;
    const hipError_t e = c.precision == PTALM_FP64    ? launch_alm_fp64(a, c.kp, c.lb, c.mode, stream, &supported)
                         : c.precision == PTALM_MIXED ? launch_alm_mixed(a, c.kp, c.lb, c.mode, stream, &supported)
                                                      : launch_alm_fp32(a, c.kp, c.lb, c.mode, stream, &supported);
    return supported ? e : hipErrorInvalidKernelFile;
}

hipError_t launch_sliced_finish(const SlicedCall &c, double *alm, hipStream_t stream) {
    return launch_reduce_partials(c.a.partial, c.a.n_slices, c.sigma, c.a.lmax, alm, stream);
}

}  // namespace ptalm
