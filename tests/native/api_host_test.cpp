// Host-side checks of the C ABI's validation and planning code (api.hip) built
// with AddressSanitizer and UBSan on the host side, run on the CPU: every call
// here returns before any device work (bad arguments, sizes, plans), so no GPU
// is needed.  Device pointers are fake addresses that are never dereferenced.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ptalm.h"

#define CHECK(c)                                                                       \
    do {                                                                               \
        if (!(c)) {                                                                    \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                              \
        }                                                                              \
    } while (0)

extern "C" int ptalm_plan_m_ranges(int lmax, int R, int *bounds);

static double *fake(uintptr_t a) { return reinterpret_cast<double *>(a); }

static void sizes_and_indices() {
    for (int lmax : {0, 1, 2, 7, 64, 3072, PTALM_LMAX_MAX}) {
        CHECK(ptalm_alm_size(lmax) == (int64_t)(lmax + 1) * (lmax + 2) / 2);
        CHECK(ptalm_alm_index(lmax, lmax, lmax) == ptalm_alm_size(lmax) - 1);
        CHECK(ptalm_alm_index(lmax, 0, 0) == 0);
    }
    CHECK(ptalm_alm_size(-1) == 0 && ptalm_alm_size(PTALM_LMAX_MAX + 1) == 0);
    CHECK(ptalm_alm_index(10, 3, 4) == -1 && ptalm_alm_index(10, 11, 0) == -1 && ptalm_alm_index(-1, 0, 0) == -1);
}

static void m_ranges() {
    for (int lmax : {0, 5, 64, 1000, 3072, PTALM_LMAX_MAX})
        for (int R : {1, 2, 7, 256, 2048}) {
            if (R > lmax + 1) {
                std::vector<int> b(R + 1);
                CHECK(ptalm_plan_m_ranges(lmax, R, b.data()) == PTALM_EINVAL);
                continue;
            }
            std::vector<int> b(R + 1, -7);
            CHECK(ptalm_plan_m_ranges(lmax, R, b.data()) == PTALM_OK);
            CHECK(b[0] == 0 && b[R] == lmax + 1);
            for (int r = 0; r < R; ++r) CHECK(b[r] < b[r + 1]);   // every range holds an order
        }
    CHECK(ptalm_plan_m_ranges(10, 0, nullptr) == PTALM_EINVAL);
}

static void workspace_plans() {
    ptalm_opts o;
    std::memset(&o, 0, sizeof o);
    for (int64_t n : {(int64_t)1, (int64_t)1000, (int64_t)100000000, ((int64_t)1 << 31) + 777})
        for (int lmax : {0, 64, 3072}) {
            const size_t b = ptalm_workspace_bytes(n, lmax, &o);
            CHECK(b > 0 && b % 8 == 0);
            CHECK(b <= (size_t)32 * 16 * (size_t)ptalm_alm_size(lmax));
        }
    CHECK(ptalm_workspace_bytes(-1, 64, &o) == 0 && ptalm_workspace_bytes(10, -1, &o) == 0);
    o.precision = 9;
    CHECK(ptalm_workspace_bytes(10, 64, &o) == 0);
    o.precision = PTALM_BF16X3;
    o.n_weights = 7;
    CHECK(ptalm_workspace_bytes(10, 64, &o) == 0);                  // 16 or 32 weight vectors only
    o.n_weights = 32;
    CHECK(ptalm_workspace_bytes(100000, 512, &o) > 0);
    std::memset(&o, 0, sizeof o);
    o.points_per_lane = 3;                                          // no such kernel variant
    CHECK(ptalm_workspace_bytes(10, 64, &o) == 0);
    std::memset(&o, 0, sizeof o);
    CHECK(ptalm_shear_workspace_bytes(1000, 64, &o) > 0 && ptalm_shear_workspace_bytes(-1, 64, &o) == 0);
    CHECK(ptalm_spline_workspace_bytes(100000, 64, 200) > ptalm_spline_workspace_bytes(1000, 64, 200));
    CHECK(ptalm_spline_workspace_bytes(10, 64, 1) == 0 && ptalm_spline_workspace_bytes(10, 64, 70000) == 0);
    CHECK(ptalm_bandpower_count(100, 2, 10) == 9 && ptalm_bandpower_count(100, 0, 0) <= 0);
}

static void refusals() {
    const uintptr_t a = (uintptr_t)1 << 40;
    ptalm_opts o;
    std::memset(&o, 0, sizeof o);
    CHECK(ptalm_alm_from_points_ex(fake(a), fake(a), fake(a), -1, 64, fake(a), &o, nullptr, 0, nullptr) ==
          PTALM_EINVAL);
    CHECK(std::strlen(ptalm_last_error()) > 0);
    CHECK(ptalm_alm_from_points_ex(fake(a), fake(a), fake(a), 10, 20000, fake(a), &o, nullptr, 0, nullptr) ==
          PTALM_EINVAL);
    CHECK(ptalm_alm_from_points_ex(nullptr, fake(a), fake(a), 10, 64, fake(a), &o, nullptr, 0, nullptr) ==
          PTALM_EINVAL);
    CHECK(ptalm_alm_from_points_ex(fake(a), fake(a), fake(a), 10, 64, nullptr, &o, nullptr, 0, nullptr) ==
          PTALM_EINVAL);
    const size_t need = ptalm_workspace_bytes(100000, 64, &o);
    CHECK(ptalm_alm_from_points_ex(fake(a), fake(a), fake(a), 100000, 64, fake(a), &o, (void *)a, need - 8,
                                   nullptr) == PTALM_EINVAL);           // workspace too small
    CHECK(ptalm_alm_from_points_ex(fake(a), fake(a), fake(a), 100000, 64, fake(a), &o, (void *)(a + 8), need,
                                   nullptr) == PTALM_EINVAL);           // misaligned
    const int64_t T = ptalm_alm_size(10);
    CHECK(ptalm_cl_from_alm(fake(a), 10, fake(a + 8 * (2 * T - 1)), nullptr) == PTALM_EINVAL);   // overlap
    CHECK(ptalm_cross_cl(fake(a), fake(a + 16 * T), 10, fake(a + 16 * T + 8), nullptr) == PTALM_EINVAL);
    CHECK(ptalm_alm_axpy(1.0, fake(a), fake(a + 16), 10, nullptr) == PTALM_EINVAL);
    CHECK(ptalm_fkp_fields(fake(a), fake(a + 16 * T), 10, fake(a), nullptr, nullptr, nullptr) == PTALM_EINVAL);
    CHECK(ptalm_alm_from_points_spline(fake(a), fake(a), fake(a), (int64_t)1 << 33, 64, 100, 0.01, fake(a), nullptr,
                                       nullptr, 0, nullptr) == PTALM_EINVAL);
    CHECK(ptalm_alm_from_points_spline(fake(a), fake(a), fake(a), 10, 64, 100, 2.0, fake(a), nullptr, nullptr, 0,
                                       nullptr) == PTALM_EINVAL);
    CHECK(ptalm_shear_alm_from_points(fake(a), fake(a), fake(a), fake(a), fake(a), 10, 64, nullptr, fake(a), &o,
                                      nullptr) == PTALM_EINVAL);
    CHECK(ptalm_coupling_matrix(nullptr, 10, nullptr, 10, fake(a), nullptr) == PTALM_EINVAL);
    CHECK(ptalm_bandpowers(fake(a), fake(a), nullptr, -1, 100, 0, 0, 0, fake(a), nullptr, nullptr) == PTALM_EINVAL);
    CHECK(ptalm_bandpowers(fake(a), fake(a), nullptr, -1, 100, 2, 10, 1, fake(a), nullptr, nullptr) == PTALM_EINVAL);
    CHECK(ptalm_alm_from_points_noalloc(fake(a), fake(a), fake(a), 10, PTALM_NOALLOC_LMAX_MAX + 1, fake(a),
                                        nullptr) == PTALM_EINVAL);
    CHECK(ptalm_alm_from_points_noalloc(fake(a), fake(a), fake(a), -1, 64, fake(a), nullptr) == PTALM_EINVAL);
    CHECK(ptalm_window_shot_noise(nullptr, 10, nullptr, fake(a), nullptr) == PTALM_EINVAL);
    ptalm_server *s = nullptr;
    CHECK(ptalm_server_create(0, 1 << 20, 0, &s) == PTALM_EINVAL && s == nullptr);
    CHECK(ptalm_server_create(0, 100, 2, &s) == PTALM_EINVAL);
    CHECK(ptalm_server_submit(nullptr, nullptr, nullptr) == PTALM_EINVAL);
    CHECK(std::strlen(ptalm_server_last_error()) > 0);
}

int main() {
    sizes_and_indices();
    m_ranges();
    workspace_plans();
    refusals();
    std::printf("OK\n");
    return 0;
}
