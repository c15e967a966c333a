// Drives the library's host-only code (pic_host.cpp: parameter validation, workspace
// layouts, the host input check) over many valid and invalid parameter sets; built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py, so any
// out-of-bounds access, overflow or other undefined behaviour ends the run with an error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "pic.h"

namespace {

std::mt19937_64 rng(12345);

template <typename T, size_t N> T pick(const T (&a)[N]) { return a[rng() % N]; }

int failures = 0;

void expect(bool ok, const char *what, long long k)
{
    if (!ok) {
        std::printf("FAILED: %s (case %lld)\n", what, k);
        ++failures;
    }
}

}  // namespace

int main()
{
    const double inf = std::numeric_limits<double>::infinity();
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const int32_t i32[] = {0, 1, 2, 3, 4, 5, 7, 64, 512, 697, 698, 1842, 1843, 2254, 2255,
                           100000, -1, std::numeric_limits<int32_t>::max(),
                           std::numeric_limits<int32_t>::min()};
    const int64_t i64[] = {1, 2, 63, 1000, 100000, 10000000, (int64_t)1 << 40,
                           ((int64_t)1 << 40) + 1, 0, -5, std::numeric_limits<int64_t>::max()};
    const double f64[] = {10.0, 0.05, 1.0, 4 * M_PI, 1e-300, 1e300, 0.0, -1.0, nan, inf};
    long long accepted = 0;
    for (long long k = 0; k < 40000; ++k) {
        pic_params p;
        std::memset(&p, 0, sizeof p);
        p.abi_version = (k % 50 == 0) ? 7 : PIC_ABI_VERSION;
        const int32_t nvs[] = {1, 3, 1, 3, 2, 0};
        p.nv = pick(nvs);
        const int32_t schemes[] = {0, 1, 2, 3, 4, 1, 5, -1};
        p.scheme = pick(schemes);
        const int32_t orders[] = {1, 2, 1, 2, 0, 3};
        p.shape_order = pick(orders);
        p.n_particles = pick(i64);
        p.n_cells = (k % 3) ? (int32_t)(3 + rng() % 600) : pick(i32);
        const int32_t rebins[] = {0, 0, 0, 1, 5, -1};
        p.rebin_every = pick(rebins);
        p.length = (k % 4) ? 10.0 : pick(f64);
        p.dt = (k % 4) ? 0.1 : pick(f64);
        p.c = (k % 4) ? 1.0 : pick(f64);
        for (int i = 0; i < 3; ++i)
            p.b_ext[i] = (k % 5) ? 0.5 * i : pick(f64);
        p.flags = (uint32_t)(rng() % 64);
        if (k % 2)
            p.flags &= ~(uint32_t)PIC_F_DETERMINISTIC;
        const int32_t threads[] = {0, 0, 64, 256, 1024, 100, 2048, -64};
        p.block_threads = pick(threads);
        const int32_t grids[] = {0, 0, 1, 256, 8192, 9000, -1};
        p.grid_blocks = pick(grids);
        const int32_t modes[] = {0, 0, 1, 2, 3, 4, 5, -1};
        p.deposit_mode = pick(modes);
        const int32_t recs[] = {0, 0, 1, 4096, -1, 1 << 20};
        p.record_capacity = pick(recs);
        p.reserved = (k % 97 == 0) ? 1 : 0;
        if (k % 2 == 0) {
            // mostly valid: small runs of every scheme, whose inputs are then checked
            p.abi_version = PIC_ABI_VERSION;
            p.scheme = (int32_t)(rng() % 5);
            p.nv = (p.scheme == PIC_EMEC_LI || p.scheme == PIC_EMEC_PSATD || rng() % 2) ? 3 : 1;
            p.shape_order = 1 + (int32_t)(rng() % 2);
            p.n_particles = 1 + (int64_t)(rng() % 2000);
            p.n_cells = 2 * p.shape_order + 1 + (int32_t)(rng() % 300);
            p.length = 10.0;
            p.dt = 0.1;
            p.c = 1.0;
            p.flags = (p.scheme == PIC_STANDARD ? PIC_F_INIT_GAUSS : 0) | (uint32_t)(rng() % 4);
            p.rebin_every = (rng() % 4 == 0) ? 3 : 0;
            p.deposit_mode = p.rebin_every ? 2 : 0;
            p.block_threads = 0;
            p.grid_blocks = 0;
            p.record_capacity = 0;
            p.reserved = 0;
        }

        const int rc = pic_validate_params(&p);
        const size_t ws = pic_workspace_size(&p);
        expect((rc == PIC_OK) == (ws > 0), "workspace size is nonzero exactly when valid", k);
        expect(rc == PIC_OK || rc == PIC_EINVAL || rc == PIC_EUNSUPPORTED, "status", k);
        if (rc != PIC_OK || p.n_particles > 2000 || p.n_cells > 600)
            continue;
        ++accepted;
        // host input check on small finite arrays, then with one non-finite value
        std::vector<double> x(p.n_particles, 0.5), v((size_t)p.nv * p.n_particles, -0.25),
            w(p.n_particles, 1.0), E(3 * (size_t)p.n_cells, 0.0), B(2 * (size_t)p.n_cells, 0.0);
        const bool em = p.scheme == PIC_EMEC_LI || p.scheme == PIC_EMEC_PSATD;
        int64_t bad = 7;
        expect(pic_check_inputs(&p, x.data(), v.data(), w.data(), E.data(), em ? B.data() : nullptr,
                                &bad) == PIC_OK && bad == -1, "finite inputs pass", k);
        std::vector<double> *arrs[] = {&x, &v, &w, &E, &B};
        std::vector<double> &a = *arrs[rng() % (em ? 5 : 4)];
        const size_t at = rng() % a.size();
        a[at] = (k % 2) ? nan : -inf;
        expect(pic_check_inputs(&p, x.data(), v.data(), w.data(), E.data(), em ? B.data() : nullptr,
                                &bad) == PIC_ENONFINITE && bad == (int64_t)at,
               "a non-finite value is found at its index", k);
        expect(pic_check_inputs(&p, nullptr, v.data(), nullptr, E.data(), B.data(), &bad) == PIC_EINVAL,
               "NULL x", k);
    }
    expect(accepted > 1000, "enough valid cases", -1);
    expect(pic_validate_params(nullptr) == PIC_EINVAL, "NULL params", -1);
    expect(pic_workspace_size(nullptr) == 0, "NULL params size", -1);
    expect(pic_check_inputs(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == PIC_EINVAL,
           "NULL check", -1);
    for (int s = -20; s <= 5; ++s)
        expect(pic_strerror(s) != nullptr, "strerror", s);
    std::printf("%s: %lld valid parameter sets checked\n", failures ? "FAILED" : "ok", accepted);
    return failures ? 1 : 0;
}
