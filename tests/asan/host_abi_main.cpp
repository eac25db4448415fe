// Host-only exercise of the C ABI's argument checking and workspace planning,
// built with AddressSanitizer (host code) by tests/test_asan_host.py.  No
// device call is reached: every call below returns before the library's
// first HIP call, and the kernel launchers are replaced by stubs that fail.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "hevi.h"
#include "hevi_kernels.h"

namespace hv {
// stand-ins for the device side (never reached by the calls below)
hipError_t launch_slow_prep(int, int, int, const Group &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_slow_flux(int, int, int, const Group &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_short_step(int, int, int, const Group &, double, double, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_clock(const Group &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_sums(int, int, int, const Group &, bool, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_diffuse(int, int, int, const DiffArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t scratch_address(double **out) { *out = nullptr; return hipErrorInvalidValue; }
}  // namespace hv

static int failures = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) { std::printf("FAILED line %d: %s\n", __LINE__, #c); ++failures; } \
    } while (0)

static std::vector<double> levels(int nz)
{
    std::vector<double> z(nz + 1);
    for (int k = 0; k <= nz; ++k) {
        const double s = (double)k / nz;
        z[k] = 20000.0 * (s + s * s) / 2.0;
    }
    return z;
}

static hv_grid_desc desc(int nx, int ny, int nz, const double *zf, const double *terrain, int prec)
{
    hv_grid_desc d;
    std::memset(&d, 0, sizeof d);
    d.nx = nx; d.ny = ny; d.nz = nz;
    d.dx = d.dy = 2000.0;
    d.zeta_faces = zf;
    d.terrain = terrain;
    d.precision = prec;
    d.layout = HV_KIJ;
    d.beta = 0.55;
    return d;
}

int main()
{
    for (int nz : {32, 64, 128}) {
        const std::vector<double> zf = levels(nz);
        std::vector<double> h(13 * 9);
        for (size_t c = 0; c < h.size(); ++c) h[c] = 100.0 * (double)(c % 7);
        for (int prec : {HV_FP64, HV_FP32, HV_MIXED}) {
            hv_grid_desc d = desc(13, 9, nz, zf.data(), nullptr, prec);
            const size_t flat = hv_workspace_bytes(&d);
            CHECK(flat >= (size_t)25 * 13 * 9 * nz * (prec == HV_FP64 ? 8 : 4));
            d.terrain = h.data();
            const size_t tr = hv_workspace_bytes(&d);
            CHECK(tr > flat);
            d.short_scheme = HV_SHORT_RK2;
            d.damping = 1;
            CHECK(hv_workspace_bytes(&d) > tr);
            // an ensemble of three differently shaped members
            hv_grid_desc m[3] = {desc(13, 9, nz, zf.data(), nullptr, prec),
                                 desc(4, 31, nz, zf.data(), nullptr, prec),
                                 desc(13, 9, nz, zf.data(), h.data(), prec)};
            CHECK(hv_ens_workspace_bytes(3, m) > hv_workspace_bytes(&m[0]) + hv_workspace_bytes(&m[1]));
            m[1].precision = (prec + 1) % 3;
            hv_ens_t e = nullptr;
            CHECK(hv_ens_create(3, m, nullptr, 0, nullptr, &e) == HV_ERR_ARG && !e);
            CHECK(std::strlen(hv_ens_last_error(nullptr)) > 0);
        }
        // invalid descriptions
        hv_grid_desc d = desc(3, 9, nz, zf.data(), nullptr, HV_FP32);
        CHECK(hv_workspace_bytes(&d) == 0);
        CHECK(std::strstr(hv_last_error(nullptr), "nx and ny") != nullptr);
        d = desc(13, 9, nz, zf.data(), nullptr, HV_FP32);
        d.mass_drift_bound = std::nan("");
        CHECK(hv_workspace_bytes(&d) == 0);
        d = desc(13, 9, nz, zf.data(), nullptr, 7);
        CHECK(hv_workspace_bytes(&d) == 0);
        std::vector<double> bad = zf;
        bad[nz / 2] = bad[nz / 2 - 1];
        d = desc(13, 9, nz, bad.data(), nullptr, HV_FP32);
        CHECK(hv_workspace_bytes(&d) == 0);
        std::vector<double> hb(13 * 9, 19000.0);
        d = desc(13, 9, nz, zf.data(), hb.data(), HV_FP32);
        CHECK(hv_workspace_bytes(&d) == 0);
        // create: rejected before any device call
        d = desc(13, 9, nz, zf.data(), nullptr, HV_FP32);
        const size_t n = hv_workspace_bytes(&d);
        hv_grid_t g = nullptr;
        CHECK(hv_grid_create(&d, nullptr, n, nullptr, &g) == HV_ERR_ARG && !g);
        CHECK(hv_grid_create(&d, (void *)4104, n, nullptr, &g) == HV_ERR_ARG && !g);
        CHECK(hv_grid_create(&d, (void *)4096, n - 1, nullptr, &g) == HV_ERR_ARG && !g);
        CHECK(std::strstr(hv_last_error(nullptr), "too small") != nullptr);
        CHECK(hv_grid_create(&d, (void *)4096, n, nullptr, nullptr) == HV_ERR_ARG);
        d.div_damp = 0.1;
        CHECK(hv_grid_create(&d, (void *)4096, n, nullptr, &g) == HV_ERR_UNSUPPORTED && !g);
    }
    // calls without a handle
    double x = 0.0;
    CHECK(hv_step(nullptr, 10.0, 1, 4) == HV_ERR_ARG);
    CHECK(hv_state_read(nullptr, 0, &x) == HV_ERR_ARG);
    CHECK(hv_mass(nullptr, &x, &x) == HV_ERR_ARG);
    CHECK(hv_mass_noalloc(nullptr, &x) == HV_ERR_ARG);
    CHECK(hv_tune(nullptr, nullptr, nullptr) == HV_ERR_ARG);
    CHECK(hv_configure(nullptr, nullptr, nullptr, nullptr, nullptr) == HV_ERR_ARG);
    CHECK(hv_trace(nullptr, 1) == HV_ERR_ARG);
    CHECK(hv_state_init(nullptr, nullptr, nullptr, nullptr, nullptr) == HV_ERR_ARG);
    hv_grid_destroy(nullptr);
    hv_ens_destroy(nullptr);
    // the diffusion step's checks
    CHECK(hv_diffuse(16, 16, 40, HV_FP32, HV_KIJ, 0.1, 0.1, 0.1, 16, (void *)256, (void *)512, nullptr) ==
          HV_ERR_ARG);
    CHECK(hv_diffuse(16, 16, 32, HV_MIXED, HV_KIJ, 0.1, 0.1, 0.1, 16, (void *)256, (void *)512, nullptr) ==
          HV_ERR_ARG);
    CHECK(hv_diffuse(16, 16, 32, HV_FP32, HV_KIJ, 0.1, 0.1, 0.1, 5, (void *)256, (void *)512, nullptr) ==
          HV_ERR_ARG);
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
    return failures ? 1 : 0;
}
