// hevi_runtime.cpp -- host runtime behind the C ABI declared in include/hevi.h:
// workspace carving, state copy-in/out with layout and precision conversion,
// and the RK3 / short-step launch sequence.
#include "hevi.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hevi_kernels.h"

namespace {

thread_local std::string g_global_error = "no error";

constexpr size_t kAlign = 256;
constexpr int kSeg = 16;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct hv_grid {
    int nx = 0, ny = 0, nz = 0;
    double dx = 0, dy = 0, beta = 0.55;
    int prec = 0, layout = 1;
    size_t esize = 8;            // bytes per stored value
    size_t ncell = 0;            // nx*ny*nz
    hipStream_t stream = nullptr;
    std::vector<double> zf;
    hv::Geom geom{};

    // device arrays carved from the caller's workspace
    void *state[3][5] = {};      // three state buffers
    int cur = 0;                 // index of the buffer holding the current state
    void *slow[7] = {};          // S_U, S_V, S_W, R_Theta, theta_s, P0_s, C_s
    void *spec[3] = {};          // u, v, w of the stage input
    double *vm = nullptr;        // per-level constants
    double *partials = nullptr;  // per-block sums
    double *sums = nullptr;      // [0] perturbation mass after the last step,
                                 // [1] scratch, [2] nonfinite flag (max |.|)
    double mass_ref = 0.0;       // sum of rho_ref * volume (constant part)
    bool have_state = false;
    bool any_nonfinite = false;
    std::string err = "no error";

    // kernel timing (hv_trace)
    struct Pending { int kind; hipEvent_t a, b; };
    bool tracing = false;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double trace_ms[HV_K_COUNT] = {};
    int64_t trace_n[HV_K_COUNT] = {};

    ~hv_grid()
    {
        for (auto &p : pending) { pool.push_back(p.a); pool.push_back(p.b); }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

namespace {

int fail(hv_grid *g, int code, const std::string &msg)
{
    if (g) g->err = msg;
    else g_global_error = msg;
    return code;
}

int hip_fail(hv_grid *g, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(g, HV_ERR_HIP, m);
}

// Validate a description; returns an empty string if it is usable.
std::string check_desc(const hv_grid_desc *d)
{
    if (!d) return "desc is NULL";
    if (d->nx < 4 || d->ny < 4) return "nx and ny must be >= 4";
    if (d->nz != 32 && d->nz != 64 && d->nz != 128) return "nz must be 32, 64 or 128";
    if (!(d->dx > 0.0) || !(d->dy > 0.0) || !std::isfinite(d->dx) || !std::isfinite(d->dy))
        return "dx and dy must be positive";
    if ((size_t)d->nx * (size_t)d->ny > (size_t)INT32_MAX / 2) return "too many columns";
    if (!d->zeta_faces) return "zeta_faces is NULL";
    if (d->zeta_faces[0] != 0.0) return "zeta_faces[0] must be 0";
    for (int k = 0; k < d->nz; ++k)
        if (!(d->zeta_faces[k + 1] > d->zeta_faces[k]) || !std::isfinite(d->zeta_faces[k + 1]))
            return "zeta_faces must be finite and strictly increasing";
    if (d->precision < HV_FP64 || d->precision > HV_MIXED) return "unknown precision";
    if (d->layout != HV_IJK && d->layout != HV_KIJ) return "unknown layout";
    if (!(d->beta >= 0.5 && d->beta <= 1.0)) return "beta must be in [0.5, 1]";
    return "";
}

bool unsupported(const hv_grid_desc *d, std::string *why)
{
    if (d->terrain) { *why = "terrain-following coordinates are not built (terrain must be NULL)"; return true; }
    if (d->div_damp != 0.0) { *why = "divergence damping is not built (div_damp must be 0)"; return true; }
    return false;
}

size_t elem_size(int prec) { return prec == HV_FP64 ? 8 : 4; }

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    }
};

// Layout of the workspace; returns the total size.
size_t plan(const hv_grid_desc *d, size_t *offs /* 3*5 + 7 + 3 + 3 */)
{
    const size_t n = (size_t)d->nx * d->ny * d->nz;
    const size_t es = elem_size(d->precision);
    hv::Geom g{d->nx, d->ny, d->nz, 0, 0, 0};
    Carve c;
    int q = 0;
    for (int b = 0; b < 3; ++b)
        for (int f = 0; f < 5; ++f) offs[q++] = c.take(n * es);
    for (int f = 0; f < 7; ++f) offs[q++] = c.take(n * es);
    for (int f = 0; f < 3; ++f) offs[q++] = c.take(n * es);
    offs[q++] = c.take(sizeof(double) * hv::VM_NFIELDS * d->nz);
    offs[q++] = c.take(sizeof(double) * (size_t)hv::mass_partials(g));
    offs[q++] = c.take(sizeof(double) * 4);
    return c.off;
}
constexpr int kNOffs = 15 + 7 + 3 + 3;

// canonical (i-fastest, float64) index of cell (i, j, k)
inline size_t canon(int i, int j, int k, int nx, int ny) { return ((size_t)k * ny + j) * nx + i; }

inline size_t dev_index(const hv_grid *g, int i, int j, int k)
{
    if (g->layout == HV_KIJ) return ((size_t)j * g->nx + i) * g->nz + k;
    return ((size_t)k * g->ny + j) * g->nx + i;
}

template <typename T>
void to_device_order(const hv_grid *g, const double *src, T *dst)
{
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i)
                dst[dev_index(g, i, j, k)] = (T)src[canon(i, j, k, g->nx, g->ny)];
}

template <typename T>
void from_device_order(const hv_grid *g, const T *src, double *dst)
{
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i)
                dst[canon(i, j, k, g->nx, g->ny)] = (double)src[dev_index(g, i, j, k)];
}

void fill_vmet(hv_grid *g, const double *rho, const double *rt, const double *p, std::vector<double> &vm)
{
    const int nz = g->nz;
    vm.assign((size_t)hv::VM_NFIELDS * nz, 0.0);
    auto at = [&](int f, int k) -> double & { return vm[(size_t)f * nz + k]; };
    for (int k = 0; k < nz; ++k) {
        const double dz = g->zf[k + 1] - g->zf[k];
        at(hv::VM_DZ, k) = dz;
        at(hv::VM_RDZ, k) = 1.0 / dz;
        at(hv::VM_VOL, k) = g->dx * g->dy * dz;
        at(hv::VM_ZC, k) = 0.5 * (g->zf[k + 1] + g->zf[k]);
        at(hv::VM_RHO, k) = rho ? rho[k] : 0.0;
        at(hv::VM_RT, k) = rt ? rt[k] : 1.0;
        at(hv::VM_P, k) = p ? p[k] : 0.0;
        if (k == 0) {
            at(hv::VM_DZF, k) = 1.0;
            at(hv::VM_RDZF, k) = 1.0;
            at(hv::VM_A, k) = 0.0;
            at(hv::VM_B, k) = 0.0;
        } else {
            const double dzm = g->zf[k] - g->zf[k - 1];
            const double dzf = 0.5 * (g->zf[k + 1] + g->zf[k]) - 0.5 * (g->zf[k] + g->zf[k - 1]);
            at(hv::VM_DZF, k) = dzf;
            at(hv::VM_RDZF, k) = 1.0 / dzf;
            at(hv::VM_A, k) = dzm / (dzm + dz);
            at(hv::VM_B, k) = dz / (dzm + dz);
        }
    }
}

hipError_t sync(hv_grid *g) { return hipStreamSynchronize(g->stream); }

hipError_t take_event(hv_grid *g, hipEvent_t *e)
{
    if (!g->pool.empty()) {
        *e = g->pool.back();
        g->pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Run one launch, bracketed by events when tracing is on.
template <class F>
hipError_t traced(hv_grid *g, int kind, F &&launch)
{
    if (!g->tracing) return launch();
    hipEvent_t a, b;
    hipError_t e = take_event(g, &a);
    if (e != hipSuccess) return e;
    e = take_event(g, &b);
    if (e != hipSuccess) return e;
    e = hipEventRecord(a, g->stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, g->stream);
    if (e != hipSuccess) return e;
    g->pending.push_back({kind, a, b});
    return hipSuccess;
}

hipError_t fold_trace(hv_grid *g)
{
    hipError_t e = sync(g);
    if (e != hipSuccess) return e;
    for (auto &p : g->pending) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) return e;
        g->trace_ms[p.kind] += ms;
        g->trace_n[p.kind] += 1;
        g->pool.push_back(p.a);
        g->pool.push_back(p.b);
    }
    g->pending.clear();
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t hv_workspace_bytes(const hv_grid_desc *desc)
{
    std::string why = check_desc(desc);
    if (!why.empty()) { g_global_error = why; return 0; }
    size_t offs[kNOffs];
    return plan(desc, offs);
}

int hv_grid_create(const hv_grid_desc *desc, void *dev_workspace, size_t bytes, void *hip_stream,
                   hv_grid_t *out)
{
    if (!out) return fail(nullptr, HV_ERR_ARG, "out is NULL");
    *out = nullptr;
    std::string why = check_desc(desc);
    if (!why.empty()) return fail(nullptr, HV_ERR_ARG, why);
    if (unsupported(desc, &why)) return fail(nullptr, HV_ERR_UNSUPPORTED, why);
    size_t offs[kNOffs];
    const size_t need = plan(desc, offs);
    if (!dev_workspace) return fail(nullptr, HV_ERR_ARG, "workspace is NULL");
    if (((uintptr_t)dev_workspace) % kAlign) return fail(nullptr, HV_ERR_ARG, "workspace not 256-byte aligned");
    if (bytes < need) {
        char b[160];
        std::snprintf(b, sizeof b, "workspace too small: %zu bytes given, %zu needed", bytes, need);
        return fail(nullptr, HV_ERR_ARG, b);
    }
    hv_grid *g = new (std::nothrow) hv_grid();
    if (!g) return fail(nullptr, HV_ERR_ARG, "out of host memory");
    g->nx = desc->nx; g->ny = desc->ny; g->nz = desc->nz;
    g->dx = desc->dx; g->dy = desc->dy; g->beta = desc->beta;
    g->prec = desc->precision; g->layout = desc->layout;
    g->esize = elem_size(g->prec);
    g->ncell = (size_t)g->nx * g->ny * g->nz;
    g->stream = (hipStream_t)hip_stream;
    g->zf.assign(desc->zeta_faces, desc->zeta_faces + desc->nz + 1);
    g->geom = hv::Geom{g->nx, g->ny, g->nz, 1.0 / g->dx, 1.0 / g->dy, g->beta};
    char *ws = (char *)dev_workspace;
    int q = 0;
    for (int b = 0; b < 3; ++b)
        for (int f = 0; f < 5; ++f) g->state[b][f] = ws + offs[q++];
    for (int f = 0; f < 7; ++f) g->slow[f] = ws + offs[q++];
    for (int f = 0; f < 3; ++f) g->spec[f] = ws + offs[q++];
    g->vm = (double *)(ws + offs[q++]);
    g->partials = (double *)(ws + offs[q++]);
    g->sums = (double *)(ws + offs[q++]);
    *out = g;
    return HV_OK;
}

int hv_state_init(hv_grid_t g, const double *const fields[5], const double *rho_ref,
                  const double *rhotheta_ref, const double *p_ref)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (!fields || !rho_ref || !rhotheta_ref || !p_ref) return fail(g, HV_ERR_ARG, "NULL input array");
    for (int f = 0; f < 5; ++f)
        if (!fields[f]) return fail(g, HV_ERR_ARG, "NULL field pointer");
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t nxy = (size_t)nx * ny;
    for (int k = 0; k < nz; ++k)
        if (!std::isfinite(rho_ref[k]) || !(rho_ref[k] > 0) || !std::isfinite(p_ref[k]) ||
            !(p_ref[k] > 0) || !std::isfinite(rhotheta_ref[k]) || !(rhotheta_ref[k] > 0))
            return fail(g, HV_ERR_ARG, "reference columns must be finite and positive");
    for (int f = 0; f < 5; ++f) {
        const size_t n = (f == HV_RHOW ? nxy * (nz + 1) : nxy * nz);
        for (size_t q = 0; q < n; ++q)
            if (!std::isfinite(fields[f][q])) return fail(g, HV_ERR_ARG, "non-finite value in a field");
    }
    for (size_t q = 0; q < nxy; ++q)
        if (fields[HV_RHOW][q] != 0.0 || fields[HV_RHOW][nxy * nz + q] != 0.0)
            return fail(g, HV_ERR_ARG, "rho*w must be 0 on both lids");

    std::vector<double> vm;
    fill_vmet(g, rho_ref, rhotheta_ref, p_ref, vm);
    hipError_t e = hipMemcpyAsync(g->vm, vm.data(), vm.size() * sizeof(double), hipMemcpyHostToDevice,
                                  g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "hipMemcpyAsync(vmet)");

    // convert each field to the device layout and precision, then copy in
    std::vector<double> bd;
    std::vector<float> bf;
    if (g->prec == HV_FP64) bd.resize(g->ncell);
    else bf.resize(g->ncell);
    g->cur = 0;
    for (int f = 0; f < 5; ++f) {
        const void *src;
        if (g->prec == HV_FP64) { to_device_order(g, fields[f], bd.data()); src = bd.data(); }
        else { to_device_order(g, fields[f], bf.data()); src = bf.data(); }
        e = hipMemcpyAsync(g->state[0][f], src, g->ncell * g->esize, hipMemcpyHostToDevice, g->stream);
        if (e == hipSuccess) e = sync(g);   // staging buffer is reused by the next field
        if (e != hipSuccess) return hip_fail(g, e, "hipMemcpyAsync(state)");
    }
    // constant part of the mass, summed on the host with compensation
    double s = 0.0, c = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double x = rho_ref[k] * (g->dx * g->dy * (g->zf[k + 1] - g->zf[k])) * (double)nxy;
        const double t = s + x;
        c += (std::fabs(s) >= std::fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    g->mass_ref = s + c;
    e = hv::launch_mass(g->prec, g->layout, g->geom, g->vm, g->state[0][HV_RHO_PTB], g->partials,
                        g->sums, g->stream);
    if (e == hipSuccess) e = sync(g);
    if (e != hipSuccess) return hip_fail(g, e, "mass after state_init");
    g->have_state = true;
    g->any_nonfinite = false;
    return HV_OK;
}

int hv_step(hv_grid_t g, double dt, int32_t n_long, int32_t n_short)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (!g->have_state) return fail(g, HV_ERR_STATE, "hv_step before hv_state_init");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(g, HV_ERR_ARG, "dt must be positive");
    if (n_long < 0) return fail(g, HV_ERR_ARG, "n_long must be >= 0");
    if (n_short < 1) return fail(g, HV_ERR_ARG, "n_short must be >= 1");
    const double frac[3] = {1.0 / 3.0, 0.5, 1.0};
    for (int step = 0; step < n_long; ++step) {
        const int P = g->cur;                         // start state
        const int R0 = (P + 1) % 3, R1 = (P + 2) % 3; // running buffers
        int stage_in = P;
        for (int s = 0; s < 3; ++s) {
            void *const *in = g->state[stage_in];
            const void *st[5] = {in[0], in[1], in[2], in[3], in[4]};
            void *prep[6] = {g->spec[0], g->spec[1], g->spec[2], g->slow[4], g->slow[5], g->slow[6]};
            hipError_t e = traced(g, HV_K_SLOW_PREP, [&] {
                return hv::launch_slow_prep(g->prec, g->layout, g->geom, g->vm, st, prep, g->stream);
            });
            if (e != hipSuccess) return hip_fail(g, e, "slow sweep (prep)");
            const void *uvw[3] = {in[1], in[2], in[3]};
            const void *spec[4] = {g->spec[0], g->spec[1], g->spec[2], g->slow[4]};
            void *fl[4] = {g->slow[0], g->slow[1], g->slow[2], g->slow[3]};
            e = traced(g, HV_K_SLOW_FLUX, [&] {
                return hv::launch_slow_flux(g->prec, g->layout, g->geom, g->vm, uvw, spec, fl, g->stream);
            });
            if (e != hipSuccess) return hip_fail(g, e, "slow sweep (flux)");
            const double dtau = dt * frac[s] / n_short;
            int src = P;
            for (int q = 0; q < n_short; ++q) {
                const int dst = (q & 1) ? R1 : R0;
                const void *sin[5], *sl[7];
                for (int f = 0; f < 5; ++f) sin[f] = g->state[src][f];
                for (int f = 0; f < 7; ++f) sl[f] = g->slow[f];
                e = traced(g, HV_K_SHORT_STEP, [&] {
                    return hv::launch_short_step(g->prec, g->layout, g->geom, g->vm, sin, g->state[dst],
                                                 sl, dtau, g->stream);
                });
                if (e != hipSuccess) return hip_fail(g, e, "short step");
                src = dst;
            }
            stage_in = src;
        }
        g->cur = stage_in;
        hipError_t e = traced(g, HV_K_MASS, [&] {
            return hv::launch_mass(g->prec, g->layout, g->geom, g->vm, g->state[g->cur][HV_RHO_PTB],
                                   g->partials, g->sums, g->stream);
        });
        if (e != hipSuccess) return hip_fail(g, e, "mass sum");
    }
    return HV_OK;
}

int hv_state_read(hv_grid_t g, int32_t field, double *host_out)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (!host_out) return fail(g, HV_ERR_ARG, "host_out is NULL");
    if (field < HV_RHO_PTB || field > HV_RHOTHETA_PTB) return fail(g, HV_ERR_ARG, "unknown field id");
    if (!g->have_state) return fail(g, HV_ERR_STATE, "hv_state_read before hv_state_init");
    hipError_t e = sync(g);
    if (e != hipSuccess) return hip_fail(g, e, "stream synchronize");
    const size_t nxy = (size_t)g->nx * g->ny;
    double *dst = host_out;
    std::vector<double> bd;
    std::vector<float> bf;
    const void *src = g->state[g->cur][field];
    if (g->prec == HV_FP64) {
        bd.resize(g->ncell);
        e = hipMemcpy(bd.data(), src, g->ncell * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(g, e, "hipMemcpy(read)");
        from_device_order(g, bd.data(), dst);
    } else {
        bf.resize(g->ncell);
        e = hipMemcpy(bf.data(), src, g->ncell * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(g, e, "hipMemcpy(read)");
        from_device_order(g, bf.data(), dst);
    }
    if (field == HV_RHOW)
        for (size_t q = 0; q < nxy; ++q) dst[nxy * g->nz + q] = 0.0;   // upper lid
    return HV_OK;
}

int hv_mass(hv_grid_t g, double *mass_out, double *energy_out)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (!g->have_state) return fail(g, HV_ERR_STATE, "hv_mass before hv_state_init");
    hipError_t e = hipSuccess;
    if (energy_out) {
        void *const *st = g->state[g->cur];
        const void *cst[5] = {st[0], st[1], st[2], st[3], st[4]};
        e = hv::launch_energy(g->prec, g->layout, g->geom, g->vm, cst, g->partials, g->sums + 1,
                              g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "energy sum");
    }
    double h[2] = {0.0, 0.0};
    e = hipMemcpyAsync(h, g->sums, 2 * sizeof(double), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = sync(g);
    if (e != hipSuccess) return hip_fail(g, e, "read sums");
    const double m = g->mass_ref + h[0];
    if (mass_out) *mass_out = m;
    if (energy_out) *energy_out = h[1];
    if (!std::isfinite(m)) {
        g->any_nonfinite = true;
    }
    if (g->any_nonfinite) return fail(g, HV_ERR_NONFINITE, "mass sum is not finite");
    return HV_OK;
}

int hv_trace(hv_grid_t g, int32_t on)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (on) {
        hipError_t e = fold_trace(g);
        if (e != hipSuccess) return hip_fail(g, e, "hv_trace");
        for (int k = 0; k < HV_K_COUNT; ++k) { g->trace_ms[k] = 0.0; g->trace_n[k] = 0; }
    }
    g->tracing = on != 0;
    return HV_OK;
}

int hv_trace_read(hv_grid_t g, int32_t kind, double *ms_total, int64_t *launches)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (kind < 0 || kind >= HV_K_COUNT) return fail(g, HV_ERR_ARG, "unknown kernel kind");
    hipError_t e = fold_trace(g);
    if (e != hipSuccess) return hip_fail(g, e, "hv_trace_read");
    if (ms_total) *ms_total = g->trace_ms[kind];
    if (launches) *launches = g->trace_n[kind];
    return HV_OK;
}

void hv_grid_destroy(hv_grid_t g) { delete g; }

const char *hv_last_error(hv_grid_t g)
{
    if (!g) return g_global_error.c_str();
    return g->err.c_str();
}

}  // extern "C"
