// hevi_runtime.cpp -- host runtime behind the C ABI declared in include/hevi.h.
//
// A grid is an ensemble of one member.  An ensemble keeps, inside the
// caller's workspace, a device table with one record per member (sizes,
// spacings, long-step length and array pointers) and, per group of members
// with the same nz, the member ids and a per-block (member, tile) map each
// grouped launch uses; a single member's record travels in the kernel
// arguments instead.  One long step is the launch sequence
//   for each stage: slow prep, slow flux, n short steps   (per group;
//                   two launches per short step in the Runge-Kutta form)
//   mass partials + final sums                             (per group)
// over three state buffers whose roles (start state, two running buffers)
// rotate from one long step to the next; the roles cycle with period 2 or 3,
// so each long step replays one of at most three hipGraphs recorded on a
// private stream.  With tracing on, the same sequence is launched directly
// with an event pair around each launch.
#include "hevi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <filesystem>
#include <fstream>
#include <functional>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "hevi_kernels.h"

namespace {

thread_local std::string g_global_error = "no error";
constexpr size_t kAlign = 256;
constexpr double kDefaultDriftBound = 1e-9;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// tile shapes the autotuner tries: log2 of the columns along x (16x1, 8x2, 4x4);
// a launch configuration is a shape, a block order (launch order or
// XCD-chunked) and a column width: index c = shape + 3 * chunked + 6 * w,
// c in 0..11.  Column-fastest layout: w = 0 the default lanes per column,
// w = 1 the other width (see alt_seg).  i-fastest layout: w = 0 one lane per
// column (64 columns per wavefront; single grids), w = 1 column segments of
// the default width.  The column-fastest slow flux has 12 more, c + 12: the
// same with every segment walking a run of kRun columns along x, in blocks
// of 1x16, 2x8 or 4x4 runs (runs along x by rows), which keep the rows a
// block reads around its own (its y-stencils) few.
constexpr int kShapes[3] = {4, 3, 2};
constexpr int kRunShapes[3] = {0, 1, 2};
int shape_log2(int sh) { return sh < 3 ? kShapes[sh] : kRunShapes[sh - 3]; }   // sh 0..5
constexpr int kConfigs = 24;   // most configurations of a kind
constexpr int kRun = 32;
enum { KIND_PREP = 0, KIND_FLUX = 1, KIND_SHORT = 2, NKIND = 3 };

struct MemberHost {
    int nx = 0, ny = 0, nz = 0, L = 0;
    bool damp_room = false;    // workspace holds damping data
    double *d_nu = nullptr;    // device: nu_lat (nx*ny) then nu_top (nz)
    double dx = 0, dy = 0, beta = 0.55, dt = -1.0;
    std::vector<double> zf;
    std::vector<double> h;     // surface heights (terrain), empty when flat
    size_t ncell = 0;
    hv::MemberDev dev{};       // host copy of the device record
    double mass_ref = 0.0;
    bool have_state = false;
};

struct GroupHost {
    int L = 0;
    bool terrain = false;
    bool damping = false;      // some member has damping data
    bool off32 = false;        // every member's arrays fit 32-bit byte offsets
    std::vector<int> ids;
    int *d_ids = nullptr;
    // per tile shape, then per tile shape of runs (kRun columns per segment
    // along x): block -> slot << 24 | tile (nm > 1)
    unsigned *d_blk[6] = {};
    unsigned *d_pblk = nullptr;  // block -> slot << 24 | partial (nm > 1)
    int nblocks[6] = {};
    int npblocks = 0;
    int shape[NKIND] = {0, 0, 0};  // launch configuration per kernel kind (0..kConfigs-1)
};

struct GraphEntry {
    int n_short, roles[3];
    hipGraphExec_t exec;
};

}  // namespace

struct hv_ens {
    int n = 0, prec = 0, layout = 1;
    bool rk2 = false;                // two-stage Runge-Kutta short steps
    size_t esize = 8;
    hipStream_t stream = nullptr;    // caller's stream
    hipStream_t own = nullptr;       // private stream for graph replay
    hipEvent_t fork = nullptr, join = nullptr;
    std::vector<MemberHost> m;
    std::vector<GroupHost> groups;
    hv::MemberDev *d_mem = nullptr;
    int roles[3] = {0, 1, 2};        // start/current buffer, two running buffers
    std::vector<GraphEntry> graphs;
    std::string err = "no error";

    struct Pending { int kind; hipEvent_t a, b; };
    bool tracing = false;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double trace_ms[HV_K_COUNT] = {};
    int64_t trace_n[HV_K_COUNT] = {};

    ~hv_ens()
    {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
        for (auto &p : pending) { pool.push_back(p.a); pool.push_back(p.b); }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (own) (void)hipStreamDestroy(own);
    }
};

struct hv_grid : hv_ens {
    double *scratch = nullptr;   // this device's copy of the library scratch
};

namespace {

int fail(hv_ens *e, int code, const std::string &msg)
{
    if (e) e->err = msg;
    else g_global_error = msg;
    return code;
}

int hip_fail(hv_ens *e, hipError_t err, const char *what)
{
    return fail(e, HV_ERR_HIP, std::string(what) + ": " + hipGetErrorString(err));
}

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
    if (d->short_scheme != HV_SHORT_FB && d->short_scheme != HV_SHORT_RK2) return "unknown short_scheme";
    if (d->damping != 0 && d->damping != 1) return "damping must be 0 or 1";
    if (std::isnan(d->mass_drift_bound)) return "mass_drift_bound must not be NaN";
    if (d->terrain) {
        const double H = d->zeta_faces[d->nz];
        const size_t nxy = (size_t)d->nx * d->ny;
        for (size_t c = 0; c < nxy; ++c)
            if (!std::isfinite(d->terrain[c]) || !(1.0 - d->terrain[c] / H >= 0.1))
                return "terrain heights must be finite with 1 - h/H >= 0.1";
    }
    return "";
}

bool unsupported(const hv_grid_desc *d, std::string *why)
{
    if (d->div_damp != 0.0) { *why = "divergence damping is not built (div_damp must be 0)"; return true; }
    return false;
}

size_t elem_size(int prec) { return prec == HV_FP64 ? 8 : 4; }
size_t solve_size(int prec) { return prec == HV_FP32 ? 4 : 8; }   // column-solve values

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    }
};

// Workspace plan of an ensemble.
struct Plan {
    size_t total = 0;
    size_t table = 0;
    std::vector<size_t> group_off;  // per group: ids, 3 block maps, partial map
    std::vector<size_t> member_off; // per member: 25 arrays (+4 and geometry over
                                    // terrain), vm, partials, sums
};

size_t group_words(const std::vector<int> &ids, const hv_grid_desc *d)
{
    size_t w = ids.size();
    if (ids.size() > 1) {
        for (int s = 0; s < 6; ++s)
            for (int q : ids)
                w += (size_t)hv::tiles_of_run(d[q].nx, d[q].ny, shape_log2(s), s < 3 ? 1 : kRun);
        for (int q : ids) w += (size_t)hv::partials_of(d[q].nx, d[q].ny);
    }
    return w;
}

// Members grouped by (flat before terrain, nz): one launch per group and phase.
std::vector<std::vector<int>> group_members(int n, const hv_grid_desc *d)
{
    std::vector<std::vector<int>> g;
    for (int tr = 0; tr < 2; ++tr)
        for (int nz : {32, 64, 128}) {
            std::vector<int> ids;
            for (int q = 0; q < n; ++q)
                if (d[q].nz == nz && (d[q].terrain != nullptr) == (tr == 1)) ids.push_back(q);
            if (!ids.empty()) g.push_back(ids);
        }
    return g;
}

Plan make_plan(int n, const hv_grid_desc *d)
{
    Plan p;
    Carve c;
    p.table = c.take(sizeof(hv::MemberDev) * (size_t)n);
    for (auto &ids : group_members(n, d)) p.group_off.push_back(c.take(sizeof(int) * group_words(ids, d)));
    const size_t es = elem_size(d[0].precision);
    for (int q = 0; q < n; ++q) {
        const size_t ncell = (size_t)d[q].nx * d[q].ny * d[q].nz;
        const size_t start = c.take(0);
        for (int a = 0; a < 25; ++a) c.take(ncell * es);
        if (d[q].short_scheme == HV_SHORT_RK2)
            for (int a = 0; a < 5; ++a) c.take(ncell * es);   // first-stage state
        if (d[q].damping) {
            for (int a = 0; a < 10; ++a) c.take(ncell * es);  // two boundary states
            c.take(sizeof(double) * ((size_t)d[q].nx * d[q].ny + d[q].nz));
        }
        if (d[q].terrain) {
            // Omega, three reference fields, per-column geometry
            for (int a = 0; a < 4; ++a) c.take(ncell * es);
            c.take(sizeof(double) * hv::GEO_NFIELDS * (size_t)d[q].nx * d[q].ny);
        }
        if (d[q].layout == HV_IJK && n == 1)   // one-lane-per-column solve (single grids)
            for (int a = 0; a < 4; ++a) c.take(ncell * solve_size(d[q].precision));
        c.take(hv::vm_bytes(d[q].nz));
        c.take(sizeof(double) * (size_t)hv::partials_of(d[q].nx, d[q].ny));
        c.take(sizeof(double) * hv::kSums);
        p.member_off.push_back(start);
    }
    p.total = c.off;
    return p;
}

inline size_t canon(int i, int j, int k, int nx, int ny) { return ((size_t)k * ny + j) * nx + i; }

inline size_t dev_index(int layout, const MemberHost &m, int i, int j, int k)
{
    if (layout == HV_KIJ) return ((size_t)j * m.nx + i) * m.nz + k;
    return ((size_t)k * m.ny + j) * m.nx + i;
}

// body(j0, j1) over rows [0, n) of per_row elements each, split between up
// to 16 host threads when there are more than 2^20 elements (serial if
// threads cannot be started); every element is written by one thread.
template <typename F>
void parallel_rows(int n, size_t per_row, F &&body)
{
    unsigned nt = std::thread::hardware_concurrency();
    nt = std::max(1u, std::min(nt, 16u));
    nt = std::min(nt, (unsigned)std::max(n, 1));
    if (nt > 1 && (size_t)n * per_row > (size_t(1) << 20)) {
        std::vector<std::thread> th;
        try {
            for (unsigned t = 1; t < nt; ++t)
                th.emplace_back([&, t] { body((int)((size_t)n * t / nt), (int)((size_t)n * (t + 1) / nt)); });
        } catch (...) {
            for (auto &x : th) x.join();
            body(0, n);   // idempotent: plain element copies
            return;
        }
        body(0, (int)((size_t)n / nt));
        for (auto &x : th) x.join();
        return;
    }
    body(0, n);
}

// Canonical i-fastest <-> device order.  For the column-fastest order each
// row j is a transpose of an nz x nx block, done in 32 x 32 tiles.
template <typename S, typename D>
void reorder(int layout, const MemberHost &m, const S *src, D *dst, bool to_device)
{
    const int nx = m.nx, ny = m.ny, nz = m.nz;
    parallel_rows(ny, (size_t)nx * nz, [&](int j0, int j1) {
        for (int j = j0; j < j1; ++j) {
            if (layout != HV_KIJ) {
                for (int k = 0; k < nz; ++k) {
                    const size_t o = canon(0, j, k, nx, ny);
                    for (int i = 0; i < nx; ++i) dst[o + i] = (D)src[o + i];
                }
                continue;
            }
            for (int i0 = 0; i0 < nx; i0 += 32)
                for (int k0 = 0; k0 < nz; k0 += 32) {
                    const int i1 = std::min(nx, i0 + 32), k1 = std::min(nz, k0 + 32);
                    if (to_device) {
                        for (int i = i0; i < i1; ++i)
                            for (int k = k0; k < k1; ++k)
                                dst[dev_index(layout, m, i, j, k)] = (D)src[canon(i, j, k, nx, ny)];
                    } else {
                        for (int k = k0; k < k1; ++k)
                            for (int i = i0; i < i1; ++i)
                                dst[canon(i, j, k, nx, ny)] = (D)src[dev_index(layout, m, i, j, k)];
                    }
                }
        }
    });
}

template <typename T>
void to_device_order(int layout, const MemberHost &m, const double *src, T *dst)
{
    reorder(layout, m, src, dst, true);
}

template <typename T>
void from_device_order(int layout, const MemberHost &m, const T *src, double *dst)
{
    reorder(layout, m, src, dst, false);
}

// Per-level table; rho, rt, p are the reference columns (NULL over terrain,
// where the reference is per cell).
void fill_vmet(const MemberHost &m, const double *rho, const double *rt, const double *p,
               std::vector<double> &vm)
{
    const int nz = m.nz;
    const double H = m.zf[nz];
    vm.assign((size_t)hv::VM_NFIELDS * nz, 0.0);
    auto at = [&](int f, int k) -> double & { return vm[(size_t)f * nz + k]; };
    for (int k = 0; k < nz; ++k) {
        const double dz = m.zf[k + 1] - m.zf[k];
        at(hv::VM_DZ, k) = dz;
        at(hv::VM_RDZ, k) = 1.0 / dz;
        at(hv::VM_VOL, k) = m.dx * m.dy * dz;
        at(hv::VM_ZC, k) = 0.5 * (m.zf[k + 1] + m.zf[k]);
        at(hv::VM_DC, k) = 1.0 - 0.5 * (m.zf[k] + m.zf[k + 1]) / H;
        at(hv::VM_DF, k) = 1.0 - m.zf[k] / H;
        if (rho) {
            at(hv::VM_RHO, k) = rho[k];
            at(hv::VM_RT, k) = rt[k];
            at(hv::VM_P, k) = p[k];
        }
        if (k == 0) {
            at(hv::VM_DZF, k) = 1.0;
            at(hv::VM_RDZF, k) = 1.0;
        } else {
            const double dzm = m.zf[k] - m.zf[k - 1];
            const double dzf = 0.5 * (m.zf[k + 1] + m.zf[k]) - 0.5 * (m.zf[k] + m.zf[k - 1]);
            at(hv::VM_DZF, k) = dzf;
            at(hv::VM_RDZF, k) = 1.0 / dzf;
            at(hv::VM_A, k) = dzm / (dzm + dz);
            at(hv::VM_B, k) = dz / (dzm + dz);
        }
    }
}

// Per-column geometry of z = zeta + h (1 - zeta/H): J = 1 - h/H, the face
// Jacobians as means of the two columns, the face slopes as differences of h.
void fill_geo(const MemberHost &m, std::vector<double> &geo)
{
    const int nx = m.nx, ny = m.ny;
    const double H = m.zf[m.nz];
    geo.assign((size_t)hv::GEO_NFIELDS * nx * ny, 0.0);
    auto wrap = [](int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); };
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double h = m.h[(size_t)j * nx + i];
            const double hw = m.h[(size_t)j * nx + wrap(i - 1, nx)];
            const double hs = m.h[(size_t)wrap(j - 1, ny) * nx + i];
            double *g = &geo[((size_t)j * nx + i) * hv::GEO_NFIELDS];
            g[hv::GEO_J] = 1.0 - h / H;
            g[hv::GEO_JU] = 0.5 * ((1.0 - hw / H) + (1.0 - h / H));
            g[hv::GEO_JV] = 0.5 * ((1.0 - hs / H) + (1.0 - h / H));
            g[hv::GEO_SU] = (h - hw) / m.dx;
            g[hv::GEO_SV] = (h - hs) / m.dy;
            g[hv::GEO_H] = h;
        }
}

hipError_t sync(hv_ens *e) { return hipStreamSynchronize(e->stream); }

// Lanes per column: the default (32 for float64 storage with 64 levels,
// else 16) and the other width the kernels offer for the column-fastest
// layout (8 lanes for 32 levels, 32 for 64 levels in float32, 16 for 64
// levels in float64, 32 for 128 levels).
int default_seg(int prec, int L) { return (prec == HV_FP64 && L == 4) ? 32 : 16; }
int alt_seg(int prec, int L)
{
    if (L == 2) return 8;
    if (L == 4) return default_seg(prec, L) == 32 ? 16 : 32;
    return 32;
}
// configurations of a kernel kind (runs: the column-fastest slow flux)
int configs_of(const hv_ens *e, int kind)
{
    return (kind == KIND_FLUX && e->layout == HV_KIJ) ? 24 : 12;
}

// Launch description of group g for a kernel kind (< 0: the sums); ev < 0
// means the short step takes its explicit terms from src.
hv::Group group_launch(const hv_ens *e, const GroupHost &g, int kind, int src, int dst = 0,
                       int ev = -1)
{
    hv::Group gr{};
    gr.mem = e->d_mem;
    gr.ids = g.d_ids;
    gr.nm = (int)g.ids.size();
    gr.src = src;
    gr.dst = dst;
    gr.ev = ev < 0 ? src : ev;
    gr.terrain = g.terrain ? 1 : 0;
    gr.off32 = g.off32 ? 1 : 0;
    if (kind < 0) {
        gr.blk = g.d_pblk;
        gr.nblocks = g.npblocks;
        gr.ti_log2 = 4;
    } else {
        const int sh = g.shape[kind] % 3, run = g.shape[kind] / 12;
        gr.blk = g.d_blk[sh + 3 * run];
        gr.nblocks = g.nblocks[sh + 3 * run];
        gr.ti_log2 = shape_log2(sh + 3 * run);
        gr.xcd = (g.shape[kind] / 3) % 2;
        gr.run = run ? kRun : 0;
        const bool w = (g.shape[kind] / 6) % 2;
        const bool col = !w;
        if (e->layout == HV_KIJ) {
            gr.seg = w ? alt_seg(e->prec, g.L) : 0;
        } else {
            // one lane per column for a single grid (whose workspace holds the
            // column solve's arrays); the Runge-Kutta short step keeps its
            // column segments (both of its stages alike)
            gr.colmap = (col && e->n == 1 && !(kind == KIND_SHORT && e->rk2)) ? 1 : 0;
        }
    }
    gr.first = g.ids[0];
    gr.nx1 = e->m[g.ids[0]].nx;
    gr.ny1 = e->m[g.ids[0]].ny;
    return gr;
}

// ---- tracing ----
hipError_t take_event(hv_ens *e, hipEvent_t *ev)
{
    if (!e->pool.empty()) {
        *ev = e->pool.back();
        e->pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

template <class F>
hipError_t traced(hv_ens *e, hipStream_t s, int kind, F &&launch)
{
    if (!e->tracing) return launch();
    hipEvent_t a, b;
    hipError_t r = take_event(e, &a);
    if (r != hipSuccess) return r;
    r = take_event(e, &b);
    if (r != hipSuccess) { e->pool.push_back(a); return r; }
    if ((r = hipEventRecord(a, s)) != hipSuccess) return r;
    if ((r = launch()) != hipSuccess) return r;
    if ((r = hipEventRecord(b, s)) != hipSuccess) return r;
    e->pending.push_back({kind, a, b});
    return hipSuccess;
}

hipError_t fold_trace(hv_ens *e)
{
    hipError_t r = sync(e);
    if (r != hipSuccess) return r;
    for (auto &p : e->pending) {
        float ms = 0.f;
        if ((r = hipEventElapsedTime(&ms, p.a, p.b)) != hipSuccess) return r;
        e->trace_ms[p.kind] += ms;
        e->trace_n[p.kind] += 1;
        e->pool.push_back(p.a);
        e->pool.push_back(p.b);
    }
    e->pending.clear();
    return hipSuccess;
}

// Enqueue one long step of every member on stream s, for buffer roles r.
hipError_t enqueue_long_step(hv_ens *e, int n_short, const int r[3], hipStream_t s)
{
    const double frac[3] = {1.0 / 3.0, 0.5, 1.0};
    const int P = r[0], R[2] = {r[1], r[2]};
    hipError_t err = hipSuccess;
    // Successive launches of a group take its tiles in alternating
    // directions, so that each starts on the tiles whose data the previous
    // one touched last (still in the Infinity Cache and the L2s).
    std::vector<int> dir(e->groups.size(), 0);
    auto flip = [&](const GroupHost &g, hv::Group gr) {
        int &d = dir[&g - e->groups.data()];
        gr.rev = d;
        d ^= 1;
        return gr;
    };
    for (int st = 0; st < 3; ++st) {
        const int in = st == 0 ? P : R[(n_short - 1) & 1];
        for (auto &g : e->groups) {
            const hv::Group gp = flip(g, group_launch(e, g, KIND_PREP, in)), gf = flip(g, group_launch(e, g, KIND_FLUX, in));
            err = traced(e, s, HV_K_SLOW_PREP, [&] { return hv::launch_slow_prep(e->prec, e->layout, g.L, gp, s); });
            if (err != hipSuccess) return err;
            err = traced(e, s, HV_K_SLOW_FLUX, [&] { return hv::launch_slow_flux(e->prec, e->layout, g.L, gf, s); });
            if (err != hipSuccess) return err;
        }
        for (int q = 0; q < n_short; ++q) {
            const int src = q == 0 ? P : R[(q - 1) & 1], dst = R[q & 1];
            const double f = frac[st] / n_short;
            // damping (groups with damping data) at the end of this short
            // step, model time t_n + (q + 1) dtau, inside the step's kernel
            const double off = (q + 1) * f;
            for (auto &g : e->groups) {
                if (e->rk2) {
                    // X* = Phi(X, X, dtau/2) into buffer 3, then X+ = Phi(X, X*, dtau)
                    const hv::Group g1 = flip(g, group_launch(e, g, KIND_SHORT, src, 3));
                    err = traced(e, s, HV_K_SHORT_STEP, [&] {
                        return hv::launch_short_step(e->prec, e->layout, g.L, g1, 0.5 * f, 0.0, s);
                    });
                    if (err != hipSuccess) return err;
                    hv::Group g2 = flip(g, group_launch(e, g, KIND_SHORT, src, dst, 3));
                    g2.damp = g.damping ? 1 : 0;
                    err = traced(e, s, HV_K_SHORT_STEP, [&] {
                        return hv::launch_short_step(e->prec, e->layout, g.L, g2, f, off, s);
                    });
                } else {
                    hv::Group gs = flip(g, group_launch(e, g, KIND_SHORT, src, dst));
                    gs.damp = g.damping ? 1 : 0;
                    err = traced(e, s, HV_K_SHORT_STEP, [&] {
                        return hv::launch_short_step(e->prec, e->layout, g.L, gs, f, off, s);
                    });
                }
                if (err != hipSuccess) return err;
            }
        }
    }
    const int cur = R[(n_short - 1) & 1];
    for (auto &g : e->groups) {
        const hv::Group gm = group_launch(e, g, -1, cur);
        err = traced(e, s, HV_K_MASS, [&] { return hv::launch_sums(e->prec, e->layout, g.L, gm, false, s); });
        if (err != hipSuccess) return err;
        if (g.damping && (err = hv::launch_clock(gm, s)) != hipSuccess) return err;
    }
    return hipSuccess;
}

// The long step's result becomes the start buffer of the next long step.
void rotate_roles(int r[3], int n_short)
{
    const int cur = r[1 + ((n_short - 1) & 1)];
    const int a = r[0], b = r[1 + (n_short & 1)];
    r[0] = cur;
    r[1] = a;
    r[2] = b;
}

void drop_graphs(hv_ens *e)
{
    for (auto &g : e->graphs) (void)hipGraphExecDestroy(g.exec);
    e->graphs.clear();
}

// ---- autotuner cache: one line per key, "key c_prep c_flux c_short" with
// the launch configuration index of each kind ----
std::string cache_path()
{
    if (const char *p = std::getenv("HV_TUNE_CACHE")) return p;
    if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/hevi/tune.txt";
    return "";
}

std::string tune_key(const hv_ens *e, const GroupHost &g)
{
    size_t cols = 0;
    for (int q : g.ids) cols += (size_t)e->m[q].nx * e->m[q].ny;
    // bucket the group size by powers of two
    int b = 0;
    while ((size_t(1) << (b + 1)) <= cols) ++b;
    std::ostringstream k;
    k << "gfx950:p" << e->prec << ":l" << e->layout << ":L" << g.L << (g.terrain ? ":t" : "") << ":c2^" << b
      << ":m" << g.ids.size();
    return k.str();
}

bool cache_lookup(const std::string &key, int shape[NKIND], int nconf)
{
    const std::string path = cache_path();
    if (path.empty()) return false;
    std::ifstream f(path);
    std::string k;
    int a, b, c;
    bool found = false;
    while (f >> k >> a >> b >> c)
        if (k == key && a >= 0 && a < nconf && b >= 0 && b < nconf && c >= 0 && c < nconf) {
            shape[0] = a; shape[1] = b; shape[2] = c;
            found = true;
        }
    return found;
}

// Replaces the key's line (the file keeps one line per key); written to a
// temporary file and renamed, so a reader never sees a partial file.
void cache_store(const std::string &key, const int shape[NKIND])
{
    const std::string path = cache_path();
    if (path.empty()) return;
    const std::filesystem::path dir = std::filesystem::path(path).parent_path();
    std::error_code ec;   // an unwritable cache only costs the tuning next time
    if (!dir.empty()) std::filesystem::create_directories(dir, ec);
    std::vector<std::string> keep;
    {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            if ((ls >> k) && k != key) keep.push_back(line);
        }
    }
    const std::string tmp = path + ".tmp" + std::to_string((unsigned long)std::hash<std::string>{}(key) & 0xFFFFu);
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out) return;
        for (const auto &l : keep) out << l << '\n';
        out << key << ' ' << shape[0] << ' ' << shape[1] << ' ' << shape[2] << '\n';
        if (!out) return;
    }
    std::filesystem::rename(tmp, path, ec);
    if (ec) std::filesystem::remove(tmp, ec);
}

// ---- creation ----
int ens_create(hv_ens *e, int n, const hv_grid_desc *descs, void *ws, size_t bytes, void *stream)
{
    if (n < 1) return fail(nullptr, HV_ERR_ARG, "member count must be >= 1");
    if (!descs) return fail(nullptr, HV_ERR_ARG, "descs is NULL");
    for (int q = 0; q < n; ++q) {
        std::string why = check_desc(&descs[q]);
        if (!why.empty()) return fail(nullptr, HV_ERR_ARG, (n > 1 ? "member " + std::to_string(q) + ": " : "") + why);
        if (descs[q].precision != descs[0].precision || descs[q].layout != descs[0].layout ||
            descs[q].short_scheme != descs[0].short_scheme)
            return fail(nullptr, HV_ERR_ARG, "all members must share precision, layout and short_scheme");
        if (unsupported(&descs[q], &why)) return fail(nullptr, HV_ERR_UNSUPPORTED, why);
    }
    const Plan p = make_plan(n, descs);
    if (!ws) return fail(nullptr, HV_ERR_ARG, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(nullptr, HV_ERR_ARG, "workspace not 256-byte aligned");
    if (bytes < p.total) {
        char b[160];
        std::snprintf(b, sizeof b, "workspace too small: %zu bytes given, %zu needed", bytes, p.total);
        return fail(nullptr, HV_ERR_ARG, b);
    }
    char *base = (char *)ws;
    e->n = n;
    e->prec = descs[0].precision;
    e->layout = descs[0].layout;
    e->rk2 = descs[0].short_scheme == HV_SHORT_RK2;
    e->esize = elem_size(e->prec);
    e->stream = (hipStream_t)stream;
    e->d_mem = (hv::MemberDev *)(base + p.table);
    e->m.resize(n);
    for (int q = 0; q < n; ++q) {
        MemberHost &m = e->m[q];
        const hv_grid_desc &d = descs[q];
        m.nx = d.nx; m.ny = d.ny; m.nz = d.nz; m.L = d.nz / hv::kSeg;
        m.dx = d.dx; m.dy = d.dy; m.beta = d.beta;
        m.zf.assign(d.zeta_faces, d.zeta_faces + d.nz + 1);
        m.ncell = (size_t)d.nx * d.ny * d.nz;
        Carve c;
        c.off = p.member_off[q];
        hv::MemberDev &v = m.dev;
        v.nx = m.nx; v.ny = m.ny; v.nz = m.nz;
        v.npart = hv::partials_of(m.nx, m.ny);
        v.rdx = 1.0 / m.dx; v.rdy = 1.0 / m.dy; v.beta = m.beta; v.dt = 0.0;
        for (int b = 0; b < 3; ++b)
            for (int f = 0; f < 5; ++f) v.st[b][f] = base + c.take(m.ncell * e->esize);
        for (int f = 0; f < 5; ++f) v.st[3][f] = e->rk2 ? base + c.take(m.ncell * e->esize) : nullptr;
        for (int f = 0; f < 7; ++f) v.slow[f] = base + c.take(m.ncell * e->esize);
        for (int f = 0; f < 3; ++f) v.spec[f] = base + c.take(m.ncell * e->esize);
        v.spec[3] = nullptr;
        v.geo = nullptr;
        v.ref[0] = v.ref[1] = v.ref[2] = nullptr;
        v.nu_lat = v.nu_top = nullptr;
        v.t1 = 0.0;
        v.t2 = 1.0;
        for (int b = 0; b < 2; ++b)
            for (int f = 0; f < 5; ++f) v.bnd[b][f] = nullptr;
        if (d.damping) {
            m.damp_room = true;
            for (int b = 0; b < 2; ++b)
                for (int f = 0; f < 5; ++f) v.bnd[b][f] = base + c.take(m.ncell * e->esize);
            m.d_nu = (double *)(base + c.take(sizeof(double) * ((size_t)m.nx * m.ny + m.nz)));
        }
        if (d.terrain) {
            m.h.assign(d.terrain, d.terrain + (size_t)d.nx * d.ny);
            v.spec[3] = base + c.take(m.ncell * e->esize);
            for (int f = 0; f < 3; ++f) v.ref[f] = base + c.take(m.ncell * e->esize);
            v.geo = (const double *)(base + c.take(sizeof(double) * hv::GEO_NFIELDS * (size_t)m.nx * m.ny));
            std::vector<double> geo;
            fill_geo(m, geo);
            hipError_t r = hipMemcpyAsync((void *)v.geo, geo.data(), geo.size() * sizeof(double),
                                          hipMemcpyHostToDevice, e->stream);
            if (r == hipSuccess) r = sync(e);
            if (r != hipSuccess) return hip_fail(nullptr, r, "upload geometry");
        }
        for (int a = 0; a < 4; ++a)
            v.col[a] = (e->layout == HV_IJK && n == 1) ? base + c.take(m.ncell * solve_size(e->prec)) : nullptr;
        v.vm = (const double *)(base + c.take(hv::vm_bytes(m.nz)));
        v.partials = (double *)(base + c.take(sizeof(double) * (size_t)v.npart));
        v.sums = (double *)(base + c.take(sizeof(double) * hv::kSums));
        v.mass_ref = 0.0;
        v.drift_bound = d.mass_drift_bound > 0.0 ? d.mass_drift_bound
                        : (d.mass_drift_bound == 0.0 && !d.damping ? kDefaultDriftBound : 0.0);
    }
    auto gm = group_members(n, descs);
    e->groups.resize(gm.size());
    for (size_t gi = 0; gi < gm.size(); ++gi) {
        GroupHost &g = e->groups[gi];
        g.ids = gm[gi];
        g.L = descs[g.ids[0]].nz / hv::kSeg;
        g.terrain = descs[g.ids[0]].terrain != nullptr;
        // HV_ADDR64=1 keeps 64-bit addressing everywhere (same results)
        const char *a64 = std::getenv("HV_ADDR64");
        g.off32 = !(a64 && a64[0] == '1');
        for (int q : g.ids)
            if ((size_t)descs[q].nx * descs[q].ny * descs[q].nz * e->esize > 0xFFFFFFFFull) g.off32 = false;
        const int nm = (int)g.ids.size();
        if (n > 255) return fail(nullptr, HV_ERR_ARG, "at most 255 members");
        int *dst = (int *)(base + p.group_off[gi]);
        std::vector<unsigned> h;
        h.reserve(group_words(g.ids, descs));
        for (int a = 0; a < nm; ++a) h.push_back((unsigned)g.ids[a]);
        g.d_ids = dst;
        for (int sh = 0; sh < 6; ++sh) {
            g.nblocks[sh] = 0;
            if (nm > 1) g.d_blk[sh] = (unsigned *)dst + h.size();
            for (int a = 0; a < nm; ++a) {
                const int nt = hv::tiles_of_run(e->m[g.ids[a]].nx, e->m[g.ids[a]].ny, shape_log2(sh),
                                                sh < 3 ? 1 : kRun);
                if (nt >= (1 << 24)) return fail(nullptr, HV_ERR_ARG, "member too large");
                if (nm > 1)
                    for (int t = 0; t < nt; ++t) h.push_back(((unsigned)g.ids[a] << 24) | (unsigned)t);
                g.nblocks[sh] += nt;
            }
        }
        g.npblocks = 0;
        if (nm > 1) g.d_pblk = (unsigned *)dst + h.size();
        for (int a = 0; a < nm; ++a) {
            const int np = e->m[g.ids[a]].dev.npart;
            if (nm > 1)
                for (int t = 0; t < np; ++t) h.push_back(((unsigned)g.ids[a] << 24) | (unsigned)t);
            g.npblocks += np;
        }
        hipError_t r = hipMemcpyAsync(dst, h.data(), h.size() * sizeof(unsigned), hipMemcpyHostToDevice, e->stream);
        if (r == hipSuccess) r = sync(e);
        if (r != hipSuccess) return hip_fail(nullptr, r, "upload group tables");
        int shape[NKIND];
        if (cache_lookup(tune_key(e, g), shape, kConfigs) && shape[KIND_PREP] < configs_of(e, KIND_PREP) &&
            shape[KIND_FLUX] < configs_of(e, KIND_FLUX) && shape[KIND_SHORT] < configs_of(e, KIND_SHORT))
            std::copy(shape, shape + NKIND, g.shape);
    }
    std::vector<hv::MemberDev> table(n);
    for (int q = 0; q < n; ++q) table[q] = e->m[q].dev;
    hipError_t r = hipMemcpyAsync(e->d_mem, table.data(), sizeof(hv::MemberDev) * n,
                                  hipMemcpyHostToDevice, e->stream);
    if (r == hipSuccess) r = sync(e);
    if (r != hipSuccess) return hip_fail(nullptr, r, "upload member table");
    if ((r = hipStreamCreateWithFlags(&e->own, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(nullptr, r, "hipStreamCreateWithFlags");
    if ((r = hipEventCreateWithFlags(&e->fork, hipEventDisableTiming)) != hipSuccess ||
        (r = hipEventCreateWithFlags(&e->join, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(nullptr, r, "hipEventCreate");
    return HV_OK;
}

hipError_t upload_table(hv_ens *e)
{
    std::vector<hv::MemberDev> table(e->n);
    for (int q = 0; q < e->n; ++q) table[q] = e->m[q].dev;
    return hipMemcpy(e->d_mem, table.data(), sizeof(hv::MemberDev) * e->n, hipMemcpyHostToDevice);
}

int member_init(hv_ens *e, int q, const double *const fields[5], const double *rho_ref,
                const double *rhotheta_ref, const double *p_ref)
{
    if (q < 0 || q >= e->n) return fail(e, HV_ERR_ARG, "member index out of range");
    if (!fields || !rho_ref || !rhotheta_ref || !p_ref) return fail(e, HV_ERR_ARG, "NULL input array");
    for (int f = 0; f < 5; ++f)
        if (!fields[f]) return fail(e, HV_ERR_ARG, "NULL field pointer");
    MemberHost &m = e->m[q];
    const size_t nxy = (size_t)m.nx * m.ny;
    const bool terrain = !m.h.empty();
    const size_t nref = terrain ? m.ncell : (size_t)m.nz;
    for (size_t k = 0; k < nref; ++k)
        if (!std::isfinite(rho_ref[k]) || !(rho_ref[k] > 0) || !std::isfinite(p_ref[k]) ||
            !(p_ref[k] > 0) || !std::isfinite(rhotheta_ref[k]) || !(rhotheta_ref[k] > 0))
            return fail(e, HV_ERR_ARG, "reference values must be finite and positive");
    for (int f = 0; f < 5; ++f) {
        const int levels = f == HV_RHOW ? m.nz + 1 : m.nz;
        std::vector<char> bad(levels, 0);
        parallel_rows(levels, nxy, [&](int k0, int k1) {
            for (int k = k0; k < k1; ++k)
                for (size_t c = 0; c < nxy; ++c)
                    if (!std::isfinite(fields[f][(size_t)k * nxy + c])) { bad[k] = 1; break; }
        });
        for (char b : bad)
            if (b) return fail(e, HV_ERR_ARG, "non-finite value in a field");
    }
    for (size_t c = 0; c < nxy; ++c)
        if (fields[HV_RHOW][c] != 0.0 || fields[HV_RHOW][nxy * m.nz + c] != 0.0)
            return fail(e, HV_ERR_ARG, "rho*w must be 0 on both lids");
    hipError_t r = sync(e);   // no step of this ensemble may still read the buffers
    if (r != hipSuccess) return hip_fail(e, r, "stream synchronize");
    std::vector<double> vm;
    if (terrain) fill_vmet(m, nullptr, nullptr, nullptr, vm);
    else fill_vmet(m, rho_ref, rhotheta_ref, p_ref, vm);
    std::vector<unsigned char> vmb(hv::vm_bytes(m.nz));
    std::memcpy(vmb.data(), vm.data(), vm.size() * sizeof(double));
    float *vmf = (float *)(vmb.data() + vm.size() * sizeof(double));
    for (size_t q = 0; q < vm.size(); ++q) vmf[q] = (float)vm[q];
    r = hipMemcpy((void *)m.dev.vm, vmb.data(), vmb.size(), hipMemcpyHostToDevice);
    if (r != hipSuccess) return hip_fail(e, r, "hipMemcpy(vmet)");
    std::vector<double> bd;
    std::vector<float> bf;
    if (e->prec == HV_FP64) bd.resize(m.ncell);
    else bf.resize(m.ncell);
    const int P = e->roles[0];
    auto upload = [&](const double *host, void *dev) -> hipError_t {
        const void *src;
        if (e->prec == HV_FP64) { to_device_order(e->layout, m, host, bd.data()); src = bd.data(); }
        else { to_device_order(e->layout, m, host, bf.data()); src = bf.data(); }
        return hipMemcpy(dev, src, m.ncell * e->esize, hipMemcpyHostToDevice);
    };
    for (int f = 0; f < 5; ++f)
        if ((r = upload(fields[f], m.dev.st[P][f])) != hipSuccess) return hip_fail(e, r, "hipMemcpy(state)");
    if (terrain) {
        const double *refs[3] = {rho_ref, rhotheta_ref, p_ref};
        for (int f = 0; f < 3; ++f)
            if ((r = upload(refs[f], m.dev.ref[f])) != hipSuccess) return hip_fail(e, r, "hipMemcpy(reference)");
    }
    // reference mass: sum of rho_ref J dx dy dzeta (J = 1 on flat ground)
    double s = 0.0, c = 0.0;
    auto add = [&](double x) {
        const double t = s + x;
        c += (std::fabs(s) >= std::fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    };
    const double H = m.zf[m.nz];
    for (int k = 0; k < m.nz; ++k) {
        const double vol = m.dx * m.dy * (m.zf[k + 1] - m.zf[k]);
        if (!terrain) {
            add(rho_ref[k] * vol * (double)nxy);
            continue;
        }
        for (size_t col = 0; col < nxy; ++col)
            add(rho_ref[(size_t)k * nxy + col] * vol * (1.0 - m.h[col] / H));
    }
    m.mass_ref = s + c;
    m.dev.mass_ref = m.mass_ref;
    if ((r = upload_table(e)) != hipSuccess) return hip_fail(e, r, "upload member table");
    const double zero = 0.0;   // model time
    if ((r = hipMemcpy(m.dev.sums + 2, &zero, sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, r, "hipMemcpy(time)");
    m.have_state = true;
    for (auto &g : e->groups) {
        // the mass of this state is the reference of member q's drift check
        hv::Group gm = group_launch(e, g, -1, e->roles[0]);
        gm.mass_init = q + 1;
        r = hv::launch_sums(e->prec, e->layout, g.L, gm, false, e->stream);
        if (r != hipSuccess) return hip_fail(e, r, "mass after state_init");
    }
    if ((r = sync(e)) != hipSuccess) return hip_fail(e, r, "mass after state_init");
    return HV_OK;
}

int ens_step(hv_ens *e, const double *dts, int n_long, int n_short)
{
    for (int q = 0; q < e->n; ++q) {
        if (!e->m[q].have_state) return fail(e, HV_ERR_STATE, "step before every member's state_init");
        if (!(dts[q] > 0.0) || !std::isfinite(dts[q])) return fail(e, HV_ERR_ARG, "dt must be positive");
    }
    if (n_long < 0) return fail(e, HV_ERR_ARG, "n_long must be >= 0");
    if (n_short < 1) return fail(e, HV_ERR_ARG, "n_short must be >= 1");
    hipError_t r;
    bool changed = false;
    for (int q = 0; q < e->n; ++q)
        if (e->m[q].dt != dts[q]) {
            e->m[q].dt = dts[q];
            e->m[q].dev.dt = dts[q];
            changed = true;
        }
    if (changed) {
        // the table is read by running steps: update it between them
        drop_graphs(e);
        if ((r = sync(e)) != hipSuccess) return hip_fail(e, r, "stream synchronize");
        std::vector<hv::MemberDev> table(e->n);
        for (int q = 0; q < e->n; ++q) table[q] = e->m[q].dev;
        r = hipMemcpy(e->d_mem, table.data(), sizeof(hv::MemberDev) * e->n, hipMemcpyHostToDevice);
        if (r != hipSuccess) return hip_fail(e, r, "upload member table");
    }
    if (n_long == 0) return HV_OK;
    if (e->tracing) {
        for (int s = 0; s < n_long; ++s) {
            if ((r = enqueue_long_step(e, n_short, e->roles, e->stream)) != hipSuccess)
                return hip_fail(e, r, "long step");
            rotate_roles(e->roles, n_short);
        }
        return HV_OK;
    }
    // order the private stream after the caller's work, replay, then join back
    if ((r = hipEventRecord(e->fork, e->stream)) != hipSuccess) return hip_fail(e, r, "hipEventRecord");
    if ((r = hipStreamWaitEvent(e->own, e->fork, 0)) != hipSuccess) return hip_fail(e, r, "hipStreamWaitEvent");
    for (int s = 0; s < n_long; ++s) {
        hipGraphExec_t exec = nullptr;
        for (auto &g : e->graphs)
            if (g.n_short == n_short && std::equal(g.roles, g.roles + 3, e->roles)) exec = g.exec;
        if (!exec) {
            hipGraph_t graph = nullptr;
            if ((r = hipStreamBeginCapture(e->own, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return hip_fail(e, r, "hipStreamBeginCapture");
            const hipError_t rl = enqueue_long_step(e, n_short, e->roles, e->own);
            r = hipStreamEndCapture(e->own, &graph);
            if (rl != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return hip_fail(e, rl, "capture long step");
            }
            if (r != hipSuccess) return hip_fail(e, r, "hipStreamEndCapture");
            r = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (r != hipSuccess) return hip_fail(e, r, "hipGraphInstantiate");
            GraphEntry ge{n_short, {e->roles[0], e->roles[1], e->roles[2]}, exec};
            e->graphs.push_back(ge);
        }
        if ((r = hipGraphLaunch(exec, e->own)) != hipSuccess) return hip_fail(e, r, "hipGraphLaunch");
        rotate_roles(e->roles, n_short);
    }
    if ((r = hipEventRecord(e->join, e->own)) != hipSuccess) return hip_fail(e, r, "hipEventRecord");
    if ((r = hipStreamWaitEvent(e->stream, e->join, 0)) != hipSuccess) return hip_fail(e, r, "hipStreamWaitEvent");
    return HV_OK;
}

// HV_ERR_DRIFT once a long step left the member's mass drift bound (the
// device's sticky flag); call with the stream synchronised.
int check_drift(hv_ens *e, const MemberHost &m)
{
    if (!(m.dev.drift_bound > 0.0)) return HV_OK;
    double h[2] = {0.0, 0.0};
    hipError_t r = hipMemcpy(h, m.dev.sums + 4, 2 * sizeof(double), hipMemcpyDeviceToHost);
    if (r != hipSuccess) return hip_fail(e, r, "read drift flag");
    if (h[0] != 0.0) {
        char b[160];
        std::snprintf(b, sizeof b, "mass drift %.3e exceeds the bound %.3e", h[1], m.dev.drift_bound);
        return fail(e, HV_ERR_DRIFT, b);
    }
    return HV_OK;
}

int member_read(hv_ens *e, int q, int field, double *out)
{
    if (q < 0 || q >= e->n) return fail(e, HV_ERR_ARG, "member index out of range");
    if (!out) return fail(e, HV_ERR_ARG, "host_out is NULL");
    if (field < HV_RHO_PTB || field > HV_RHOTHETA_PTB) return fail(e, HV_ERR_ARG, "unknown field id");
    MemberHost &m = e->m[q];
    if (!m.have_state) return fail(e, HV_ERR_STATE, "read before state_init");
    hipError_t r = sync(e);
    if (r != hipSuccess) return hip_fail(e, r, "stream synchronize");
    const void *src = m.dev.st[e->roles[0]][field];
    if (e->prec == HV_FP64) {
        std::vector<double> b(m.ncell);
        if ((r = hipMemcpy(b.data(), src, m.ncell * 8, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(e, r, "hipMemcpy(read)");
        from_device_order(e->layout, m, b.data(), out);
    } else {
        std::vector<float> b(m.ncell);
        if ((r = hipMemcpy(b.data(), src, m.ncell * 4, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(e, r, "hipMemcpy(read)");
        from_device_order(e->layout, m, b.data(), out);
    }
    if (field == HV_RHOW) {
        const size_t nxy = (size_t)m.nx * m.ny;
        for (size_t c = 0; c < nxy; ++c) out[nxy * m.nz + c] = 0.0;
    }
    // failure detection: non-finite values, then the device's drift flag
    const size_t nxy = (size_t)m.nx * m.ny;
    const int levels = field == HV_RHOW ? m.nz + 1 : m.nz;
    std::vector<char> bad(levels, 0);
    parallel_rows(levels, nxy, [&](int k0, int k1) {
        for (int k = k0; k < k1; ++k)
            for (size_t c = 0; c < nxy; ++c)
                if (!std::isfinite(out[(size_t)k * nxy + c])) { bad[k] = 1; break; }
    });
    for (char b : bad)
        if (b) return fail(e, HV_ERR_NONFINITE, "the field holds non-finite values");
    return check_drift(e, m);
}

int member_mass(hv_ens *e, int q, double *mass, double *energy)
{
    if (q < 0 || q >= e->n) return fail(e, HV_ERR_ARG, "member index out of range");
    MemberHost &m = e->m[q];
    if (!m.have_state) return fail(e, HV_ERR_STATE, "mass before state_init");
    hipError_t r;
    if (energy)
        for (auto &g : e->groups) {
            const hv::Group gm = group_launch(e, g, -1, e->roles[0]);
            if ((r = hv::launch_sums(e->prec, e->layout, g.L, gm, true, e->stream)) != hipSuccess)
                return hip_fail(e, r, "energy sum");
        }
    double h[2] = {0.0, 0.0};
    r = hipMemcpyAsync(h, m.dev.sums, 2 * sizeof(double), hipMemcpyDeviceToHost, e->stream);
    if (r == hipSuccess) r = sync(e);
    if (r != hipSuccess) return hip_fail(e, r, "read sums");
    const double ms = m.mass_ref + h[0];
    if (mass) *mass = ms;
    if (energy) *energy = h[1];
    if (!std::isfinite(ms)) return fail(e, HV_ERR_NONFINITE, "mass sum is not finite");
    return check_drift(e, m);
}


int member_damping(hv_ens *e, int q, const double *nu_lat, const double *nu_top,
                   const double *const bnd1[5], const double *const bnd2[5], double t1, double t2,
                   double time_now)
{
    if (q < 0 || q >= e->n) return fail(e, HV_ERR_ARG, "member index out of range");
    MemberHost &m = e->m[q];
    if (!m.damp_room) return fail(e, HV_ERR_ARG, "workspace has no room for damping (desc.damping = 0)");
    if (!nu_lat || !nu_top || !bnd1 || !bnd2) return fail(e, HV_ERR_ARG, "NULL damping array");
    if (!(t2 > t1) || !std::isfinite(t1) || !std::isfinite(t2) || !std::isfinite(time_now))
        return fail(e, HV_ERR_ARG, "need finite t1 < t2 and time_now");
    const size_t nxy = (size_t)m.nx * m.ny;
    for (size_t c = 0; c < nxy; ++c)
        if (!(nu_lat[c] >= 0.0) || !std::isfinite(nu_lat[c])) return fail(e, HV_ERR_ARG, "rates must be finite and >= 0");
    for (int k = 0; k < m.nz; ++k)
        if (!(nu_top[k] >= 0.0) || !std::isfinite(nu_top[k])) return fail(e, HV_ERR_ARG, "rates must be finite and >= 0");
    for (int b = 0; b < 2; ++b) {
        const double *const *bs = b ? bnd2 : bnd1;
        for (int f = 0; f < 5; ++f) {
            if (!bs[f]) return fail(e, HV_ERR_ARG, "NULL boundary field");
            const size_t cnt = f == HV_RHOW ? nxy * (m.nz + 1) : nxy * m.nz;
            for (size_t c = 0; c < cnt; ++c)
                if (!std::isfinite(bs[f][c])) return fail(e, HV_ERR_ARG, "non-finite boundary value");
        }
        for (size_t c = 0; c < nxy; ++c)
            if (bs[HV_RHOW][c] != 0.0 || bs[HV_RHOW][nxy * m.nz + c] != 0.0)
                return fail(e, HV_ERR_ARG, "boundary rho*w must be 0 on both lids");
    }
    hipError_t r = sync(e);
    if (r != hipSuccess) return hip_fail(e, r, "stream synchronize");
    std::vector<double> nu(nxy + m.nz);
    std::copy(nu_lat, nu_lat + nxy, nu.begin());
    std::copy(nu_top, nu_top + m.nz, nu.begin() + nxy);
    if ((r = hipMemcpy(m.d_nu, nu.data(), nu.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, r, "hipMemcpy(rates)");
    std::vector<double> bd;
    std::vector<float> bf;
    if (e->prec == HV_FP64) bd.resize(m.ncell);
    else bf.resize(m.ncell);
    for (int b = 0; b < 2; ++b)
        for (int f = 0; f < 5; ++f) {
            const double *src = (b ? bnd2 : bnd1)[f];
            const void *h;
            if (e->prec == HV_FP64) { to_device_order(e->layout, m, src, bd.data()); h = bd.data(); }
            else { to_device_order(e->layout, m, src, bf.data()); h = bf.data(); }
            if ((r = hipMemcpy(m.dev.bnd[b][f], h, m.ncell * e->esize, hipMemcpyHostToDevice)) != hipSuccess)
                return hip_fail(e, r, "hipMemcpy(boundary)");
        }
    if ((r = hipMemcpy(m.dev.sums + 2, &time_now, sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, r, "hipMemcpy(time)");
    m.dev.nu_lat = m.d_nu;
    m.dev.nu_top = m.d_nu + nxy;
    m.dev.t1 = t1;
    m.dev.t2 = t2;
    if ((r = upload_table(e)) != hipSuccess) return hip_fail(e, r, "upload member table");
    for (auto &g : e->groups)
        if (std::find(g.ids.begin(), g.ids.end(), q) != g.ids.end()) g.damping = true;
    drop_graphs(e);
    return HV_OK;
}

// Per group and kernel kind: the tile x-extent (negative for the
// XCD-chunked order) and the lanes per column of its configuration.
void report_configs(const hv_ens *e, int32_t *tiles, int32_t *lanes, int32_t *ngroups,
                    int32_t *configs = nullptr)
{
    if (ngroups) *ngroups = (int32_t)e->groups.size();
    for (size_t gi = 0; gi < e->groups.size(); ++gi)
        for (int k = 0; k < NKIND; ++k) {
            const GroupHost &g = e->groups[gi];
            const int c = g.shape[k];
            if (configs) configs[gi * NKIND + k] = c;
            if (tiles)
                tiles[gi * NKIND + k] = ((c / 3) % 2 ? -1 : 1) * (1 << shape_log2(c % 3 + 3 * (c / 12))) *
                                        (c / 12 ? kRun : 1);
            const bool w = (c / 6) % 2;
            int n = w ? alt_seg(e->prec, g.L) : default_seg(e->prec, g.L);
            if (e->layout == HV_IJK)
                n = (!w && e->n == 1 && !(k == KIND_SHORT && e->rk2)) ? 1 : default_seg(e->prec, g.L);
            if (lanes) lanes[gi * NKIND + k] = n;
        }
}

// Time one kernel kind of one group in every launch configuration; keep the fastest.
int tune(hv_ens *e, int32_t *out, int32_t *lanes, int32_t *ngroups)
{
    for (int q = 0; q < e->n; ++q)
        if (!e->m[q].have_state) return fail(e, HV_ERR_STATE, "tune before every member's state_init");
    hipError_t r = sync(e);
    if (r != hipSuccess) return hip_fail(e, r, "stream synchronize");
    const bool was_tracing = e->tracing;
    e->tracing = false;
    hipEvent_t a, b;
    if ((r = hipEventCreate(&a)) != hipSuccess) return hip_fail(e, r, "hipEventCreate");
    if ((r = hipEventCreate(&b)) != hipSuccess) { (void)hipEventDestroy(a); return hip_fail(e, r, "hipEventCreate"); }
    const int n_short = 6;
    // stage 1 on the current state; the short step writes a running buffer
    auto launch = [&](const GroupHost &g, int kind, hipStream_t s) -> hipError_t {
        const hv::Group gr = group_launch(e, g, kind, e->roles[0], e->roles[1]);
        if (kind == KIND_PREP) return hv::launch_slow_prep(e->prec, e->layout, g.L, gr, s);
        if (kind == KIND_FLUX) return hv::launch_slow_flux(e->prec, e->layout, g.L, gr, s);
        return hv::launch_short_step(e->prec, e->layout, g.L, gr, 1.0 / (3.0 * n_short), 0.0, s);
    };
    int rc = HV_OK;
    for (auto &g : e->groups) {
        for (int kind = 0; kind < NKIND && rc == HV_OK; ++kind) {
            // three interleaved rounds, the fastest of each configuration's
            // timings counts (one round alone let run-to-run noise decide)
            const int nconf = configs_of(e, kind);
            float t[kConfigs];
            std::fill(t, t + kConfigs, 1e30f);
            for (int it = 0; it < 3 * nconf && rc == HV_OK; ++it) {
                const int s = it % nconf;
                g.shape[kind] = s;
                // the slow arrays the flux and short step read must hold this stage's values
                if ((r = launch(g, KIND_PREP, e->stream)) != hipSuccess ||
                    (kind == KIND_SHORT && (r = launch(g, KIND_FLUX, e->stream)) != hipSuccess) ||
                    (r = launch(g, kind, e->stream)) != hipSuccess ||
                    (r = hipEventRecord(a, e->stream)) != hipSuccess) { rc = hip_fail(e, r, "tune"); break; }
                for (int rep = 0; rep < 4; ++rep)
                    if ((r = launch(g, kind, e->stream)) != hipSuccess) break;
                if (r == hipSuccess) r = hipEventRecord(b, e->stream);
                if (r == hipSuccess) r = hipEventSynchronize(b);
                float ms = 0.f;
                if (r == hipSuccess) r = hipEventElapsedTime(&ms, a, b);
                if (r != hipSuccess) { rc = hip_fail(e, r, "tune"); break; }
                t[s] = std::min(t[s], ms);
            }
            g.shape[kind] = (int)(std::min_element(t, t + nconf) - t);
        }
        if (rc != HV_OK) break;
        cache_store(tune_key(e, g), g.shape);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    e->tracing = was_tracing;
    if (rc != HV_OK) return rc;
    drop_graphs(e);
    report_configs(e, out, lanes, ngroups);
    return HV_OK;
}

// Set the launch configurations of group gi (config[k] per kernel kind, as
// the tuner numbers them).
int configure(hv_ens *e, int gi, const int32_t *config)
{
    if (gi < 0 || gi >= (int)e->groups.size()) return fail(e, HV_ERR_ARG, "group index out of range");
    if (!config) return fail(e, HV_ERR_ARG, "config is NULL");
    for (int k = 0; k < NKIND; ++k)
        if (config[k] < 0 || config[k] >= configs_of(e, k))
            return fail(e, HV_ERR_ARG, "configuration index out of range");
    hipError_t r = sync(e);   // running steps use the current graphs
    if (r != hipSuccess) return hip_fail(e, r, "stream synchronize");
    for (int k = 0; k < NKIND; ++k) e->groups[gi].shape[k] = config[k];
    drop_graphs(e);
    return HV_OK;
}

int trace_on(hv_ens *e, int32_t on)
{
    if (on) {
        hipError_t r = fold_trace(e);
        if (r != hipSuccess) return hip_fail(e, r, "trace");
        for (int k = 0; k < HV_K_COUNT; ++k) { e->trace_ms[k] = 0.0; e->trace_n[k] = 0; }
    }
    e->tracing = on != 0;
    return HV_OK;
}

int trace_read(hv_ens *e, int32_t kind, double *ms, int64_t *n)
{
    if (kind < 0 || kind >= HV_K_COUNT) return fail(e, HV_ERR_ARG, "unknown kernel kind");
    hipError_t r = fold_trace(e);
    if (r != hipSuccess) return hip_fail(e, r, "trace read");
    if (ms) *ms = e->trace_ms[kind];
    if (n) *n = e->trace_n[kind];
    return HV_OK;
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------- grid ---
size_t hv_workspace_bytes(const hv_grid_desc *desc)
{
    return hv_ens_workspace_bytes(1, desc);
}

int hv_grid_create(const hv_grid_desc *desc, void *dev_workspace, size_t bytes, void *hip_stream,
                   hv_grid_t *out)
{
    if (!out) return fail(nullptr, HV_ERR_ARG, "out is NULL");
    *out = nullptr;
    hv_grid *g = new (std::nothrow) hv_grid();
    if (!g) return fail(nullptr, HV_ERR_ARG, "out of host memory");
    const int rc = ens_create(g, 1, desc, dev_workspace, bytes, hip_stream);
    if (rc != HV_OK) { delete g; return rc; }
    // set-up of the allocation-free sums: the device address of the library
    // scratch on this device (looked up once per device)
    const hipError_t r = hv::scratch_address(&g->scratch);
    if (r != hipSuccess) { delete g; return hip_fail(nullptr, r, "scratch address"); }
    *out = g;
    return HV_OK;
}

int hv_state_init(hv_grid_t g, const double *const fields[5], const double *rho_ref,
                  const double *rhotheta_ref, const double *p_ref)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return member_init(g, 0, fields, rho_ref, rhotheta_ref, p_ref);
}

int hv_step(hv_grid_t g, double dt, int32_t n_long, int32_t n_short)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (!g->m[0].have_state) return fail(g, HV_ERR_STATE, "hv_step before hv_state_init");
    return ens_step(g, &dt, n_long, n_short);
}

int hv_state_read(hv_grid_t g, int32_t field, double *host_out)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return member_read(g, 0, field, host_out);
}

int hv_mass(hv_grid_t g, double *mass_out, double *energy_out)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return member_mass(g, 0, mass_out, energy_out);
}

int hv_mass_noalloc(hv_grid_t g, double *dev_out)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (!dev_out) return fail(g, HV_ERR_ARG, "dev_out is NULL");
    const MemberHost &m = g->m[0];
    if (!m.have_state) return fail(g, HV_ERR_STATE, "mass before state_init");
    if (m.dev.npart > hv::kScratchDoubles) {
        char b[128];
        std::snprintf(b, sizeof b, "grid needs %d partial sums, the scratch holds %d", m.dev.npart,
                      hv::kScratchDoubles);
        return fail(g, HV_ERR_ARG, b);
    }
    if (!g->scratch) return fail(g, HV_ERR_STATE, "no scratch address on this device");
    hv::Group gm = group_launch(g, g->groups[0], -1, g->roles[0]);
    gm.part = g->scratch;
    gm.out = dev_out;
    gm.out_add = m.mass_ref;
    hipError_t r = hv::launch_sums(g->prec, g->layout, g->groups[0].L, gm, false, g->stream);
    if (r == hipSuccess) r = hv::launch_sums(g->prec, g->layout, g->groups[0].L, gm, true, g->stream);
    if (r != hipSuccess) return hip_fail(g, r, "allocation-free sums");
    return HV_OK;
}

int hv_tune(hv_grid_t g, int32_t *tile_x_out, int32_t *lanes_out)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return tune(g, tile_x_out, lanes_out, nullptr);
}

int hv_configure(hv_grid_t g, const int32_t config[3], int32_t *config_out, int32_t *tile_x_out,
                 int32_t *lanes_out)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (config) {
        const int rc = configure(g, 0, config);
        if (rc != HV_OK) return rc;
    }
    report_configs(g, tile_x_out, lanes_out, nullptr, config_out);
    return HV_OK;
}

int hv_damping(hv_grid_t g, const double *nu_lat, const double *nu_top,
               const double *const bnd1[5], const double *const bnd2[5], double t1, double t2,
               double time_now)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return member_damping(g, 0, nu_lat, nu_top, bnd1, bnd2, t1, t2, time_now);
}

int hv_trace(hv_grid_t g, int32_t on)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return trace_on(g, on);
}

int hv_trace_read(hv_grid_t g, int32_t kind, double *ms_total, int64_t *launches)
{
    if (!g) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return trace_read(g, kind, ms_total, launches);
}

void hv_grid_destroy(hv_grid_t g) { delete g; }

const char *hv_last_error(hv_grid_t g) { return g ? g->err.c_str() : g_global_error.c_str(); }

// ------------------------------------------------------------ ensemble ---
size_t hv_ens_workspace_bytes(int32_t n, const hv_grid_desc *descs)
{
    if (n < 1 || !descs) { g_global_error = "need n >= 1 member descriptions"; return 0; }
    for (int q = 0; q < n; ++q) {
        std::string why = check_desc(&descs[q]);
        if (!why.empty()) { g_global_error = (n > 1 ? "member " + std::to_string(q) + ": " : "") + why; return 0; }
        if (descs[q].precision != descs[0].precision || descs[q].layout != descs[0].layout ||
            descs[q].short_scheme != descs[0].short_scheme) {
            g_global_error = "all members must share precision, layout and short_scheme";
            return 0;
        }
    }
    return make_plan(n, descs).total;
}

int hv_ens_create(int32_t n, const hv_grid_desc *descs, void *ws, size_t bytes, void *stream,
                  hv_ens_t *out)
{
    if (!out) return fail(nullptr, HV_ERR_ARG, "out is NULL");
    *out = nullptr;
    hv_ens *e = new (std::nothrow) hv_ens();
    if (!e) return fail(nullptr, HV_ERR_ARG, "out of host memory");
    const int rc = ens_create(e, n, descs, ws, bytes, stream);
    if (rc != HV_OK) { delete e; return rc; }
    *out = e;
    return HV_OK;
}

int hv_ens_state_init(hv_ens_t e, int32_t member, const double *const fields[5],
                      const double *rho_ref, const double *rhotheta_ref, const double *p_ref)
{
    if (!e) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return member_init(e, member, fields, rho_ref, rhotheta_ref, p_ref);
}

int hv_ens_step(hv_ens_t e, const double *dt_per_member, int32_t n_long, int32_t n_short)
{
    if (!e) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (!dt_per_member) return fail(e, HV_ERR_ARG, "dt_per_member is NULL");
    return ens_step(e, dt_per_member, n_long, n_short);
}

int hv_ens_state_read(hv_ens_t e, int32_t member, int32_t field, double *host_out)
{
    if (!e) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return member_read(e, member, field, host_out);
}

int hv_ens_mass(hv_ens_t e, int32_t member, double *mass_out, double *energy_out)
{
    if (!e) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return member_mass(e, member, mass_out, energy_out);
}

int hv_ens_tune(hv_ens_t e, int32_t *tile_x_out, int32_t *lanes_out, int32_t *ngroups_out)
{
    if (!e) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return tune(e, tile_x_out, lanes_out, ngroups_out);
}

int hv_ens_configure(hv_ens_t e, int32_t group, const int32_t config[3], int32_t *config_out,
                     int32_t *tile_x_out, int32_t *lanes_out, int32_t *ngroups_out)
{
    if (!e) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    if (config) {
        const int rc = configure(e, group, config);
        if (rc != HV_OK) return rc;
    }
    report_configs(e, tile_x_out, lanes_out, ngroups_out, config_out);
    return HV_OK;
}

int hv_ens_damping(hv_ens_t e, int32_t member, const double *nu_lat, const double *nu_top,
                   const double *const bnd1[5], const double *const bnd2[5], double t1, double t2,
                   double time_now)
{
    if (!e) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return member_damping(e, member, nu_lat, nu_top, bnd1, bnd2, t1, t2, time_now);
}

int hv_ens_trace(hv_ens_t e, int32_t on)
{
    if (!e) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return trace_on(e, on);
}

int hv_ens_trace_read(hv_ens_t e, int32_t kind, double *ms_total, int64_t *launches)
{
    if (!e) return fail(nullptr, HV_ERR_ARG, "handle is NULL");
    return trace_read(e, kind, ms_total, launches);
}

void hv_ens_destroy(hv_ens_t e) { delete e; }

// ------------------------------------------------------- 7-point stencil ---
int hv_diffuse(int32_t nx, int32_t ny, int32_t nz, int32_t precision, int32_t layout, double kx,
               double ky, double kz, int32_t tile_x, const void *dev_in, void *dev_out,
               void *hip_stream)
{
    if (nx < 1 || ny < 1) return fail(nullptr, HV_ERR_ARG, "nx and ny must be >= 1");
    if (nz != 32 && nz != 64 && nz != 128) return fail(nullptr, HV_ERR_ARG, "nz must be 32, 64 or 128");
    if ((size_t)nx * (size_t)ny > (size_t)INT32_MAX / 2) return fail(nullptr, HV_ERR_ARG, "too many columns");
    if (precision != HV_FP64 && precision != HV_FP32)
        return fail(nullptr, HV_ERR_ARG, "precision must be HV_FP64 or HV_FP32");
    if (layout != HV_IJK && layout != HV_KIJ) return fail(nullptr, HV_ERR_ARG, "unknown layout");
    if (!std::isfinite(kx) || !std::isfinite(ky) || !std::isfinite(kz))
        return fail(nullptr, HV_ERR_ARG, "coefficients must be finite");
    if (!dev_in || !dev_out) return fail(nullptr, HV_ERR_ARG, "NULL device array");
    if (dev_in == dev_out) return fail(nullptr, HV_ERR_ARG, "dev_in and dev_out must differ");
    if (((uintptr_t)dev_in | (uintptr_t)dev_out) % 64)
        return fail(nullptr, HV_ERR_ARG, "device arrays must be 64-byte aligned");
    int tl = -1;
    for (int sh = 0; sh < 3; ++sh)
        if (tile_x == (1 << kShapes[sh])) tl = kShapes[sh];
    if (tl < 0) return fail(nullptr, HV_ERR_ARG, "tile_x must be 16, 8 or 4");
    hv::DiffArgs a{};
    a.nx = nx; a.ny = ny; a.nz = nz; a.ti_log2 = tl;
    a.kx = kx; a.ky = ky; a.kz = kz;
    a.in = dev_in; a.out = dev_out;
    const hipError_t r = hv::launch_diffuse(precision == HV_FP64 ? 0 : 1, layout, nz / hv::kSeg, a,
                                            (hipStream_t)hip_stream);
    if (r != hipSuccess) return hip_fail(nullptr, r, "diffuse launch");
    return HV_OK;
}

const char *hv_ens_last_error(hv_ens_t e) { return e ? e->err.c_str() : g_global_error.c_str(); }

}  // extern "C"
