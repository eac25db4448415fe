// hevi_kernels.h -- device-side member table and the host launchers of the
// HEVI step kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace hv {

constexpr int kSeg = 16;               // lanes per column
constexpr int kBlock = 256;            // threads per block
constexpr int kColsPerBlock = kBlock / kSeg;
constexpr int kMaxPartials = 1024;     // mass-sum partials per member

// Per-level constant table: VM_NFIELDS * nz float64 values, entry f*nz + k,
// followed by the same values rounded to float32 in the same order (float
// kernels read that copy: half the registers and load instructions, and the
// same values they would get by converting).
enum VmField {
    VM_DZ = 0,     // cell thickness dz_k
    VM_RDZ,        // 1/dz_k
    VM_DZF,        // centre-to-centre distance at level face k (k >= 1)
    VM_RDZF,       // 1/dzf_k
    VM_A,          // weight of cell k in the linear interpolation to face k
    VM_B,          // weight of cell k-1
    VM_RHO,        // reference density at the centre of cell k
    VM_RT,         // reference rho*theta
    VM_P,          // reference pressure
    VM_VOL,        // cell volume dx*dy*dz_k
    VM_ZC,         // height of the centre of cell k
    VM_DC,         // 1 - zeta/H at the centre of cell k (terrain decay)
    VM_DF,         // 1 - zeta/H at level face k
    VM_NFIELDS
};

inline constexpr size_t vm_bytes(int nz)
{
    return (sizeof(double) + sizeof(float)) * (size_t)VM_NFIELDS * (size_t)nz;
}

// Per-column geometry of a terrain-following grid (float64, 8 per column,
// column-major i-fastest): Jacobians and slopes of z = zeta + h (1 - zeta/H).
enum GeoField {
    GEO_J = 0,     // J = 1 - h/H of the column
    GEO_JU,        // J on the west x-face (mean of the two columns)
    GEO_JV,        // J on the south y-face
    GEO_SU,        // dh/dx on the west x-face
    GEO_SV,        // dh/dy on the south y-face
    GEO_H,         // surface height h
    GEO_NFIELDS = 8
};

// One domain as every kernel sees it: sizes, spacings, long step and the
// device arrays carved from the workspace.
struct MemberDev {
    int nx, ny, nz, npart;       // npart: mass partials of this member
    double rdx, rdy, beta, dt;   // dt: long step of this member
    const double *vm;
    double *partials;
    double *sums;                // [0] perturbation mass, [1] energy, [2] model time,
                                 // [3] perturbation mass at state_init, [4] drift
                                 // flag (1 once the bound was crossed), [5] largest
                                 // relative drift seen
    double mass_ref;             // reference mass (rho_ref J dx dy dzeta summed)
    double drift_bound;          // relative mass drift bound, <= 0: no check
    void *st[4][5];              // rho', U, V, W, Theta' of the state buffers
                                 // ([3]: first-stage value of the Runge-Kutta short step)
    void *slow[7];               // S_U, S_V, S_W, R_Theta, theta_s, P0_s, C_s
    void *spec[4];               // u, v, w of the stage input; [3] Omega (terrain)
    const double *geo;           // terrain: GEO_NFIELDS per column, else null
    void *ref[3];                // terrain: rho_ref, rhotheta_ref, p_ref per cell
    // lateral / upper damping (nu_lat null: none)
    const double *nu_lat;        // per column (nx*ny)
    const double *nu_top;        // per level (nz)
    void *bnd[2][5];             // boundary states at t1 and t2 (device layout)
    double t1, t2;
    void *col[4];                // i-fastest layout: the column solve's modified
                                 // upper diagonal and right-hand side and the
                                 // rho', Theta' of the W+ = 0 state (solve precision)
};

// One launch over the blocks of a group of members (all with the same nz).
// A group of one member names it directly; a larger group maps each block to
// (member id, tile) through a per-block table.
struct Group {
    const MemberDev *mem;   // device member table
    const int *ids;         // device: member ids of the group
    const unsigned *blk;    // device: per block, member id << 24 | tile (nm > 1)
    int nm;                 // members in the group
    int first;              // member id when nm == 1
    int nblocks;            // blocks of the launch
    int ti_log2;            // tile = (1 << ti_log2) columns along x by 16 >> ti_log2 along y
    int src, dst;           // state buffers read and written by this launch
    int ev;                 // short step: buffer of the explicit / old-time terms (src: forward-backward)
    int terrain;            // members of the group are terrain-following
    int damp;               // short step: damp the new values (members with damping data)
    int xcd;                // 1: blocks in XCD-chunked order (see block_order)
    int off32;              // 1: every array of every member is under 4 GiB
    int seg;                // lanes per column (8, 16, 32; 0: the default)
    int colmap;             // i-fastest layout, one member: one lane per column
    int nx1, ny1;           // columns of the member when nm == 1
    int rev;                // 1: blocks take the tiles in reverse order (each launch
                            // starts where the previous one ended, whose data the
                            // caches still hold)
    int run;                // slow flux, column-fastest layout: > 1 = columns per
                            // segment run along x (blocks cover runs, see
                            // tiles_of_run); else one column per segment
    // sums only (single member): null, or partials in this array and the
    // final sums written to out[slot] (the mass slot with out_add added)
    double *part;
    double *out;
    double out_add;
    int mass_init;          // sums: member id + 1 whose mass is recorded as its
                            // state_init value (0: none)
};
constexpr int kSums = 8;    // doubles of a member's sums array

// Blocks a member needs for a tile shape.
inline int tiles_of(int nx, int ny, int ti_log2)
{
    const int ti = 1 << ti_log2, tj = kColsPerBlock >> ti_log2;
    return ((nx + ti - 1) / ti) * ((ny + tj - 1) / tj);
}
// Blocks a member needs for a tile shape whose columns along x are runs of
// run columns each.
inline int tiles_of_run(int nx, int ny, int ti_log2, int run)
{
    const int span = (1 << ti_log2) * run, tj = kColsPerBlock >> ti_log2;
    return ((nx + span - 1) / span) * ((ny + tj - 1) / tj);
}
inline int partials_of(int nx, int ny)
{
    const int t = tiles_of(nx, ny, 4);
    return t < kMaxPartials ? t : kMaxPartials;
}

// prec: 0 float64, 1 float32, 2 float32 sweeps + float64 column solve.
// layout: 0 i-fastest, 1 column-fastest.  L = nz / 16.
// Slow sweep of stage `stage` on buffer gr.src.
hipError_t launch_slow_prep(int prec, int layout, int L, const Group &gr, hipStream_t s);
hipError_t launch_slow_flux(int prec, int layout, int L, const Group &gr, hipStream_t s);
// Short step gr.src -> gr.dst of length (member dt) * frac, explicit and
// old-time terms from gr.ev; with gr.damp, damping at model time
// sums[2] + offset * dt.
hipError_t launch_short_step(int prec, int layout, int L, const Group &gr, double frac, double offset,
                             hipStream_t s);
// The one-lane-per-column kernels of the i-fastest layout for a single
// member (gr.nm == 1, dims gr.nx1 x gr.ny1): kind 0 slow prep, 1 slow flux,
// 2 forward-backward undamped short step of length (member dt) * frac.
hipError_t launch_columns(int kind, int prec, const Group &gr, double frac, hipStream_t s);
// One thread per member of the group: model time += dt (end of a long step).
hipError_t launch_clock(const Group &gr, hipStream_t s);
// gr.blk maps blocks to (member, partial).  Sums the perturbation mass
// (energy = false) or the total energy of buffer gr.src into each member's sums.
hipError_t launch_sums(int prec, int layout, int L, const Group &gr, bool energy, hipStream_t s);

// Library-owned device scratch of the allocation-free sums: room for
// kScratchDoubles float64 values (the partials of one grid) on every device
// the library runs on.  *out receives its device address on the current
// device, looked up once per device and kept.
constexpr int kScratchDoubles = kMaxPartials;
hipError_t scratch_address(double **out);

// Seven-point diffusion step on one device array (nx*ny*nz values of type
// prec 0 = double, 1 = float, in `layout`): out = q + kx lx + ky ly + kz lz.
struct DiffArgs {
    int nx, ny, nz, ti_log2;
    double kx, ky, kz;
    const void *in;
    void *out;
};
hipError_t launch_diffuse(int prec, int layout, int L, const DiffArgs &a, hipStream_t s);

}  // namespace hv
