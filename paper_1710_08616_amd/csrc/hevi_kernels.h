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

// Per-level constant table (float64), entry f*nz + k.
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
    VM_NFIELDS
};

// One domain as every kernel sees it (device memory, one record per member).
// roles[0] is the buffer holding the state at the start of a long step (and
// the current state between steps); roles[1], roles[2] are the two running
// buffers.  The rotate kernel updates roles at the end of each long step, so
// one captured launch sequence serves every long step.
struct MemberDev {
    int nx, ny, nz, npart;       // npart: mass partials of this member
    int roles[4];
    double rdx, rdy, beta, dt;   // dt: long step of this member
    const double *vm;
    double *partials;
    double *sums;                // [0] perturbation mass, [1] energy
    void *st[3][5];              // rho', U, V, W, Theta' of the three buffers
    void *slow[7];               // S_U, S_V, S_W, R_Theta, theta_s, P0_s, C_s
    void *spec[3];               // u, v, w of the stage input
};

// One launch covering the blocks of a group of members (all with the same nz).
struct Group {
    const MemberDev *mem;   // device member table
    const int *ids;         // device: member ids of the group (nm)
    const int *prefix;      // device: prefix sums of the members' block counts (nm + 1)
    int nm;                 // members in the group
    int nblocks;            // blocks of the launch (= prefix[nm])
    int ti_log2;            // tile = (1 << ti_log2) columns along x by 16 >> ti_log2 along y
};

// Blocks a member needs for a tile shape.
inline int tiles_of(int nx, int ny, int ti_log2)
{
    const int ti = 1 << ti_log2, tj = kColsPerBlock >> ti_log2;
    return ((nx + ti - 1) / ti) * ((ny + tj - 1) / tj);
}
inline int partials_of(int nx, int ny)
{
    const int t = tiles_of(nx, ny, 4);
    return t < kMaxPartials ? t : kMaxPartials;
}

// prec: 0 float64, 1 float32, 2 float32 sweeps + float64 column solve.
// layout: 0 i-fastest, 1 column-fastest.  L = nz / 16.
hipError_t launch_slow_prep(int prec, int layout, int L, const Group &gr, int stage, int n_short,
                            hipStream_t s);
hipError_t launch_slow_flux(int prec, int layout, int L, const Group &gr, int stage, int n_short,
                            hipStream_t s);
hipError_t launch_short_step(int prec, int layout, int L, const Group &gr, int stage, int sub,
                             int n_short, hipStream_t s);
// gr: prefix over the members' partial counts.  Sums the perturbation mass
// (energy = false) or the total energy of the current state into sums.
hipError_t launch_sums(int prec, int layout, int L, const Group &gr, bool energy, hipStream_t s);
// After the last short step: make the long step's result the current state.
hipError_t launch_rotate(MemberDev *mem, int n, int n_short, hipStream_t s);
// Set the long-step length of member q.
hipError_t launch_set_dt(MemberDev *mem, int q, double dt, hipStream_t s);

}  // namespace hv
