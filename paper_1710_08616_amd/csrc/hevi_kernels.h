// hevi_kernels.h -- host-side launchers of the HEVI step kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace hv {

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

struct Geom {
    int nx, ny, nz;
    double rdx, rdy;     // 1/dx, 1/dy
    double beta;         // off-centring of the vertical coupling
};

// prec: 0 float64, 1 float32, 2 float32 sweeps + float64 column solve.
// layout: 0 i-fastest, 1 column-fastest.
// Arrays are device pointers of the grid's storage type.

// st = {rho', U, V, W, Theta'}; prep = {u, v, w, theta_s, P0_s, C_s}
hipError_t launch_slow_prep(int prec, int layout, const Geom &g, const double *vm,
                            const void *const st[5], void *const prep[6], hipStream_t s);

// uvw = {U, V, W}; spec = {u, v, w, theta_s}; out = {S_U, S_V, S_W, R_Theta}
hipError_t launch_slow_flux(int prec, int layout, const Geom &g, const double *vm,
                            const void *const uvw[3], const void *const spec[4],
                            void *const out[4], hipStream_t s);

// in/out = {rho', U, V, W, Theta'} (distinct buffers);
// slow = {S_U, S_V, S_W, R_Theta, theta_s, P0_s, C_s}
hipError_t launch_short_step(int prec, int layout, const Geom &g, const double *vm,
                             const void *const in[5], void *const out[5],
                             const void *const slow[7], double dtau, hipStream_t s);

// Number of float64 partials launch_mass writes (one per block).
int mass_partials(const Geom &g);

// partial[b] = sum of rho' * vol over block b's columns; then one block sums
// the partials in order into *out (out[0] = perturbation mass).
hipError_t launch_mass(int prec, int layout, const Geom &g, const double *vm, const void *rp,
                       double *partials, double *out, hipStream_t s);

// Diagnostic energy sum of the state st into *out (same two-level order).
hipError_t launch_energy(int prec, int layout, const Geom &g, const double *vm,
                         const void *const st[5], double *partials, double *out, hipStream_t s);

}  // namespace hv
