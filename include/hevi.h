/*
 * hevi.h -- C ABI of the HEVI dynamical-core step on AMD Instinct (gfx950).
 *
 * The operation: one long time step of a compressible, non-hydrostatic
 * dynamical core on a 3D structured grid, as outlined in the paper's
 * Sect. 1.1 ("ASUCA on GPU"): finite-volume discretisation, a third-order
 * Runge-Kutta long step (Wicker & Skamarock 2002), and horizontally-explicit /
 * vertically-implicit (HEVI) short steps for sound and gravity waves, with the
 * vertical coupling solved as one tridiagonal system per column.  Prognostic
 * density and rho*theta are stored as perturbations on a reference column, as
 * the paper's Listing 1 does for density (Sect. 2.1).  The paper's device data
 * region model (Sect. 2.2, "Device Data Region": copy in once at the start,
 * copy out at output, nothing in between) is the shape of this interface.
 *
 * Conventions
 *  - Host arrays are float64 in canonical i-fastest order, index
 *    i + nx*(j + ny*k).  Cell fields have nx*ny*nz values; the vertical
 *    momentum rho*w has nx*ny*(nz+1) values (level faces 0..nz), and its
 *    two lid levels must be 0.  U = rho*u sits on the west face of cell i,
 *    V = rho*v on the south face of cell j; the domain is periodic in x and y.
 *  - Terrain (optional): surface heights h(x, y) give the terrain-following
 *    height z = zeta + h (1 - zeta/H) of Gal-Chen & Somerville (1975), with
 *    H = zeta_faces[nz].  Cell volumes are J dx dy dzeta with J = 1 - h/H per
 *    column; horizontal mass fluxes carry the face J (mean of the two
 *    columns); the flux through the zeta surfaces is
 *    Omega = W - (1 - zeta/H) (dh/dx U + dh/dy V, face slopes as differences
 *    of h, averaged to the level face) and is zero on both lids, where W is
 *    held at 0; the horizontal pressure gradient along a zeta surface is
 *    corrected by (dz/dx / J) dp'/dzeta.  The paper's Sect. 1.1 fixes the
 *    finite-volume form; the coordinate is a stated reading.
 *  - Host pointers are borrowed for the duration of the call only.
 *  - Device memory: the caller owns one workspace of at least
 *    hv_workspace_bytes() bytes (any device allocation, 256-byte aligned);
 *    the library carves all its device arrays out of it and allocates no
 *    device memory of its own.
 *  - Streams: every launch goes to the hipStream_t given at creation.
 *    hv_step only enqueues work; hv_state_read and hv_mass synchronise the
 *    stream.
 *  - Errors: every int-returning call returns HV_OK (0) or a negative code;
 *    hv_last_error(handle) gives a text (hv_last_error(NULL) the text of the
 *    last failure of a call that had no valid handle).  No C++ exception
 *    crosses the ABI.  A handle is not thread-safe; distinct handles may be
 *    used from distinct threads.
 */
#ifndef HEVI_H
#define HEVI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hv_grid *hv_grid_t;
typedef struct hv_ens *hv_ens_t;

enum {
    HV_OK = 0,
    HV_ERR_ARG = -1,          /* invalid argument, size, shape or workspace   */
    HV_ERR_HIP = -2,          /* a HIP runtime call failed (see hv_last_error)*/
    HV_ERR_STATE = -3,        /* step/read/mass before hv_state_init          */
    HV_ERR_NONFINITE = -4,    /* the FP64 mass sum is not finite              */
    HV_ERR_UNSUPPORTED = -5,  /* valid request the library does not implement */
    HV_ERR_DRIFT = -6         /* the total mass left the grid's drift bound    */
};

/* Arithmetic of the stencil sweeps / of the column solve and global sums:
 * HV_FP64  float64 / float64,
 * HV_FP32  float32 / float32 (mass sums still float64),
 * HV_MIXED float32 storage and sweeps / float64 vertical solve and sums. */
enum { HV_FP64 = 0, HV_FP32 = 1, HV_MIXED = 2 };

/* Device storage order (the paper's layout question, Sect. 1.3), each with
 * its own mapping.  HV_KIJ (column-fastest, k + nz*(i + nx*j)): a column is a
 * segment of 8/16/32 lanes, each lane owning consecutive levels, the column
 * solve inside the segment.  HV_IJK (i-fastest, i + nx*(j + ny*k)): one lane
 * per column, 64 consecutive columns per wavefront, the k loop inside each
 * lane and a serial Thomas sweep per column (single grids; ensembles, the
 * Runge-Kutta short step and the damped short step run the column-segment
 * kernels on this storage, with strided column access). */
enum { HV_IJK = 0, HV_KIJ = 1 };

/* Short-step integrator.  HV_SHORT_FB: forward-backward HEVI step
 * (horizontal momentum first, then the divergences of the new momentum and
 * the beta-off-centred vertical coupling; one column solve).  HV_SHORT_RK2:
 * the paper's second-order Runge-Kutta short step (Sect. 1.1), read as the
 * midpoint rule over that step: X* = Phi(X, X, dtau/2), X+ = Phi(X, X*, dtau),
 * where Phi(X_b, X_e, d) adds its increments to X_b and takes p' of the
 * horizontal pressure gradient and the old-time (1 - beta) parts of the
 * vertical coupling from X_e; two column solves per short step, damping for
 * sound waves where the forward-backward step is neutral. */
enum { HV_SHORT_FB = 0, HV_SHORT_RK2 = 1 };

/* Field ids for hv_state_read. */
enum { HV_RHO_PTB = 0, HV_RHOU = 1, HV_RHOV = 2, HV_RHOW = 3, HV_RHOTHETA_PTB = 4 };

typedef struct {
    int32_t nx, ny, nz;        /* cells; nx, ny >= 4; nz in {32, 64, 128}    */
    double dx, dy;             /* horizontal spacing (m), > 0                */
    const double *zeta_faces;  /* nz+1 increasing level heights, [0] = 0     */
    const double *terrain;     /* NULL (flat) or nx*ny surface heights h (m),
                                  i fastest, with 1 - h/H >= 0.1; borrowed
                                  during create                             */
    int32_t precision;         /* HV_FP64 / HV_FP32 / HV_MIXED               */
    int32_t layout;            /* HV_KIJ or HV_IJK                           */
    double beta;               /* off-centring of the vertical solve, in [0.5, 1] */
    double div_damp;           /* must be 0                                  */
    int32_t short_scheme;      /* HV_SHORT_FB or HV_SHORT_RK2                */
    int32_t damping;           /* 1: reserve workspace for hv_damping        */
    double mass_drift_bound;   /* failure detection: after every long step the
                                  device compares the total mass M with M0 of
                                  hv_state_init; |M - M0| / M0 above this bound
                                  (or a non-finite M) sets a sticky flag that
                                  hv_mass and hv_state_read report as
                                  HV_ERR_DRIFT.  0: the default, 1e-9 (far
                                  above the rounding drift of any precision),
                                  or no check when damping = 1 (relaxation
                                  toward boundary data does not conserve
                                  mass); < 0: no check                        */
} hv_grid_desc;

/* Bytes of device workspace the grid needs; 0 if the description is invalid
 * (the reason is then in hv_last_error(NULL)).  Host-only, no HIP call. */
size_t hv_workspace_bytes(const hv_grid_desc *desc);

/* Create a grid.  dev_workspace: caller-owned device memory of `bytes`
 * bytes (>= hv_workspace_bytes), kept alive until hv_grid_destroy.
 * hip_stream: a hipStream_t (NULL = the default stream).  On success *out
 * receives the handle. */
int hv_grid_create(const hv_grid_desc *desc, void *dev_workspace, size_t bytes,
                   void *hip_stream, hv_grid_t *out);

/* Load a state (the paper's copy-in at the start of a run).  fields[f] for
 * f = HV_RHO_PTB..HV_RHOTHETA_PTB as described above; rho_ref, rhotheta_ref
 * and p_ref are the reference state at the cell centres: nz values (one
 * column) on flat ground, nx*ny*nz values in canonical order over terrain.
 * Values are converted to the grid's precision and layout.  Non-finite
 * input, non-positive reference values, or a non-zero rho*w on a lid,
 * returns HV_ERR_ARG.  Synchronises the stream. */
int hv_state_init(hv_grid_t g, const double *const fields[5], const double *rho_ref,
                  const double *rhotheta_ref, const double *p_ref);

/* Enqueue n_long RK3 long steps of length dt (s) with n_short HEVI short
 * steps per stage (stage lengths dt/3, dt/2, dt; each stage restarts its
 * short steps from the state at the start of the long step).  After every
 * long step the total mass is summed in float64.  The launch sequence of a
 * long step is recorded once per n_short as a hipGraph and replayed on a
 * private stream ordered after, and joined back into, the grid's stream
 * (while hv_trace is on, the kernels are launched directly instead).
 * Asynchronous: faults and non-finite mass surface at the next
 * hv_state_read / hv_mass. */
int hv_step(hv_grid_t g, double dt, int32_t n_long, int32_t n_short);

/* Copy one field back to the host in canonical float64 layout (the paper's
 * copy-out at output time).  host_out holds nx*ny*nz values, or
 * nx*ny*(nz+1) for HV_RHOW.  Synchronises the stream.  The values are
 * written in every case; the call then returns HV_ERR_NONFINITE if any of
 * them is not finite, else HV_ERR_DRIFT if the mass drift bound was crossed
 * since hv_state_init. */
int hv_state_read(hv_grid_t g, int32_t field, double *host_out);

/* Total mass sum (rho_ref + rho') J dx dy dzeta and the diagnostic total energy
 * (kinetic + internal + potential) of the current state, in float64 with a
 * fixed summation order.  Either output pointer may be NULL.  Returns
 * HV_ERR_NONFINITE if the mass of the current state is not finite (a
 * non-finite value anywhere propagates into it), else HV_ERR_DRIFT if the
 * mass drift bound was crossed after some long step since hv_state_init
 * (the outputs are written in both cases).  Synchronises the stream. */
int hv_mass(hv_grid_t g, double *mass_out, double *energy_out);

/* For callers that cannot allocate device memory or block (code between
 * kernels of a tight serving loop, work a caller records into a HIP graph):
 * the sums of hv_mass, enqueued on the grid's stream without any allocation
 * or synchronisation.  Writes dev_out[0] = total mass and dev_out[1] =
 * total energy of the current state (the same float64 values, in the same
 * fixed order, that hv_mass returns); dev_out is caller-owned device memory
 * of 2 doubles, written when the stream reaches the sums.  The partial sums
 * live in a library-owned static device array of 1024 doubles per device
 * (looked up at hv_grid_create, with the grid's device current); a grid whose
 * sums need more partials is rejected with HV_ERR_ARG (none can: the
 * partial count is capped at 1024).  The array is shared by every grid on a
 * device and keeps the last call's partials: calls that overlap in time on
 * one device (different streams or threads) race; calls on one stream are
 * ordered.  HV_ERR_STATE before hv_state_init.  Does not check the mass for
 * finiteness (read dev_out). */
int hv_mass_noalloc(hv_grid_t g, double *dev_out);

/* Kernel timing with HIP events on the grid's stream, a measurement aid.
 * hv_trace(g, 1) zeroes the totals and records an event pair around every
 * kernel launch that follows; hv_trace(g, 0) stops recording.
 * hv_trace_read synchronises the stream, folds the recorded pairs into
 * per-kind totals and returns the total milliseconds and launch count of
 * one kind (a "launch" of HV_K_MASS is its two-kernel reduction).  Either
 * output pointer may be NULL. */
enum { HV_K_SLOW_PREP = 0, HV_K_SLOW_FLUX = 1, HV_K_SHORT_STEP = 2, HV_K_MASS = 3, HV_K_COUNT = 4 };
int hv_trace(hv_grid_t g, int32_t on);
int hv_trace_read(hv_grid_t g, int32_t kind, double *ms_total, int64_t *launches);

/* Autotune: time each kernel kind (slow prep, slow flux, short step) of the
 * loaded state with every launch configuration and keep the fastest (the
 * paper's central block-size configuration, Sect. 2.3, made a measurement).
 * A configuration is a tile shape (16x1, 8x2, 4x4 columns per block), a
 * block order -- launch order, or XCD-chunked (in every group of 64
 * consecutive tiles each of the 8 XCDs runs 8 consecutive tiles, so that
 * x-neighbours share its L2; tiles past the last whole group keep launch
 * order) -- and the lanes per column (columns per wavefront).  Column-fastest
 * layout: the default width (32 for float64 storage with 64 levels, else 16)
 * or the other one (8 lanes for 32 levels, 32 for 64 levels in float32 /
 * mixed, 16 for 64 levels in float64, 32 for 128 levels).  i-fastest
 * layout: one lane per column or the default segments.  Configuration index
 * c = shape + 3 * chunked + 6 * other_width, 0..11 (shape 0..2 for 16x1,
 * 8x2, 4x4); the damped short step keeps the default.  The column-fastest
 * slow flux has 12 more, c + 12: the same with each segment walking a run of
 * 32 columns along x, carrying the flux through the face it shares with the
 * next column, in blocks of 1x16, 2x8 or 4x4 runs (shape 0..2; runs along x
 * by rows).
 * Tile shape, block order and runs do not change any
 * result; neither does the mapping of the slow sweeps; the short step's
 * mapping sets how its column solve splits into in-lane elimination and
 * cyclic reduction (or a serial sweep), which changes its rounding
 * (float64: about 1e-15 relative).  The choice is appended to
 * a plain-text cache ($HV_TUNE_CACHE, else $HOME/.cache/hevi/tune.txt; one
 * line "key c_prep c_flux c_short"; the last line of a key wins, and
 * hv_tune rewrites the file with one line per key) that later grids of the
 * same kind read at creation.  tile_x_out and lanes_out (either may be
 * NULL) receive, per kind, the chosen tile x-extent (negated for the
 * XCD-chunked order) and lanes per column.  Synchronises the stream; does
 * not change the state.
 * (Addressing: the slow-flux kernel reaches the arrays of a launch group by
 * 32-bit byte offsets when every member's arrays are under 4 GiB, else by
 * 64-bit addresses; HV_ADDR64=1 in the environment at creation forces the
 * 64-bit form.  Both give bitwise-identical results.) */
int hv_tune(hv_grid_t g, int32_t *tile_x_out, int32_t *lanes_out);

/* Set the launch configuration of each kernel kind (config[3], indices as
 * hv_tune numbers them: 0..11, and 0..23 for the column-fastest slow flux;
 * else HV_ERR_ARG) without timing, e.g. to pin a tuned
 * choice; config NULL changes nothing.  config_out, tile_x_out and lanes_out
 * (3 entries each, any may be NULL) receive the configuration in force: its
 * indices, and the tile x-extents and lanes per column as from hv_tune.
 * Synchronises the stream. */
int hv_configure(hv_grid_t g, const int32_t config[3], int32_t *config_out, int32_t *tile_x_out,
                 int32_t *lanes_out);

/* Lateral and upper damping, the relaxation kernel of the paper's Listing 1
 * (Sect. 2.1), applied after every short step.  The target of each prognostic
 * is the boundary state interpolated in time,
 *   X_target = mtratio (ref + bnd1) + tratio (ref + bnd2) - ref,
 * tratio = (t - t1)/(t2 - t1) clipped to [0, 1], mtratio = 1 - tratio, ref the
 * reference rho or rho*theta for HV_RHO_PTB / HV_RHOTHETA_PTB and 0 for the
 * momenta, t the model time at the end of the short step.  Each value then
 * relaxes implicitly, X <- (X + c X_target)/(1 + c), c = dtau (nu_lat of its
 * column + nu_top of its level; W's level face k uses level k); values with
 * rate 0 and W on the lids are left untouched.  The relaxation runs inside
 * the short-step kernel on the new values before they are stored (in the
 * Runge-Kutta form after the second stage), so it reads only the two
 * boundary states of the damped values.
 * Arguments: nu_lat nx*ny rates (1/s, >= 0, i fastest), nu_top nz rates;
 * bnd1[f], bnd2[f] boundary states in the layout of hv_state_init's fields
 * (W with zero lids); t1 < t2; time_now = model time of the current state
 * (it advances by dt per long step; hv_state_init resets it to 0).  Host
 * arrays are copied (converted to the grid's precision and layout) into the
 * workspace, which must have been sized with desc.damping = 1, else
 * HV_ERR_ARG.  Replaces earlier damping data; synchronises the stream. */
int hv_damping(hv_grid_t g, const double *nu_lat, const double *nu_top,
               const double *const bnd1[5], const double *const bnd2[5], double t1, double t2,
               double time_now);

/* Release the handle (never the caller's workspace).  NULL is a no-op. */
void hv_grid_destroy(hv_grid_t g);

/* Text of the last failure on this handle (or, for NULL, of the last
 * failure that had no valid handle).  Never NULL; valid until the next call
 * on the same handle. */
const char *hv_last_error(hv_grid_t g);

/* ---------------------------------------------------------------------------
 * Batched ensemble: n independent domains of uneven sizes advanced together.
 * Every member has its own description (same precision and layout for all),
 * state, reference columns and long-step length; all members take the same
 * n_short.  One long step of the whole ensemble is one launch per phase
 * (slow sweep, each short step, the mass sum) covering the tiles of every
 * member, recorded once as a hipGraph and replayed.  Workspace, stream and
 * error conventions are those of the single grid above; member indices are
 * 0..n-1 in the order of descs.
 * ------------------------------------------------------------------------- */
size_t hv_ens_workspace_bytes(int32_t n, const hv_grid_desc *descs);
int hv_ens_create(int32_t n, const hv_grid_desc *descs, void *dev_workspace, size_t bytes,
                  void *hip_stream, hv_ens_t *out);
int hv_ens_state_init(hv_ens_t e, int32_t member, const double *const fields[5],
                      const double *rho_ref, const double *rhotheta_ref, const double *p_ref);
/* dt_per_member: n long-step lengths (s). */
int hv_ens_step(hv_ens_t e, const double *dt_per_member, int32_t n_long, int32_t n_short);
int hv_ens_state_read(hv_ens_t e, int32_t member, int32_t field, double *host_out);
int hv_ens_mass(hv_ens_t e, int32_t member, double *mass_out, double *energy_out);
/* As hv_tune, per launch group: members with equal nz and terrain flag,
 * flat groups first, each kind in increasing nz;
 * tile_x_out and lanes_out receive 3 entries per group (room for 18: at
 * most 6 groups), *ngroups_out the group count (any may be NULL). */
int hv_ens_tune(hv_ens_t e, int32_t *tile_x_out, int32_t *lanes_out, int32_t *ngroups_out);
/* As hv_configure, setting launch group `group`; the outputs cover every
 * group (3 entries per group, room for 18), *ngroups_out the group count. */
int hv_ens_configure(hv_ens_t e, int32_t group, const int32_t config[3], int32_t *config_out,
                     int32_t *tile_x_out, int32_t *lanes_out, int32_t *ngroups_out);
int hv_ens_damping(hv_ens_t e, int32_t member, const double *nu_lat, const double *nu_top,
                   const double *const bnd1[5], const double *const bnd2[5], double t1, double t2,
                   double time_now);
int hv_ens_trace(hv_ens_t e, int32_t on);
int hv_ens_trace_read(hv_ens_t e, int32_t kind, double *ms_total, int64_t *launches);
void hv_ens_destroy(hv_ens_t e);
const char *hv_ens_last_error(hv_ens_t e);

/* ---------------------------------------------------------------------------
 * Seven-point diffusion step: the stencil whose memory traffic dominates the
 * paper's reduced weather application and its no-cache / perfect-cache
 * bandwidth model (Sect. 4).  One explicit step on a uniform grid,
 *   out = q + ((kx lx + ky ly) + kz lz),  l_d = (q_{-d} + q_{+d}) - 2 q,
 * kd = nu dt / d^2, periodic in x and y, no flux through the lids (the
 * missing vertical neighbour is the cell itself).
 * dev_in, dev_out: device arrays of nx*ny*nz values of the precision's type
 * (HV_FP64: double, HV_FP32: float; HV_MIXED is HV_ERR_ARG) in `layout`
 * (HV_KIJ: k + nz*(i + nx*j); HV_IJK: i + nx*(j + ny*k)), 64-byte aligned,
 * distinct; owned by the caller.  nz in {32, 64, 128}.  tile_x: 16, 8 or 4
 * columns along x per 256-thread block.  Enqueued on hip_stream (NULL = the
 * default stream); asynchronous.  Invalid arguments return HV_ERR_ARG before
 * any launch (text in hv_last_error(NULL)). */
int hv_diffuse(int32_t nx, int32_t ny, int32_t nz, int32_t precision, int32_t layout, double kx,
               double ky, double kz, int32_t tile_x, const void *dev_in, void *dev_out,
               void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HEVI_H */
