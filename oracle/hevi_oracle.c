/*
 * hevi_oracle.c -- plain, slow FP64 CPU oracle of the HEVI dynamical-core step.
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
 * this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant with the
 * GPU library, and it includes nothing but the C library.
 *
 * What the paper fixes (Sect. 1.1, "ASUCA on GPU"): a finite-volume spatial
 * discretisation on a rectangular grid; a third-order Runge-Kutta long step
 * after Wicker & Skamarock (2002); sound and gravity waves integrated on a
 * finer time step with a horizontally-explicit / vertically-implicit (HEVI)
 * scheme; parallelism over the horizontal I/J indices with K sequential; and,
 * from its Listing 1, prognostic density stored as a perturbation on a
 * reference state.  The paper prints no equations for any of this, so every
 * formula below is a stated reading of that outline:
 *
 *  - Arakawa-C staggering: rho', Theta' (= rho*theta perturbation) at cell
 *    centres, U = rho*u on west x-faces, V = rho*v on south y-faces,
 *    W = rho*w on the nz+1 level faces with W = 0 on both rigid lids.
 *  - Slow tendencies (frozen over a stage): flux-form momentum advection with
 *    Koren-limited face values (kappa = 1/3) of u, v, w, and the residual
 *    -div(mass flux * (limited - centred) face theta).
 *  - Stage linearisation: p' = p_ref * expm1(gamma * log1p(Theta'/Theta_ref)),
 *    C = gamma p / Theta, P0 = p' - C Theta', so that p' ~ P0 + C Theta'.
 *  - Short step: forward horizontal momentum (pressure gradient of the
 *    current p'), then horizontal mass and theta-weighted Theta divergences,
 *    then a beta-off-centred trapezoidal vertical coupling of W, rho', Theta'
 *    that is one tridiagonal system per column, solved by the Thomas
 *    algorithm (no pivoting; the system is diagonally dominant).
 *  - Short-step integrator, optional second form: the paper calls the short
 *    steps a second-order Runge-Kutta scheme.  With Phi(X_b, X_e, d) the
 *    short step above whose increments are added to X_b while every explicit
 *    term and the (1 - beta) old-time part of the vertical coupling are taken
 *    from X_e, the two-stage form is X* = Phi(X, X, dtau/2) and
 *    X+ = Phi(X, X*, dtau) (midpoint rule; the forward-backward step is
 *    Phi(X, X, dtau)).  Two column solves per short step.
 *  - Lateral and upper damping (optional), the kernel of the paper's
 *    Listing 1: the target of each prognostic is the boundary state
 *    interpolated in time, mtratio (ref + bnd1) + tratio (ref + bnd2) - ref
 *    (ref = 0 for the momenta), tratio = (t - t1)/(t2 - t1) clipped to
 *    [0, 1], mtratio = 1 - tratio; after every short step each value
 *    relaxes implicitly, X <- (X + c X_target) / (1 + c), c = dtau (nu_lat of
 *    its column + nu_top of its level), with t the time at the end of that
 *    short step.  Values with nu = 0, and W on the lids, are left untouched.
 *  - RK3 stage lengths dt/3, dt/2, dt; each stage restarts its n short steps
 *    from the state at the start of the long step, with the slow tendencies
 *    evaluated on the previous stage's result.
 *  - EOS p = P00 (R Theta / P00)^gamma; gamma = 1.4, g = 9.80665 (SI).
 *  - Terrain (optional): terrain-following height z = zeta + h (1 - zeta/H)
 *    (Gal-Chen & Somerville 1975).  J = 1 - h/H per column; horizontal mass
 *    fluxes carry J (two-point means on faces), and the momentum control
 *    volumes take means of those cell-face mass fluxes; the flux through zeta
 *    surfaces is Omega = W - (1 - zeta/H) * (slope-weighted U and V, averaged
 *    to the level face), zero on both lids; divergences are divided by J;
 *    the horizontal pressure gradient gains + (z_x/J) * (mean of d p'/d zeta
 *    of the two columns; one-sided at the lowest and highest cells); in the
 *    vertical part dz becomes J dz and W* becomes Omega* = beta W+ +
 *    (1 - beta) W - E, with E the slope term of Omega evaluated with the new
 *    horizontal momentum.  The reference state is then given at every cell's true height.
 *    W is held at 0 on both lids (the lower boundary condition is Omega = 0).
 *
 * Pins (tests that hold this file to something other than itself): the
 * Koren limiter table and its smooth-regime closed form; the exact
 * one-cell shift of donor-cell advection at Courant number 1; conservation
 * of mass under periodic/lid boundaries; the rest state and horizontally
 * uniform flow staying bitwise steady; preservation of a uniform theta
 * field; discrete hydrostatic balance staying at rest; the Thomas solve
 * against a dense LU; the assembled tridiagonal against the brute-force
 * Jacobian of the vertical update equations; the horizontal and vertical
 * acoustic modes against their closed-form amplification matrices; the
 * gravity and acoustic modes of an isothermal atmosphere against their
 * dispersion relation; closed forms of single stencil terms (a uniform
 * specific velocity over a varying density, a potential temperature linear
 * in height on stretched levels); and conservation of the total rho*theta.
 * or_energy() (a diagnostic): the closed-form energy of the isothermal rest
 * state, flat and over terrain, and the kinetic increment of a uniform flow.
 *
 * Layout: canonical i-fastest, index i + nx*(j + ny*k); the vertical
 * momentum has nz+1 levels.  OpenMP parallelises over independent cells or
 * columns only, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_GAMMA 1.4

enum { OR_OK = 0, OR_EARG = -1, OR_ENOMEM = -2, OR_ENOTDOM = -3 };
enum { OR_LIM_NONE = 0, OR_LIM_KOREN = 1 };

typedef struct {
    int32_t nx, ny, nz;
    int32_t donor_cell;       /* 0: Koren-limited advection (the model);
                                 1: donor cell, a linear operator used only to
                                 hold the RK3 stage structure to its closed form */
    double dx, dy;
    double beta;              /* off-centring of the vertical coupling       */
    double grav;              /* gravitational acceleration                   */
    const double *zf;         /* nz+1 level-face heights, zf[0] = 0           */
    const double *rho_ref;    /* reference density at cell centres: nz values,
                                 or nx*ny*nz with terrain                     */
    const double *rt_ref;     /* reference rho*theta, same shape              */
    const double *p_ref;      /* reference pressure, same shape               */
    const double *terrain;    /* nx*ny surface heights, NULL = flat           */
    int32_t short_rk2;        /* 0: forward-backward short step; 1: the
                                 two-stage Runge-Kutta short step           */
    /* lateral and upper damping after every short step (nu_lat NULL: off) */
    const double *nu_lat;     /* nx*ny lateral rate (1/s) per column         */
    const double *nu_top;     /* nz    upper rate (1/s) per level            */
    const double *bnd1[5];    /* boundary states at times t1 and t2, in the  */
    const double *bnd2[5];    /* layout of the prognostic fields             */
    double t1, t2;            /* times of bnd1 and bnd2, t2 > t1             */
    double time0;             /* model time at the start of or_step          */
} or_grid;

/* index of the reference value of cell c (level k) */
static inline size_t RI(const or_grid *g, size_t c, int k) { return g->terrain ? c : (size_t)k; }

/* horizontal geometry: Jacobians and terrain slopes (flat: 1 and 0) */
typedef struct {
    double *J;    /* nx*ny  J = 1 - h/H of column (i, j)                      */
    double *Ju;   /* nx*ny  J on the west x-face of column (i, j)             */
    double *Jv;   /* nx*ny  J on the south y-face                             */
    double *su;   /* nx*ny  dh/dx on the west x-face                          */
    double *sv;   /* nx*ny  dh/dy on the south y-face                         */
    double *dc;   /* nz     1 - zeta/H at cell centres                        */
    double *df;   /* nz+1   1 - zeta/H at level faces                         */
} or_geo;

/* vertical metrics derived from the face heights */
typedef struct {
    double *dz;   /* nz   cell thickness                                        */
    double *dzf;  /* nz+1 centre-to-centre distance at face k (1..nz-1)         */
    double *a;    /* nz+1 weight of the cell above face k in a linear interp.   */
    double *b;    /* nz+1 weight of the cell below face k                       */
} or_vmet;

static int vmet_init(const or_grid *g, or_vmet *m)
{
    int nz = g->nz;
    m->dz = (double *)calloc((size_t)nz, sizeof(double));
    m->dzf = (double *)calloc((size_t)nz + 1, sizeof(double));
    m->a = (double *)calloc((size_t)nz + 1, sizeof(double));
    m->b = (double *)calloc((size_t)nz + 1, sizeof(double));
    if (!m->dz || !m->dzf || !m->a || !m->b) return OR_ENOMEM;
    for (int k = 0; k < nz; ++k) m->dz[k] = g->zf[k + 1] - g->zf[k];
    for (int k = 1; k < nz; ++k) {
        /* distance between the centres of cells k-1 and k */
        m->dzf[k] = 0.5 * (g->zf[k + 1] + g->zf[k]) - 0.5 * (g->zf[k] + g->zf[k - 1]);
        /* linear interpolation in z from the centres to face k */
        m->a[k] = m->dz[k - 1] / (m->dz[k - 1] + m->dz[k]);
        m->b[k] = m->dz[k] / (m->dz[k - 1] + m->dz[k]);
    }
    return OR_OK;
}

static void vmet_free(or_vmet *m)
{
    free(m->dz); free(m->dzf); free(m->a); free(m->b);
}

static inline int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

static inline int clampi(int i, int lo, int hi)
{
    return i < lo ? lo : (i > hi ? hi : i);
}

static void geo_free(or_geo *q)
{
    free(q->J); free(q->Ju); free(q->Jv); free(q->su); free(q->sv); free(q->dc); free(q->df);
}

static int geo_init(const or_grid *g, or_geo *q)
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t nxy = (size_t)nx * ny;
    const double H = g->zf[nz];
    q->J = (double *)malloc(nxy * sizeof(double));
    q->Ju = (double *)malloc(nxy * sizeof(double));
    q->Jv = (double *)malloc(nxy * sizeof(double));
    q->su = (double *)malloc(nxy * sizeof(double));
    q->sv = (double *)malloc(nxy * sizeof(double));
    q->dc = (double *)malloc((size_t)nz * sizeof(double));
    q->df = (double *)malloc(((size_t)nz + 1) * sizeof(double));
    if (!q->J || !q->Ju || !q->Jv || !q->su || !q->sv || !q->dc || !q->df) return OR_ENOMEM;
    for (int k = 0; k < nz; ++k) q->dc[k] = 1.0 - 0.5 * (g->zf[k] + g->zf[k + 1]) / H;
    for (int k = 0; k <= nz; ++k) q->df[k] = 1.0 - g->zf[k] / H;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            if (!g->terrain) {
                q->J[c] = q->Ju[c] = q->Jv[c] = 1.0;
                q->su[c] = q->sv[c] = 0.0;
                continue;
            }
            const double h = g->terrain[c];
            const double hw = g->terrain[(size_t)j * nx + wrapi(i - 1, nx)];
            const double hs = g->terrain[(size_t)wrapi(j - 1, ny) * nx + i];
            q->J[c] = 1.0 - h / H;
            q->Ju[c] = 0.5 * ((1.0 - hw / H) + (1.0 - h / H));
            q->Jv[c] = 0.5 * ((1.0 - hs / H) + (1.0 - h / H));
            q->su[c] = (h - hw) / g->dx;
            q->sv[c] = (h - hs) / g->dy;
        }
    return OR_OK;
}


/* ------------------------------------------------------------------------
 * Koren limiter.  With D- = q_L - q_LL (upwind difference) and
 * D+ = q_R - q_L (downwind difference), the limited increment is
 * psi(D+/D-) * D- with psi(r) = max(0, min(2r, (1+2r)/3, 2)) (Koren 1993,
 * kappa = 1/3), written without the division.
 * ---------------------------------------------------------------------- */
double or_koren_phi(double dm, double dp)
{
    if (dm > 0.0) return fmax(0.0, fmin(fmin(2.0 * dp, (dm + 2.0 * dp) / 3.0), 2.0 * dm));
    if (dm < 0.0) return fmin(0.0, fmax(fmax(2.0 * dp, (dm + 2.0 * dp) / 3.0), 2.0 * dm));
    return 0.0;
}

/* Face value between L and R for mass flux m; m >= 0 counts as flow from L.
 * Limiter NONE is the donor-cell (first-order upwind) value. */
double or_face(double qLL, double qL, double qR, double qRR, double m, int lim)
{
    if (m >= 0.0) {
        if (lim == OR_LIM_NONE) return qL;
        return qL + 0.5 * or_koren_phi(qL - qLL, qR - qL);
    }
    if (lim == OR_LIM_NONE) return qR;
    return qR + 0.5 * or_koren_phi(qR - qRR, qL - qR);
}

#define C3(i, j, k) ((size_t)(k) * nxy + (size_t)(j) * (size_t)nx + (size_t)(i))

/* ------------------------------------------------------------------------
 * One forward-Euler flux-form step of a passive scalar of unit density:
 *   q+ = q - dt * [ dx(u qf) + dy(v qf) + dz(w qf) ]
 * u, v on west/south faces (nx*ny*nz), w on level faces (nx*ny*(nz+1)) with
 * w = 0 on the lids.  Face values use or_face with the given limiter and the
 * same zero-gradient vertical ghosts as the model step.
 * ---------------------------------------------------------------------- */
int or_advect_fe(const or_grid *g, const double *q, const double *u, const double *v,
                 const double *w, double dt, int lim, double *out)
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t nxy = (size_t)nx * ny;
    or_vmet vm;
    if (vmet_init(g, &vm) != OR_OK) { vmet_free(&vm); return OR_ENOMEM; }
#pragma omp parallel for schedule(static)
    for (int jk = 0; jk < ny * nz; ++jk) {
        int j = jk % ny, k = jk / ny;
        for (int i = 0; i < nx; ++i) {
            double fx[2], fy[2], fz[2];
            for (int s = 0; s < 2; ++s) {
                int f = i + s;                        /* x-face between f-1 and f */
                double m = u[C3(wrapi(f, nx), j, k)];
                fx[s] = m * or_face(q[C3(wrapi(f - 2, nx), j, k)], q[C3(wrapi(f - 1, nx), j, k)],
                                    q[C3(wrapi(f, nx), j, k)], q[C3(wrapi(f + 1, nx), j, k)], m, lim);
                int h = j + s;
                m = v[C3(i, wrapi(h, ny), k)];
                fy[s] = m * or_face(q[C3(i, wrapi(h - 2, ny), k)], q[C3(i, wrapi(h - 1, ny), k)],
                                    q[C3(i, wrapi(h, ny), k)], q[C3(i, wrapi(h + 1, ny), k)], m, lim);
                int kk = k + s;                       /* level face */
                if (kk == 0 || kk == nz) {
                    fz[s] = 0.0;
                } else {
                    m = w[C3(i, j, kk)];
                    fz[s] = m * or_face(q[C3(i, j, clampi(kk - 2, 0, nz - 1))], q[C3(i, j, kk - 1)],
                                        q[C3(i, j, kk)], q[C3(i, j, clampi(kk + 1, 0, nz - 1))], m, lim);
                }
            }
            double div = (fx[1] - fx[0]) / g->dx + (fy[1] - fy[0]) / g->dy + (fz[1] - fz[0]) / vm.dz[k];
            out[C3(i, j, k)] = q[C3(i, j, k)] - dt * div;
        }
    }
    vmet_free(&vm);
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Slow sweep, evaluated once per RK3 stage on the stage-input state st =
 * {rho', U, V, W, Theta'}.  Outputs out = {S_U, S_V, S_W, R_Theta, theta_s,
 * P0_s, C_s}.
 *
 * Momentum: S_U = -[dx(mx qx) + dy(my qy) + dz(mz qz)] over the U control
 * volume; mass fluxes are two-point means of U, V, W onto its faces (cell
 * centres, xy-corners, xz-edges); q is the Koren face value of u = U/rho_u
 * (rho_u the two-point mean of full density).  Same for V; for W the
 * control volume spans the centres of cells k-1 and k and w = W/rho_w with
 * rho_w linearly interpolated in z.  Vertical fluxes on the lids are zero and
 * vertical ghost values are zero-gradient copies (w ghosts copy the lid 0).
 *
 * Theta: R_Theta = -div( mass flux * (limited face theta - centred face
 * theta) ), centred = two-point mean horizontally, linear in z vertically.
 *
 * Stage coefficients: p'_s from the EOS ratio form, C_s = gamma p / Theta,
 * P0_s = p'_s - C_s Theta', theta_s = Theta / rho.
 * ---------------------------------------------------------------------- */
int or_slow_sweep(const or_grid *g, const double *const st[5], double *const out[7])
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t nxy = (size_t)nx * ny, n = nxy * nz, nw = nxy * (nz + 1);
    const double *rp = st[0], *U = st[1], *V = st[2], *W = st[3], *tp = st[4];
    or_vmet vm;
    or_geo geo;
    memset(&geo, 0, sizeof geo);
    if (vmet_init(g, &vm) != OR_OK || geo_init(g, &geo) != OR_OK) {
        vmet_free(&vm); geo_free(&geo);
        return OR_ENOMEM;
    }
    double *rho = (double *)malloc(n * sizeof(double));
    double *th = (double *)malloc(n * sizeof(double));
    double *uu = (double *)malloc(n * sizeof(double));
    double *vv = (double *)malloc(n * sizeof(double));
    double *ww = (double *)malloc(nw * sizeof(double));
    double *om = (double *)malloc(nw * sizeof(double));
    if (!rho || !th || !uu || !vv || !ww || !om) {
        free(rho); free(th); free(uu); free(vv); free(ww); free(om); vmet_free(&vm); geo_free(&geo);
        return OR_ENOMEM;
    }
#define C2(i, j) ((size_t)(j) * (size_t)nx + (size_t)(i))
    /* full density, theta, and the advected specific velocities */
#pragma omp parallel for schedule(static)
    for (int jk = 0; jk < ny * nz; ++jk) {
        int j = jk % ny, k = jk / ny;
        for (int i = 0; i < nx; ++i) {
            size_t c = C3(i, j, k);
            rho[c] = g->rho_ref[RI(g, c, k)] + rp[c];
            th[c] = (g->rt_ref[RI(g, c, k)] + tp[c]) / rho[c];
        }
    }
#pragma omp parallel for schedule(static)
    for (int jk = 0; jk < ny * nz; ++jk) {
        int j = jk % ny, k = jk / ny;
        for (int i = 0; i < nx; ++i) {
            size_t c = C3(i, j, k);
            uu[c] = U[c] / (0.5 * (rho[C3(wrapi(i - 1, nx), j, k)] + rho[c]));
            vv[c] = V[c] / (0.5 * (rho[C3(i, wrapi(j - 1, ny), k)] + rho[c]));
        }
    }
    /* w on level faces, and the mass flux through the zeta surfaces:
     * Omega = W - (1 - zeta/H) * (slope-weighted U and V at the face), with
     * the slope-weighted momenta averaged to the column centre and then
     * interpolated linearly in z to the face; Omega = 0 on both lids. */
#pragma omp parallel for schedule(static)
    for (int jk = 0; jk < ny * (nz + 1); ++jk) {
        int j = jk % ny, k = jk / ny;
        for (int i = 0; i < nx; ++i) {
            size_t c = C3(i, j, k);
            if (k == 0 || k == nz) {
                ww[c] = 0.0;
                om[c] = 0.0;
                continue;
            }
            ww[c] = W[c] / (vm.a[k] * rho[C3(i, j, k)] + vm.b[k] * rho[C3(i, j, k - 1)]);
            const double su0 = geo.su[C2(i, j)], su1 = geo.su[C2(wrapi(i + 1, nx), j)];
            const double sv0 = geo.sv[C2(i, j)], sv1 = geo.sv[C2(i, wrapi(j + 1, ny))];
            const double mxk = 0.5 * (su0 * U[C3(i, j, k)] + su1 * U[C3(wrapi(i + 1, nx), j, k)]);
            const double mxm = 0.5 * (su0 * U[C3(i, j, k - 1)] + su1 * U[C3(wrapi(i + 1, nx), j, k - 1)]);
            const double myk = 0.5 * (sv0 * V[C3(i, j, k)] + sv1 * V[C3(i, wrapi(j + 1, ny), k)]);
            const double mym = 0.5 * (sv0 * V[C3(i, j, k - 1)] + sv1 * V[C3(i, wrapi(j + 1, ny), k - 1)]);
            om[c] = W[c] - geo.df[k] * ((vm.a[k] * mxk + vm.b[k] * mxm) + (vm.a[k] * myk + vm.b[k] * mym));
        }
    }

    double *SU = out[0], *SV = out[1], *SW = out[2], *RT = out[3];
    double *ths = out[4], *P0 = out[5], *Cs = out[6];
    const double dx = g->dx, dy = g->dy;
    const int LIM = g->donor_cell ? OR_LIM_NONE : OR_LIM_KOREN;

    /* S_U, S_V, R_Theta and the stage coefficients at cell level k */
#pragma omp parallel for schedule(static)
    for (int jk = 0; jk < ny * nz; ++jk) {
        int j = jk % ny, k = jk / ny;
        for (int i = 0; i < nx; ++i) {
            size_t c = C3(i, j, k);
            /* ---- x-momentum at the west face of cell i ---- */
            double fx[2], fy[2], fz[2];
            for (int s = 0; s < 2; ++s) {
                int cc = i - 1 + s;                   /* centre of cell cc */
                double m = 0.5 * (geo.Ju[C2(wrapi(cc, nx), j)] * U[C3(wrapi(cc, nx), j, k)] +
                                  geo.Ju[C2(wrapi(cc + 1, nx), j)] * U[C3(wrapi(cc + 1, nx), j, k)]);
                fx[s] = m * or_face(uu[C3(wrapi(cc - 1, nx), j, k)], uu[C3(wrapi(cc, nx), j, k)],
                                    uu[C3(wrapi(cc + 1, nx), j, k)], uu[C3(wrapi(cc + 2, nx), j, k)],
                                    m, LIM);
                int jf = j + s;                       /* corner (face i, face jf) */
                m = 0.5 * (geo.Jv[C2(wrapi(i - 1, nx), wrapi(jf, ny))] * V[C3(wrapi(i - 1, nx), wrapi(jf, ny), k)] +
                           geo.Jv[C2(i, wrapi(jf, ny))] * V[C3(i, wrapi(jf, ny), k)]);
                fy[s] = m * or_face(uu[C3(i, wrapi(jf - 2, ny), k)], uu[C3(i, wrapi(jf - 1, ny), k)],
                                    uu[C3(i, wrapi(jf, ny), k)], uu[C3(i, wrapi(jf + 1, ny), k)],
                                    m, LIM);
                int kf = k + s;                       /* edge (face i, level face kf) */
                if (kf == 0 || kf == nz) {
                    fz[s] = 0.0;
                } else {
                    m = 0.5 * (om[C3(wrapi(i - 1, nx), j, kf)] + om[C3(i, j, kf)]);
                    fz[s] = m * or_face(uu[C3(i, j, clampi(kf - 2, 0, nz - 1))], uu[C3(i, j, kf - 1)],
                                        uu[C3(i, j, kf)], uu[C3(i, j, clampi(kf + 1, 0, nz - 1))],
                                        m, LIM);
                }
            }
            SU[c] = -((fx[1] - fx[0]) / dx + (fy[1] - fy[0]) / dy + (fz[1] - fz[0]) / vm.dz[k]) /
                    geo.Ju[C2(i, j)];

            /* ---- y-momentum at the south face of cell j ---- */
            for (int s = 0; s < 2; ++s) {
                int iff = i + s;                      /* corner (face iff, face j) */
                double m = 0.5 * (geo.Ju[C2(wrapi(iff, nx), wrapi(j - 1, ny))] * U[C3(wrapi(iff, nx), wrapi(j - 1, ny), k)] +
                                  geo.Ju[C2(wrapi(iff, nx), j)] * U[C3(wrapi(iff, nx), j, k)]);
                fx[s] = m * or_face(vv[C3(wrapi(iff - 2, nx), j, k)], vv[C3(wrapi(iff - 1, nx), j, k)],
                                    vv[C3(wrapi(iff, nx), j, k)], vv[C3(wrapi(iff + 1, nx), j, k)],
                                    m, LIM);
                int cc = j - 1 + s;                   /* centre of cell cc */
                m = 0.5 * (geo.Jv[C2(i, wrapi(cc, ny))] * V[C3(i, wrapi(cc, ny), k)] +
                           geo.Jv[C2(i, wrapi(cc + 1, ny))] * V[C3(i, wrapi(cc + 1, ny), k)]);
                fy[s] = m * or_face(vv[C3(i, wrapi(cc - 1, ny), k)], vv[C3(i, wrapi(cc, ny), k)],
                                    vv[C3(i, wrapi(cc + 1, ny), k)], vv[C3(i, wrapi(cc + 2, ny), k)],
                                    m, LIM);
                int kf = k + s;
                if (kf == 0 || kf == nz) {
                    fz[s] = 0.0;
                } else {
                    m = 0.5 * (om[C3(i, wrapi(j - 1, ny), kf)] + om[C3(i, j, kf)]);
                    fz[s] = m * or_face(vv[C3(i, j, clampi(kf - 2, 0, nz - 1))], vv[C3(i, j, kf - 1)],
                                        vv[C3(i, j, kf)], vv[C3(i, j, clampi(kf + 1, 0, nz - 1))],
                                        m, LIM);
                }
            }
            SV[c] = -((fx[1] - fx[0]) / dx + (fy[1] - fy[0]) / dy + (fz[1] - fz[0]) / vm.dz[k]) /
                    geo.Jv[C2(i, j)];

            /* ---- Theta residual: limited minus centred face theta ---- */
            for (int s = 0; s < 2; ++s) {
                int f = i + s;
                double m = geo.Ju[C2(wrapi(f, nx), j)] * U[C3(wrapi(f, nx), j, k)];
                double tl = or_face(th[C3(wrapi(f - 2, nx), j, k)], th[C3(wrapi(f - 1, nx), j, k)],
                                    th[C3(wrapi(f, nx), j, k)], th[C3(wrapi(f + 1, nx), j, k)],
                                    m, LIM);
                double tcen = 0.5 * (th[C3(wrapi(f - 1, nx), j, k)] + th[C3(wrapi(f, nx), j, k)]);
                fx[s] = m * (tl - tcen);
                int h = j + s;
                m = geo.Jv[C2(i, wrapi(h, ny))] * V[C3(i, wrapi(h, ny), k)];
                tl = or_face(th[C3(i, wrapi(h - 2, ny), k)], th[C3(i, wrapi(h - 1, ny), k)],
                             th[C3(i, wrapi(h, ny), k)], th[C3(i, wrapi(h + 1, ny), k)], m, LIM);
                tcen = 0.5 * (th[C3(i, wrapi(h - 1, ny), k)] + th[C3(i, wrapi(h, ny), k)]);
                fy[s] = m * (tl - tcen);
                int kf = k + s;
                if (kf == 0 || kf == nz) {
                    fz[s] = 0.0;
                } else {
                    m = om[C3(i, j, kf)];
                    tl = or_face(th[C3(i, j, clampi(kf - 2, 0, nz - 1))], th[C3(i, j, kf - 1)],
                                 th[C3(i, j, kf)], th[C3(i, j, clampi(kf + 1, 0, nz - 1))], m, LIM);
                    tcen = vm.a[kf] * th[C3(i, j, kf)] + vm.b[kf] * th[C3(i, j, kf - 1)];
                    fz[s] = m * (tl - tcen);
                }
            }
            RT[c] = -((fx[1] - fx[0]) / dx + (fy[1] - fy[0]) / dy + (fz[1] - fz[0]) / vm.dz[k]) /
                    geo.J[C2(i, j)];

            /* ---- stage coefficients ---- */
            const size_t r = RI(g, c, k);
            double pps = g->p_ref[r] * expm1(OR_GAMMA * log1p(tp[c] / g->rt_ref[r]));
            double cs = OR_GAMMA * (g->p_ref[r] + pps) / (g->rt_ref[r] + tp[c]);
            ths[c] = th[c];
            Cs[c] = cs;
            P0[c] = pps - cs * tp[c];
        }
    }

    /* S_W on the level faces; zero on the lids */
#pragma omp parallel for schedule(static)
    for (int jk = 0; jk < ny * (nz + 1); ++jk) {
        int j = jk % ny, k = jk / ny;
        for (int i = 0; i < nx; ++i) {
            size_t c = C3(i, j, k);
            if (k == 0 || k == nz) { SW[c] = 0.0; continue; }
            double fx[2], fy[2], fz[2];
            for (int s = 0; s < 2; ++s) {
                int iff = i + s;                      /* edge (x-face iff, level face k) */
                double ju = geo.Ju[C2(wrapi(iff, nx), j)];
                double m = 0.5 * (ju * U[C3(wrapi(iff, nx), j, k - 1)] + ju * U[C3(wrapi(iff, nx), j, k)]);
                fx[s] = m * or_face(ww[C3(wrapi(iff - 2, nx), j, k)], ww[C3(wrapi(iff - 1, nx), j, k)],
                                    ww[C3(wrapi(iff, nx), j, k)], ww[C3(wrapi(iff + 1, nx), j, k)],
                                    m, LIM);
                int jf = j + s;
                double jv = geo.Jv[C2(i, wrapi(jf, ny))];
                m = 0.5 * (jv * V[C3(i, wrapi(jf, ny), k - 1)] + jv * V[C3(i, wrapi(jf, ny), k)]);
                fy[s] = m * or_face(ww[C3(i, wrapi(jf - 2, ny), k)], ww[C3(i, wrapi(jf - 1, ny), k)],
                                    ww[C3(i, wrapi(jf, ny), k)], ww[C3(i, wrapi(jf + 1, ny), k)],
                                    m, LIM);
                int cc = k - 1 + s;                   /* centre of cell cc */
                m = 0.5 * (om[C3(i, j, cc)] + om[C3(i, j, cc + 1)]);
                fz[s] = m * or_face(ww[C3(i, j, clampi(cc - 1, 0, nz))], ww[C3(i, j, cc)],
                                    ww[C3(i, j, cc + 1)], ww[C3(i, j, clampi(cc + 2, 0, nz))],
                                    m, LIM);
            }
            SW[c] = -((fx[1] - fx[0]) / dx + (fy[1] - fy[0]) / dy + (fz[1] - fz[0]) / vm.dzf[k]) /
                    geo.J[C2(i, j)];
        }
    }
#undef C2
    free(rho); free(th); free(uu); free(vv); free(ww); free(om);
    vmet_free(&vm);
    geo_free(&geo);
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Thomas algorithm for a[r] x[r-1] + b[r] x[r] + c[r] x[r+1] = d[r],
 * r = 0..n-1 (a[0] and c[n-1] ignored), no pivoting.  Returns OR_ENOTDOM if
 * a row is not strictly diagonally dominant.
 * ---------------------------------------------------------------------- */
int or_thomas(int n, const double *a, const double *b, const double *c, const double *d,
              double *x, double *work)
{
    if (n <= 0) return OR_OK;
    int rc = OR_OK;
    for (int r = 0; r < n; ++r) {
        double off = (r > 0 ? fabs(a[r]) : 0.0) + (r < n - 1 ? fabs(c[r]) : 0.0);
        if (!(fabs(b[r]) > off)) rc = OR_ENOTDOM;
    }
    double *cp = work, *dp = work + n;
    cp[0] = c[0] / b[0];
    dp[0] = d[0] / b[0];
    for (int r = 1; r < n; ++r) {
        double den = b[r] - a[r] * cp[r - 1];
        cp[r] = c[r] / den;
        dp[r] = (d[r] - a[r] * dp[r - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int r = n - 2; r >= 0; --r) x[r] = dp[r] - cp[r] * x[r + 1];
    return rc;
}

/* ------------------------------------------------------------------------
 * The vertical part of one short step for one column.
 *
 * Inputs per cell m = 0..nz-1: rt (rho' after the horizontal divergence),
 * tt (Theta' after it), rp and pp (rho' and p' at the start of the short
 * step), P0, Cs, ths (stage coefficients); per level face k = 0..nz: W (old),
 * Wb (the W the increment is added to; W itself except in the second stage
 * of the Runge-Kutta short step), SW and E (the terrain-slope part of the
 * flux through the zeta surface, zero on flat ground).  dz and dzf are the column's own thicknesses
 * (J dzeta with terrain).  With Omega* = beta W+ + (1-beta) W - E:
 *   rho'+_m   = rt_m - (dtau/dz_m) (Omega*_{m+1} - Omega*_m)
 *   Theta'+_m = tt_m - (dtau/dz_m) (thf_{m+1} Omega*_{m+1} - thf_m Omega*_m)
 *   p'+       = P0 + Cs Theta'+
 *   W+_k      = Wb_k + dtau [ SW_k - (p*_k - p*_{k-1})/dzf_k
 *                            - g (a_k rho*_k + b_k rho*_{k-1}) ]
 * with p* = beta p'+ + (1-beta) p', rho* = beta rho'+ + (1-beta) rho',
 * thf the linear interpolation of ths to the faces, and W+ = Omega* = 0 on
 * the lids.  Substituting the first three lines into the last gives the
 * tridiagonal system assembled by or_vi_assemble for the interior faces
 * k = 1..nz-1.
 * ---------------------------------------------------------------------- */
typedef struct {
    int nz;
    const double *dz, *dzf, *a, *b, *E;
    double beta, dtau, grav;
} or_col;

static void col_thf(const or_col *c, const double *ths, double *thf)
{
    thf[0] = 0.0;
    thf[c->nz] = 0.0;
    for (int k = 1; k < c->nz; ++k) thf[k] = c->a[k] * ths[k] + c->b[k] * ths[k - 1];
}

/* A, B, C, D indexed by face k (entries 1..nz-1 used). */
static void col_assemble(const or_col *c, const double *rt, const double *tt, const double *rp,
                         const double *pp, const double *P0, const double *Cs, const double *ths,
                         const double *W, const double *Wb, const double *SW, double *A,
                         double *B, double *Cc, double *D, double *thf, double *pE, double *rEs)
{
    const int nz = c->nz;
    const double be = c->beta, dt = c->dtau, g = c->grav;
    const double *E = c->E;
    col_thf(c, ths, thf);
    for (int m = 0; m < nz; ++m) {
        /* the state each cell would reach with W+ = 0 */
        double the = tt[m] - ((1.0 - be) * dt / c->dz[m]) * (thf[m + 1] * W[m + 1] - thf[m] * W[m])
                     + (dt / c->dz[m]) * (thf[m + 1] * E[m + 1] - thf[m] * E[m]);
        double rhe = rt[m] - ((1.0 - be) * dt / c->dz[m]) * (W[m + 1] - W[m])
                     + (dt / c->dz[m]) * (E[m + 1] - E[m]);
        pE[m] = be * (P0[m] + Cs[m] * the) + (1.0 - be) * pp[m];
        rEs[m] = be * rhe + (1.0 - be) * rp[m];
    }
    const double mu = be * be * dt * dt;
    for (int k = 1; k < nz; ++k) {
        const double dzm = c->dz[k - 1], dzp = c->dz[k], dzf = c->dzf[k];
        A[k] = -mu * Cs[k - 1] * thf[k - 1] / (dzf * dzm) + mu * g * c->b[k] / dzm;
        Cc[k] = -mu * Cs[k] * thf[k + 1] / (dzf * dzp) - mu * g * c->a[k] / dzp;
        B[k] = 1.0 + mu * thf[k] * (Cs[k] / dzp + Cs[k - 1] / dzm) / dzf
               + mu * g * (c->a[k] / dzp - c->b[k] / dzm);
        D[k] = Wb[k] + dt * SW[k] - (dt / dzf) * (pE[k] - pE[k - 1])
               - dt * g * (c->a[k] * rEs[k] + c->b[k] * rEs[k - 1]);
    }
}

/* Apply the update equations above for a given W+ (lids set to 0 by caller). */
static void col_update(const or_col *c, const double *rt, const double *tt, const double *thf,
                       const double *W, const double *Wp, double *rpo, double *tpo)
{
    const int nz = c->nz;
    const double be = c->beta, dt = c->dtau;
    const double *E = c->E;
    for (int m = 0; m < nz; ++m) {
        double wsl = be * Wp[m] + (1.0 - be) * W[m] - E[m];
        double wsu = be * Wp[m + 1] + (1.0 - be) * W[m + 1] - E[m + 1];
        rpo[m] = rt[m] - (dt / c->dz[m]) * (wsu - wsl);
        tpo[m] = tt[m] - (dt / c->dz[m]) * (thf[m + 1] * wsu - thf[m] * wsl);
    }
}

/* Residual of the W+ equation, R_k = W+_k - (right-hand side), k = 1..nz-1,
 * evaluated directly from the update equations for a trial W+ (lids 0). */
static void col_residual(const or_col *c, const double *rt, const double *tt, const double *rp,
                         const double *pp, const double *P0, const double *Cs, const double *ths,
                         const double *W, const double *Wb, const double *SW, const double *Wp,
                         double *R, double *thf, double *rpo, double *tpo)
{
    const int nz = c->nz;
    const double be = c->beta, dt = c->dtau, g = c->grav;
    col_thf(c, ths, thf);
    col_update(c, rt, tt, thf, W, Wp, rpo, tpo);
    R[0] = 0.0;
    R[nz] = 0.0;
    for (int k = 1; k < nz; ++k) {
        double pk = be * (P0[k] + Cs[k] * tpo[k]) + (1.0 - be) * pp[k];
        double pkm = be * (P0[k - 1] + Cs[k - 1] * tpo[k - 1]) + (1.0 - be) * pp[k - 1];
        double rk = be * rpo[k] + (1.0 - be) * rp[k];
        double rkm = be * rpo[k - 1] + (1.0 - be) * rp[k - 1];
        double rhs = Wb[k] + dt * (SW[k] - (pk - pkm) / c->dzf[k] - g * (c->a[k] * rk + c->b[k] * rkm));
        R[k] = Wp[k] - rhs;
    }
}

/* Column set-up of the test entry points below: the column's thicknesses
 * scaled by its Jacobian jac, and E (NULL: zero).  Returns the scratch of
 * 6 (nz+1) doubles that holds them and the column temporaries. */
static double *col_setup(int nz, const or_vmet *vm, double jac, const double *E, or_col *c,
                         double beta, double dtau, double grav)
{
    const size_t np = (size_t)nz + 1;
    double *tmp = (double *)calloc(6 * np, sizeof(double));
    if (!tmp) return NULL;
    double *dz = tmp + 3 * np, *dzf = tmp + 4 * np, *e = tmp + 5 * np;
    for (int k = 0; k < nz; ++k) dz[k] = jac * vm->dz[k];
    for (int k = 0; k <= nz; ++k) {
        dzf[k] = jac * vm->dzf[k];
        e[k] = (E && k > 0 && k < nz) ? E[k] : 0.0;
    }
    c->nz = nz; c->dz = dz; c->dzf = dzf; c->a = vm->a; c->b = vm->b; c->E = e;
    c->beta = beta; c->dtau = dtau; c->grav = grav;
    return tmp;
}

/* Column test entry points.  All arrays follow the column conventions above;
 * A, B, C, D and R have nz+1 entries indexed by face.  jac is the column's
 * Jacobian (1 on flat ground); E has nz+1 entries or is NULL (zero). */
int or_vi_assemble(int nz, const double *zf, double beta, double dtau, double grav, double jac,
                   const double *E, const double *rt, const double *tt, const double *rp,
                   const double *pp, const double *P0, const double *Cs, const double *ths,
                   const double *W, const double *SW, double *A, double *B, double *C, double *D)
{
    or_grid g;
    memset(&g, 0, sizeof g);
    g.nz = nz; g.zf = zf;
    or_vmet vm;
    if (vmet_init(&g, &vm) != OR_OK) { vmet_free(&vm); return OR_ENOMEM; }
    or_col c;
    double *tmp = col_setup(nz, &vm, jac, E, &c, beta, dtau, grav);
    if (!tmp) { vmet_free(&vm); return OR_ENOMEM; }
    col_assemble(&c, rt, tt, rp, pp, P0, Cs, ths, W, W, SW, A, B, C, D, tmp, tmp + nz + 1,
                 tmp + 2 * (nz + 1));
    A[0] = B[0] = C[0] = D[0] = 0.0;
    A[nz] = B[nz] = C[nz] = D[nz] = 0.0;
    free(tmp);
    vmet_free(&vm);
    return OR_OK;
}

int or_vi_residual(int nz, const double *zf, double beta, double dtau, double grav, double jac,
                   const double *E, const double *rt, const double *tt, const double *rp,
                   const double *pp, const double *P0, const double *Cs, const double *ths,
                   const double *W, const double *SW, const double *Wp, double *R)
{
    or_grid g;
    memset(&g, 0, sizeof g);
    g.nz = nz; g.zf = zf;
    or_vmet vm;
    if (vmet_init(&g, &vm) != OR_OK) { vmet_free(&vm); return OR_ENOMEM; }
    or_col c;
    double *tmp = col_setup(nz, &vm, jac, E, &c, beta, dtau, grav);
    if (!tmp) { vmet_free(&vm); return OR_ENOMEM; }
    col_residual(&c, rt, tt, rp, pp, P0, Cs, ths, W, W, SW, Wp, R, tmp, tmp + nz + 1, tmp + 2 * (nz + 1));
    free(tmp);
    vmet_free(&vm);
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * One short step Phi(base, ev, dtau) into out (distinct from both) with the
 * stage's slow arrays sl = {S_U, S_V, S_W, R_Theta, theta_s, P0_s, C_s}:
 * increments are added to `base`; p' of the horizontal pressure gradient and
 * the old-time (1 - beta) parts of the vertical coupling come from `ev`.
 * The forward-backward short step is Phi(X, X, dtau).
 * ---------------------------------------------------------------------- */
static int short_step(const or_grid *g, const or_vmet *vm, const or_geo *geo,
                      const double *const sl[7], const double *const base[5],
                      const double *const ev[5], double dtau, double *const out[5], double *pp)
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t nxy = (size_t)nx * ny;
    const double *rp = base[0], *U = base[1], *V = base[2], *Wb = base[3], *tp = base[4];
    const double *rpe = ev[0], *W = ev[3], *tpe = ev[4];
    const double *SU = sl[0], *SV = sl[1], *SW = sl[2], *RT = sl[3];
    const double *ths = sl[4], *P0 = sl[5], *Cs = sl[6];
    double *rpo = out[0], *Uo = out[1], *Vo = out[2], *Wo = out[3], *tpo = out[4];
    const double dx = g->dx, dy = g->dy;
    int bad = 0;
#define C2(i, j) ((size_t)(j) * (size_t)nx + (size_t)(i))

    /* p' of the evaluation state's Theta' with the stage linearisation */
#pragma omp parallel for schedule(static)
    for (int jk = 0; jk < ny * nz; ++jk) {
        int j = jk % ny, k = jk / ny;
        for (int i = 0; i < nx; ++i) {
            size_t c = C3(i, j, k);
            pp[c] = P0[c] + Cs[c] * tpe[c];
        }
    }
    /* horizontally explicit momentum, forward in time.  Over terrain the
     * gradient along the zeta surface is corrected by (z_x/J) dp'/dzeta,
     * with dp'/dzeta at a cell centre the mean of the differences over its
     * two level faces (the one inner face at the lowest and highest cell),
     * averaged over the two columns of the face. */
#pragma omp parallel for schedule(static)
    for (int jk = 0; jk < ny * nz; ++jk) {
        int j = jk % ny, k = jk / ny;
        for (int i = 0; i < nx; ++i) {
            size_t c = C3(i, j, k);
            double corr_x = 0.0, corr_y = 0.0;
            if (g->terrain) {
                double gz[3];
                const int ci[3] = {i, wrapi(i - 1, nx), i};
                const int cj[3] = {j, j, wrapi(j - 1, ny)};
                for (int q = 0; q < 3; ++q) {
                    const int ii = ci[q], jj = cj[q];
                    if (k == 0) {
                        gz[q] = (pp[C3(ii, jj, 1)] - pp[C3(ii, jj, 0)]) / vm->dzf[1];
                    } else if (k == nz - 1) {
                        gz[q] = (pp[C3(ii, jj, k)] - pp[C3(ii, jj, k - 1)]) / vm->dzf[k];
                    } else {
                        gz[q] = 0.5 * ((pp[C3(ii, jj, k)] - pp[C3(ii, jj, k - 1)]) / vm->dzf[k] +
                                       (pp[C3(ii, jj, k + 1)] - pp[C3(ii, jj, k)]) / vm->dzf[k + 1]);
                    }
                }
                corr_x = (geo->dc[k] * geo->su[C2(i, j)] / geo->Ju[C2(i, j)]) * (0.5 * (gz[1] + gz[0]));
                corr_y = (geo->dc[k] * geo->sv[C2(i, j)] / geo->Jv[C2(i, j)]) * (0.5 * (gz[2] + gz[0]));
            }
            Uo[c] = U[c] + dtau * (SU[c] - ((pp[c] - pp[C3(wrapi(i - 1, nx), j, k)]) / dx - corr_x));
            Vo[c] = V[c] + dtau * (SV[c] - ((pp[c] - pp[C3(i, wrapi(j - 1, ny), k)]) / dy - corr_y));
        }
    }
    /* horizontal divergences of the new momentum; rho~ and Theta~ are kept
     * in the output arrays until the vertical part overwrites them */
#pragma omp parallel for schedule(static)
    for (int jk = 0; jk < ny * nz; ++jk) {
        int j = jk % ny, k = jk / ny;
        for (int i = 0; i < nx; ++i) {
            size_t c = C3(i, j, k);
            size_t ce = C3(wrapi(i + 1, nx), j, k), cw = C3(wrapi(i - 1, nx), j, k);
            size_t cn = C3(i, wrapi(j + 1, ny), k), cs = C3(i, wrapi(j - 1, ny), k);
            const double jw = geo->Ju[C2(i, j)], je = geo->Ju[C2(wrapi(i + 1, nx), j)];
            const double js = geo->Jv[C2(i, j)], jn = geo->Jv[C2(i, wrapi(j + 1, ny))];
            const double jc = geo->J[C2(i, j)];
            double div = ((je * Uo[ce] - jw * Uo[c]) / dx + (jn * Vo[cn] - js * Vo[c]) / dy) / jc;
            double thw = 0.5 * (ths[cw] + ths[c]), the = 0.5 * (ths[c] + ths[ce]);
            double ths_ = 0.5 * (ths[cs] + ths[c]), thn = 0.5 * (ths[c] + ths[cn]);
            double tdiv = ((the * (je * Uo[ce]) - thw * (jw * Uo[c])) / dx +
                           (thn * (jn * Vo[cn]) - ths_ * (js * Vo[c])) / dy) / jc;
            rpo[c] = rp[c] - dtau * div;
            tpo[c] = tp[c] + dtau * (RT[c] - tdiv);
        }
    }
    /* vertically implicit part, one tridiagonal system per column */
#pragma omp parallel reduction(| : bad)
    {
        size_t nzp = (size_t)nz + 1;
        double *buf = (double *)malloc(sizeof(double) * nzp * 28);
        if (!buf) {
            bad |= 2;
        } else {
            double *crt = buf, *ctt = buf + nzp, *crp = buf + 2 * nzp, *cpp = buf + 3 * nzp;
            double *cP0 = buf + 4 * nzp, *cCs = buf + 5 * nzp, *cth = buf + 6 * nzp;
            double *cW = buf + 7 * nzp, *cSW = buf + 8 * nzp, *A = buf + 9 * nzp;
            double *B = buf + 10 * nzp, *Cc = buf + 11 * nzp, *D = buf + 12 * nzp;
            double *thf = buf + 13 * nzp, *pE = buf + 14 * nzp, *rEs = buf + 15 * nzp;
            double *Wp = buf + 16 * nzp, *x = buf + 17 * nzp, *work = buf + 18 * nzp;
            double *orp = buf + 20 * nzp, *otp = buf + 21 * nzp;
            double *cdz = buf + 22 * nzp, *cdzf = buf + 23 * nzp, *cE = buf + 24 * nzp;
            double *cWb = buf + 27 * nzp;
#pragma omp for schedule(static)
            for (long col_id = 0; col_id < (long)nxy; ++col_id) {
                int i = (int)(col_id % nx), j = (int)(col_id / nx);
                const double jc = geo->J[C2(i, j)];
                const double su0 = geo->su[C2(i, j)], su1 = geo->su[C2(wrapi(i + 1, nx), j)];
                const double sv0 = geo->sv[C2(i, j)], sv1 = geo->sv[C2(i, wrapi(j + 1, ny))];
                for (int m = 0; m < nz; ++m) {
                    size_t c = C3(i, j, m);
                    crt[m] = rpo[c]; ctt[m] = tpo[c]; crp[m] = rpe[c]; cpp[m] = pp[c];
                    cP0[m] = P0[c]; cCs[m] = Cs[c]; cth[m] = ths[c];
                    cdz[m] = jc * vm->dz[m];
                }
                for (int k = 0; k <= nz; ++k) {
                    cW[k] = W[C3(i, j, k)];
                    cWb[k] = Wb[C3(i, j, k)];
                    cSW[k] = SW[C3(i, j, k)];
                    cdzf[k] = jc * vm->dzf[k];
                    cE[k] = 0.0;
                    if (g->terrain && k > 0 && k < nz) {
                        /* slope part of Omega from the new horizontal momentum */
                        const double mxk = 0.5 * (su0 * Uo[C3(i, j, k)] + su1 * Uo[C3(wrapi(i + 1, nx), j, k)]);
                        const double mxm = 0.5 * (su0 * Uo[C3(i, j, k - 1)] + su1 * Uo[C3(wrapi(i + 1, nx), j, k - 1)]);
                        const double myk = 0.5 * (sv0 * Vo[C3(i, j, k)] + sv1 * Vo[C3(i, wrapi(j + 1, ny), k)]);
                        const double mym = 0.5 * (sv0 * Vo[C3(i, j, k - 1)] + sv1 * Vo[C3(i, wrapi(j + 1, ny), k - 1)]);
                        cE[k] = geo->df[k] * ((vm->a[k] * mxk + vm->b[k] * mxm) + (vm->a[k] * myk + vm->b[k] * mym));
                    }
                }
                or_col col = {nz, cdz, cdzf, vm->a, vm->b, cE, g->beta, dtau, g->grav};
                col_assemble(&col, crt, ctt, crp, cpp, cP0, cCs, cth, cW, cWb, cSW, A, B, Cc, D, thf, pE,
                             rEs);
                Wp[0] = 0.0;
                Wp[nz] = 0.0;
                if (nz > 1) {
                    if (or_thomas(nz - 1, A + 1, B + 1, Cc + 1, D + 1, x, work) != OR_OK) bad |= 1;
                    for (int k = 1; k < nz; ++k) Wp[k] = x[k - 1];
                }
                col_update(&col, crt, ctt, thf, cW, Wp, orp, otp);
                for (int m = 0; m < nz; ++m) {
                    size_t c = C3(i, j, m);
                    rpo[c] = orp[m];
                    tpo[c] = otp[m];
                }
                for (int k = 0; k <= nz; ++k) Wo[C3(i, j, k)] = Wp[k];
            }
            free(buf);
        }
    }
#undef C2
    if (bad & 2) return OR_ENOMEM;
    if (bad & 1) return OR_ENOTDOM;
    return OR_OK;
}

static void round_f32(double *x, size_t n)
{
#pragma omp parallel for schedule(static)
    for (long q = 0; q < (long)n; ++q) x[q] = (double)(float)x[q];
}

/* ------------------------------------------------------------------------
 * Lateral and upper damping of st in place at time t after a short step of
 * length dtau (see the header).  W's level face k uses nu_top of level k.
 * ---------------------------------------------------------------------- */
int or_damp(const or_grid *g, double *const st[5], double dtau, double t)
{
    if (!g || !g->nu_lat || !g->nu_top) return OR_OK;
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t nxy = (size_t)nx * ny;
    double tr = (t - g->t1) / (g->t2 - g->t1);
    tr = tr < 0.0 ? 0.0 : (tr > 1.0 ? 1.0 : tr);
    const double mt = 1.0 - tr;
    for (int f = 0; f < 5; ++f) {
        const int nk = f == 3 ? nz + 1 : nz;
        double *x = st[f];
        const double *b1 = g->bnd1[f], *b2 = g->bnd2[f];
#pragma omp parallel for schedule(static)
        for (int jk = 0; jk < ny * nk; ++jk) {
            int j = jk % ny, k = jk / ny;
            if (f == 3 && (k == 0 || k == nz)) continue;
            const int kl = k < nz ? k : nz - 1;
            for (int i = 0; i < nx; ++i) {
                size_t c = C3(i, j, k);
                const double nu = g->nu_lat[(size_t)j * nx + i] + g->nu_top[kl];
                if (nu == 0.0) continue;
                double ref = 0.0;
                if (f == 0) ref = g->rho_ref[RI(g, c, k)];
                if (f == 4) ref = g->rt_ref[RI(g, c, k)];
                const double tgt = mt * (ref + b1[c]) + tr * (ref + b2[c]) - ref;
                const double cf = dtau * nu;
                x[c] = (x[c] + cf * tgt) / (1.0 + cf);
            }
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * n_long RK3 long steps of length dt with n_short short steps per stage,
 * in place on st = {rho', U, V, W, Theta'}.
 *
 * Stage s = 1, 2, 3 has length dt/3, dt/2, dt: the slow sweep is evaluated on
 * the previous stage's result (the start state for s = 1), then the n short
 * steps of length (stage length)/n restart from the start state.  The third
 * stage's result is the new state.  Each short step is the forward-backward
 * step, or with g->short_rk2 the two-stage Runge-Kutta form.
 *
 * f32_storage != 0 rounds every stored field and slow array to binary32
 * after each sweep: a model of binary32 storage used to size the tolerances
 * of reduced-precision runs (it is not part of the method).
 * ---------------------------------------------------------------------- */
int or_step(const or_grid *g, double *const st[5], double dt, int n_long, int n_short,
            int f32_storage)
{
    if (!g || g->nx < 1 || g->ny < 1 || g->nz < 2 || n_short < 1 || n_long < 0) return OR_EARG;
    const size_t nxy = (size_t)g->nx * g->ny, n = nxy * g->nz, nw = nxy * (g->nz + 1);
    const size_t sz[5] = {n, n, n, nw, n};
    or_vmet vm;
    or_geo geo;
    memset(&geo, 0, sizeof geo);
    if (vmet_init(g, &vm) != OR_OK || geo_init(g, &geo) != OR_OK) {
        vmet_free(&vm); geo_free(&geo);
        return OR_ENOMEM;
    }
    double *mem = (double *)malloc(sizeof(double) * (4 * (4 * n + nw) + 6 * n + nw + n));
    if (!mem) { vmet_free(&vm); geo_free(&geo); return OR_ENOMEM; }
    double *bufs[4][5], *sl[7], *pp;   /* [3]: first-stage value of the RK2 short step */
    double *p = mem;
    for (int b = 0; b < 4; ++b)
        for (int f = 0; f < 5; ++f) { bufs[b][f] = p; p += sz[f]; }
    for (int f = 0; f < 7; ++f) { sl[f] = p; p += (f == 2 ? nw : n); }
    pp = p;
    int rc = OR_OK;
    for (int step = 0; step < n_long && rc == OR_OK; ++step) {
        double *start[5], *stage_in[5];
        for (int f = 0; f < 5; ++f) {
            start[f] = bufs[0][f];
            memcpy(start[f], st[f], sz[f] * sizeof(double));
            stage_in[f] = start[f];
        }
        const double frac[3] = {1.0 / 3.0, 0.5, 1.0};
        for (int s = 0; s < 3 && rc == OR_OK; ++s) {
            rc = or_slow_sweep(g, (const double *const *)stage_in, sl);
            if (rc != OR_OK) break;
            if (f32_storage)
                for (int f = 0; f < 7; ++f) round_f32(sl[f], f == 2 ? nw : n);
            double dtau = (dt * frac[s]) / n_short;
            double *const *src = start;
            for (int q = 0; q < n_short; ++q) {
                double *const *dst = bufs[1 + (q & 1)];
                const double *const *cs = (const double *const *)sl;
                const double *const *in = (const double *const *)src;
                int r;
                if (g->short_rk2) {
                    /* X* = Phi(X, X, dtau/2), then X+ = Phi(X, X*, dtau) */
                    r = short_step(g, &vm, &geo, cs, in, in, 0.5 * dtau, bufs[3], pp);
                    if (r == OR_ENOMEM) { rc = r; break; }
                    if (r == OR_ENOTDOM) rc = r;
                    if (f32_storage)
                        for (int f = 0; f < 5; ++f) round_f32(bufs[3][f], sz[f]);
                    r = short_step(g, &vm, &geo, cs, in, (const double *const *)bufs[3], dtau, dst, pp);
                } else {
                    r = short_step(g, &vm, &geo, cs, in, in, dtau, dst, pp);
                }
                if (r == OR_ENOMEM) { rc = r; break; }
                if (r == OR_ENOTDOM) rc = r;
                /* damping at the end of the short step: t_n + (q+1) dtau */
                or_damp(g, dst, dtau, g->time0 + step * dt + (q + 1) * dtau);
                if (f32_storage)
                    for (int f = 0; f < 5; ++f) round_f32(dst[f], sz[f]);
                src = dst;
            }
            for (int f = 0; f < 5; ++f) stage_in[f] = src[f];
        }
        for (int f = 0; f < 5; ++f) memcpy(st[f], stage_in[f], sz[f] * sizeof(double));
    }
    free(mem);
    vmet_free(&vm);
    geo_free(&geo);
    return rc;
}

/* Exported single short step, for tests: st_out = short step of st_in. */
int or_short_step(const or_grid *g, const double *const sl[7], const double *const in[5],
                  double dtau, double *const out[5])
{
    const size_t n = (size_t)g->nx * g->ny * g->nz;
    or_vmet vm;
    or_geo geo;
    memset(&geo, 0, sizeof geo);
    if (vmet_init(g, &vm) != OR_OK || geo_init(g, &geo) != OR_OK) {
        vmet_free(&vm); geo_free(&geo);
        return OR_ENOMEM;
    }
    double *pp = (double *)malloc(n * sizeof(double));
    if (!pp) { vmet_free(&vm); geo_free(&geo); return OR_ENOMEM; }
    int rc = short_step(g, &vm, &geo, sl, in, in, dtau, out, pp);
    free(pp);
    vmet_free(&vm);
    geo_free(&geo);
    return rc;
}

/* ------------------------------------------------------------------------
 * Total mass M = sum (rho_ref + rho') J dx dy dz_k, summed serially in
 * memory order with Neumaier's compensated summation (J = 1 on flat ground).
 * ---------------------------------------------------------------------- */
static inline double jac_of(const or_grid *g, int i, int j)
{
    return g->terrain ? 1.0 - g->terrain[(size_t)j * g->nx + i] / g->zf[g->nz] : 1.0;
}

double or_mass(const or_grid *g, const double *rp)
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t nxy = (size_t)nx * ny;
    double s = 0.0, comp = 0.0;
    for (int k = 0; k < nz; ++k) {
        double vol = g->dx * g->dy * (g->zf[k + 1] - g->zf[k]);
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = C3(i, j, k);
                double x = ((g->rho_ref[RI(g, c, k)] + rp[c]) * vol) * jac_of(g, i, j);
                double t = s + x;
                if (fabs(s) >= fabs(x)) comp += (s - t) + x;
                else comp += (x - t) + s;
                s = t;
            }
    }
    return s + comp;
}

/* Diagnostic total energy: sum over cells of volume J dx dy dz times
 *   (1/2) [mean(U^2) + mean(V^2) + mean(W^2)] / rho + p/(gamma-1) + rho g z
 * with the means taken over the two faces of the cell and z the true height
 * of the cell centre.  Pinned by the closed-form energy of the isothermal
 * rest state (flat and over terrain) and by the kinetic increment of a
 * uniform flow. */
double or_energy(const or_grid *g, const double *const st[5])
{
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t nxy = (size_t)nx * ny;
    const double *rp = st[0], *U = st[1], *V = st[2], *W = st[3], *tp = st[4];
    const double H = g->zf[nz];
    double s = 0.0, comp = 0.0;
    for (int k = 0; k < nz; ++k) {
        double dz = g->zf[k + 1] - g->zf[k];
        double zc = 0.5 * (g->zf[k + 1] + g->zf[k]);
        double vol = g->dx * g->dy * dz;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = C3(i, j, k);
                const size_t r = RI(g, c, k);
                const double h = g->terrain ? g->terrain[(size_t)j * nx + i] : 0.0;
                const double z = zc + h * (1.0 - zc / H);
                double rho = g->rho_ref[r] + rp[c];
                double u2 = 0.5 * (U[c] * U[c] + U[C3(wrapi(i + 1, nx), j, k)] * U[C3(wrapi(i + 1, nx), j, k)]);
                double v2 = 0.5 * (V[c] * V[c] + V[C3(i, wrapi(j + 1, ny), k)] * V[C3(i, wrapi(j + 1, ny), k)]);
                double w2 = 0.5 * (W[c] * W[c] + W[C3(i, j, k + 1)] * W[C3(i, j, k + 1)]);
                double pres = g->p_ref[r] + g->p_ref[r] * expm1(OR_GAMMA * log1p(tp[c] / g->rt_ref[r]));
                double e = ((0.5 * (u2 + v2 + w2) / rho + pres / (OR_GAMMA - 1.0) + rho * g->grav * z) * vol) *
                           jac_of(g, i, j);
                double t = s + e;
                if (fabs(s) >= fabs(e)) comp += (s - t) + e;
                else comp += (e - t) + s;
                s = t;
            }
    }
    return s + comp;
}

/* Number of OpenMP threads the parallel loops use (1 without OpenMP). */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set that number (n >= 1); results do not depend on it. */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Seven-point diffusion, the stencil that dominates the paper's reduced
 * weather application (Sect. 4, performance model of no-cache and
 * perfect-cache bandwidth).  One explicit step on a uniform grid:
 *   q+ = q + ((kx lx + ky ly) + kz lz),  l_d = (q_{-d} + q_{+d}) - 2 q,
 * kd = nu dt / d^2, periodic in x and y, zero flux through the lids (the
 * missing vertical neighbour is the cell itself).  q and out are nz*ny*nx,
 * i fastest; out must not alias q.
 * ---------------------------------------------------------------------- */
int or_diffuse(int nx, int ny, int nz, double kx, double ky, double kz, const double *q,
               double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || !q || !out) return OR_EARG;
    const size_t nxy = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int jk = 0; jk < ny * nz; ++jk) {
        int j = jk % ny, k = jk / ny;
        for (int i = 0; i < nx; ++i) {
            size_t c = C3(i, j, k);
            double qc = q[c];
            double lx = (q[C3(wrapi(i - 1, nx), j, k)] + q[C3(wrapi(i + 1, nx), j, k)]) - 2.0 * qc;
            double ly = (q[C3(i, wrapi(j - 1, ny), k)] + q[C3(i, wrapi(j + 1, ny), k)]) - 2.0 * qc;
            double qd = k > 0 ? q[C3(i, j, k - 1)] : qc;
            double qu = k < nz - 1 ? q[C3(i, j, k + 1)] : qc;
            double lz = (qd + qu) - 2.0 * qc;
            out[c] = qc + ((kx * lx + ky * ly) + kz * lz);
        }
    }
    return OR_OK;
}
