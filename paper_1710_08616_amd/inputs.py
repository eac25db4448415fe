"""Seeded synthetic initial states for the HEVI dynamical-core step.

This module only *builds inputs*: vertical levels, hydrostatic reference
columns, warm bubbles, velocity noise and the named workload shapes.  It holds
none of the time-stepping arithmetic.  The CPU oracle and the GPU library both
take these arrays as inputs, and neither imports the other.

The paper runs its model on real JMA analyses (Sect. 4: a 301x301x58 grid and
the 1581x1301x58 production grid at 2 km).  Those data are not available, so
the states below stand in for them: a stretched 20 km column, an isothermal
hydrostatic atmosphere, warm bubbles and Gaussian velocity noise in a uniform
wind.  Every random number comes from a counter-based generator (splitmix64
of the seed, the field id and the cell index, then Box-Muller), so any
sub-block of a field can be regenerated without drawing the rest.

Layout: canonical i-fastest.  Cell fields have shape (nz, ny, nx); the
vertical momentum lives on the nz+1 level faces, shape (nz+1, ny, nx).

Terrain: a state may carry surface heights h (shape (ny, nx)); the cell
centres then sit at the true heights z = zeta + h (1 - zeta/H), and the
reference arrays are given per cell (shape (nz, ny, nx)) at those heights.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

# Physical constants of the synthetic atmosphere (SI units).
R_DRY = 287.04
CP_DRY = 3.5 * R_DRY
KAPPA = 2.0 / 7.0
GRAV = 9.80665
P00 = 1.0e5
H_TOP = 20000.0

FIELD_NAMES = ("rho_ptb", "rhou", "rhov", "rhow", "rhotheta_ptb")


# --------------------------------------------------------------------------
# counter-based random numbers
# --------------------------------------------------------------------------
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele, Lea & Flood 2014) on uint64 arrays."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _uniform01(bits: np.ndarray) -> np.ndarray:
    """Map 64 random bits to a double in (0, 1]."""
    return ((bits >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def gaussian(seed: int, component: int, shape, offset=(0, 0, 0), full=None) -> np.ndarray:
    """i.i.d. N(0,1) values indexed by (seed, component, k, j, i).

    ``shape`` is (nk, nj, ni); ``offset`` shifts the (k, j, i) counters so a
    sub-block reproduces the same numbers as the whole field would; ``full`` is
    the (nz, ny, nx) extent the counters are numbered over (defaults to shape).
    Generated one k-slab at a time to keep the temporaries small.
    """
    nk, nj, ni = shape
    full = shape if full is None else full
    out = np.empty((nk, nj, ni))
    j = np.arange(nj, dtype=np.uint64)[:, None] + np.uint64(offset[1])
    i = np.arange(ni, dtype=np.uint64)[None, :] + np.uint64(offset[2])
    with np.errstate(over="ignore"):
        base = splitmix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * np.uint64(0x100000001B3)
                          + np.uint64(component))
        plane = j * np.uint64(full[2]) + i
        for kk in range(nk):
            k = np.uint64(kk + offset[0])
            ctr = base + (k * np.uint64(full[1])) * np.uint64(full[2]) + plane
            u1 = _uniform01(splitmix64(ctr))
            u2 = _uniform01(splitmix64(ctr ^ np.uint64(0xD1B54A32D192ED03)))
            out[kk] = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    return out


# --------------------------------------------------------------------------
# vertical grid and reference columns
# --------------------------------------------------------------------------
def levels(nz: int, top: float = H_TOP) -> np.ndarray:
    """Stretched level faces zeta_k = H (s + s^2)/2, s = k/nz (nz+1 values)."""
    s = np.arange(nz + 1, dtype=np.float64) / nz
    z = top * (s + s * s) / 2.0
    z[0] = 0.0
    z[-1] = top
    return z


def uniform_levels(nz: int, top: float) -> np.ndarray:
    return np.linspace(0.0, top, nz + 1)


def centres(zf: np.ndarray) -> np.ndarray:
    return 0.5 * (zf[1:] + zf[:-1])


def reference_isothermal(zc: np.ndarray, t0: float = 300.0, p0: float = 1.0e5):
    """Hydrostatic isothermal atmosphere at the given heights.

    Returns (rho_ref, rhotheta_ref, p_ref): p = p0 exp(-z/Hs), Hs = R T0 / g,
    rho = p / (R T0), theta = T0 (P00/p)^kappa, rhotheta = rho * theta.
    """
    hs = R_DRY * t0 / GRAV
    p = p0 * np.exp(-zc / hs)
    rho = p / (R_DRY * t0)
    theta = t0 * (P00 / p) ** KAPPA
    return rho, rho * theta, p


def reference_neutral(zc: np.ndarray, theta0: float = 300.0):
    """Hydrostatic atmosphere of uniform potential temperature theta0."""
    exner = 1.0 - GRAV * zc / (CP_DRY * theta0)
    p = P00 * exner ** (CP_DRY / R_DRY)
    rho = p / (R_DRY * exner * theta0)
    return rho, rho * theta0, p


def reference_uniform(nz: int, rho0: float = 1.0, theta0: float = 300.0, gamma: float = 1.4):
    """Height-independent reference (only consistent for g = 0 test cases)."""
    rho = np.full(nz, rho0)
    rt = rho * theta0
    p = P00 * (R_DRY * rt / P00) ** gamma
    return rho, rt, p


# --------------------------------------------------------------------------
# states
# --------------------------------------------------------------------------
@dataclasses.dataclass
class State:
    """One synthetic domain: grid description, reference columns, fields."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    zf: np.ndarray
    rho_ref: np.ndarray
    rt_ref: np.ndarray
    p_ref: np.ndarray
    fields: List[np.ndarray]          # rho', U, V, W, Theta' (float64, canonical)
    dt: float = 10.0
    n_short: int = 4
    n_long: int = 10
    beta: float = 0.55
    name: str = ""
    terrain: Optional[np.ndarray] = None   # (ny, nx) surface heights; refs are 3D
    damping: Optional[dict] = None         # lateral / upper damping data (see damping())

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def copy(self) -> "State":
        return dataclasses.replace(self, fields=[f.copy() for f in self.fields])

    def as_f32(self, reference: bool = False) -> "State":
        """The same state with every field rounded to binary32 (kept as float64);
        with reference=True the reference arrays are rounded as well (what a
        binary32 path holds of them)."""
        r32 = lambda a: np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)
        out = dataclasses.replace(self, fields=[r32(f) for f in self.fields])
        if reference:
            out.rho_ref, out.rt_ref, out.p_ref = r32(self.rho_ref), r32(self.rt_ref), r32(self.p_ref)
        return out


def true_heights(zc: np.ndarray, terrain: Optional[np.ndarray]) -> np.ndarray:
    """Heights of the cell centres: zc as an (nz, 1, 1) column on flat
    ground, zc + h (1 - zc/H) of shape (nz, ny, nx) over terrain h."""
    zc = np.asarray(zc, dtype=np.float64)[:, None, None]
    if terrain is None:
        return zc
    return zc + terrain[None] * (1.0 - zc / H_TOP)


def orography(nx: int, ny: int, dx: float, dy: float, seed: int, hmax: float = 2000.0,
              hills: int = 8, smin: float = 8000.0, smax: float = 40000.0) -> np.ndarray:
    """Sum of ``hills`` Gaussian hills a exp(-r^2 / (2 sigma^2)), r the periodic
    horizontal distance to a centre ~ U over the domain, sigma ~ U[smin, smax],
    a ~ U[0.3, 1]; rescaled so that the highest point is ``hmax``."""
    rng = np.random.default_rng(seed)
    lx, ly = nx * dx, ny * dy
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    h = np.zeros((ny, nx))
    for _ in range(hills):
        sig = rng.uniform(smin, smax)
        amp = rng.uniform(0.3, 1.0)
        xc, yc = rng.uniform(0.0, lx), rng.uniform(0.0, ly)
        ddx = _periodic_dist(x, xc, lx)[None, :]
        ddy = _periodic_dist(y, yc, ly)[:, None]
        h += amp * np.exp(-(ddx * ddx + ddy * ddy) / (2.0 * sig * sig))
    return h * (hmax / h.max())


def _periodic_dist(x: np.ndarray, xc: float, length: float) -> np.ndarray:
    d = np.abs(x - xc)
    return np.minimum(d, length - d)


def bubble_theta(nx, ny, zc, dx, dy, bubbles, amp=2.0) -> np.ndarray:
    """Sum of cos^2 warm bubbles: amp * cos^2(pi r / 2) for r < 1.

    ``bubbles`` is a list of (xc, yc, zc, radius); r is the 3D distance
    (periodic in x and y) divided by the radius.  Each bubble is evaluated
    only on the index box that can hold r < 1.
    """
    lx, ly = nx * dx, ny * dy
    th = np.zeros((len(zc), ny, nx))
    for (xb, yb, zb, rb) in bubbles:
        kk = np.nonzero(np.abs(zc - zb) < rb)[0]
        if kk.size == 0:
            continue
        wi = min(nx, 2 * int(math.ceil(rb / dx)) + 3)
        wj = min(ny, 2 * int(math.ceil(rb / dy)) + 3)
        ii = (int(math.floor((xb - rb) / dx)) - 1 + np.arange(wi)) % nx
        jj = (int(math.floor((yb - rb) / dy)) - 1 + np.arange(wj)) % ny
        ddx = _periodic_dist((ii + 0.5) * dx, xb, lx)[None, None, :]
        ddy = _periodic_dist((jj + 0.5) * dy, yb, ly)[None, :, None]
        ddz = (zc[kk] - zb)[:, None, None]
        r = np.sqrt(ddx * ddx + ddy * ddy + ddz * ddz) / rb
        box = np.ix_(kk, jj, ii)
        th[box] += np.where(r < 1.0, amp * np.cos(0.5 * math.pi * np.minimum(r, 1.0)) ** 2, 0.0)
    return th


def random_bubbles(seed: int, count: int, lx: float, ly: float,
                   rmin=2000.0, rmax=8000.0, ztop=12000.0):
    """count bubbles: radius ~ U[rmin, rmax], x, y ~ U[0, L), z ~ U[r + 500 m, ztop]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        rb = rng.uniform(rmin, rmax)
        xb = rng.uniform(0.0, lx)
        yb = rng.uniform(0.0, ly)
        zb = rng.uniform(rb + 500.0, ztop)
        out.append((xb, yb, zb, rb))
    return out


def make_state(nx: int, ny: int, nz: int, dx: float = 2000.0, dy: float = 2000.0,
               seed: int = 1710, bubbles: Optional[list] = None, u_bg: float = 10.0,
               v_bg: float = 0.0, noise: float = 0.1, dt: float = 10.0, n_short: int = 4,
               n_long: int = 10, beta: float = 0.55, zf: Optional[np.ndarray] = None,
               reference: str = "isothermal", name: str = "",
               terrain: Optional[np.ndarray] = None, shear: float = 0.0) -> State:
    """Warm-bubble state at constant pressure in a uniform wind plus noise.

    Theta' = 0 and rho' = rhotheta_ref / (theta_ref + theta_bubble) - rho_ref,
    so the pressure is the reference pressure everywhere.  U = rho_u (u + n)
    with rho_u the two-point mean density on the x-face, u = u_bg +
    shear * z / H (z the mean true height of the face's two cells) and
    n ~ N(0, noise^2); V likewise with v_bg; W = rho_w n on interior faces and
    0 on the lids.  With ``terrain`` (surface heights, (ny, nx)) the reference
    is evaluated at every cell's true height; the bubbles stay defined in the
    zeta coordinate.
    """
    zf = levels(nz) if zf is None else np.asarray(zf, dtype=np.float64)
    zc = centres(zf)
    if terrain is not None:
        terrain = np.ascontiguousarray(terrain, dtype=np.float64)
        assert terrain.shape == (ny, nx)
    z3 = true_heights(zc, terrain)
    if reference == "isothermal":
        rho_ref, rt_ref, p_ref = reference_isothermal(z3)
    elif reference == "neutral":
        rho_ref, rt_ref, p_ref = reference_neutral(z3)
    else:
        raise ValueError(reference)
    th_ref = rt_ref / rho_ref
    if bubbles is None:
        bubbles = [(0.5 * nx * dx, 0.5 * ny * dy, 5000.0, 4000.0)]
    thb = bubble_theta(nx, ny, zc, dx, dy, bubbles)
    rho_full = rt_ref / (th_ref + thb)
    rho_p = rho_full - rho_ref
    rt_p = np.zeros((nz, ny, nx))
    rho_u = 0.5 * (np.roll(rho_full, 1, axis=2) + rho_full)
    rho_v = 0.5 * (np.roll(rho_full, 1, axis=1) + rho_full)
    u_prof = u_bg
    if shear != 0.0:
        zb = np.broadcast_to(z3, (nz, ny, nx))
        u_prof = u_bg + shear * (0.5 * (np.roll(zb, 1, axis=2) + zb)) / H_TOP
    U = rho_u * (u_prof + noise * gaussian(seed, 0, (nz, ny, nx)))
    V = rho_v * (v_bg + noise * gaussian(seed, 1, (nz, ny, nx)))
    dz = np.diff(zf)
    W = np.zeros((nz + 1, ny, nx))
    if nz > 1:
        a = dz[:-1] / (dz[:-1] + dz[1:])           # weight of the cell above face k
        b = dz[1:] / (dz[:-1] + dz[1:])            # weight of the cell below face k
        rho_w = a[:, None, None] * rho_full[1:] + b[:, None, None] * rho_full[:-1]
        W[1:nz] = rho_w * noise * gaussian(seed, 2, (nz + 1, ny, nx))[1:nz]
    if terrain is None:
        rho_ref, rt_ref, p_ref = (np.ascontiguousarray(r[:, 0, 0]) for r in (rho_ref, rt_ref, p_ref))
    return State(nx, ny, nz, dx, dy, zf, rho_ref, rt_ref, p_ref,
                 [rho_p, U, V, W, rt_p], dt=dt, n_short=n_short, n_long=n_long,
                 beta=beta, name=name, terrain=terrain)


def rest_state(nx, ny, nz, dx=2000.0, dy=2000.0, zf=None, reference="isothermal",
               **kw) -> State:
    zf = levels(nz) if zf is None else zf
    zc = centres(zf)
    ref = reference_isothermal(zc) if reference == "isothermal" else reference_neutral(zc)
    f = [np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx)),
         np.zeros((nz + 1, ny, nx)), np.zeros((nz, ny, nx))]
    return State(nx, ny, nz, dx, dy, zf, ref[0], ref[1], ref[2], f, **kw)


# --------------------------------------------------------------------------
# lateral and upper damping data
# --------------------------------------------------------------------------
def damping(s: "State", width: int = 8, nu_lat: float = 1.0 / 60.0, z_start: float = 15000.0,
            nu_top: float = 1.0 / 300.0, u1: float = 10.0, u2: float = 15.0, v2: float = 2.0,
            theta_amp: float = 0.5, t1: float = 0.0, t2: float = 600.0) -> dict:
    """Synthetic damping set-up for a state (boundary data stand in for a
    parent model).

    Rates: nu_lat (1 - d/width)^2 for columns d < width cells from the nearest
    domain edge, nu_top sin^2(pi/2 (z - z_start)/(H - z_start)) for cell
    centres above z_start.  Boundary states: at t1 a uniform wind u1 (U =
    rho_u u1, rho_u the mean reference density of the face's two cells), at
    t2 the wind
    (u2, v2) with a Theta perturbation theta_amp rho_ref sin(2 pi x / Lx);
    rho' = W = 0 in both.
    """
    nx, ny, nz = s.nx, s.ny, s.nz
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    d = np.minimum(np.minimum(i, nx - 1 - i), np.minimum(j, ny - 1 - j)).astype(np.float64)
    lat = np.where(d < width, nu_lat * ((width - d) / width) ** 2, 0.0)
    zc = centres(s.zf)
    top = np.where(zc > z_start,
                   nu_top * np.sin(0.5 * math.pi * (zc - z_start) / (s.zf[-1] - z_start)) ** 2, 0.0)
    rho = s.rho_ref if np.ndim(s.rho_ref) == 3 else np.broadcast_to(
        np.asarray(s.rho_ref)[:, None, None], (nz, ny, nx))
    rho_u = 0.5 * (np.roll(rho, 1, axis=2) + rho)
    rho_v = 0.5 * (np.roll(rho, 1, axis=1) + rho)
    zero_c = np.zeros((nz, ny, nx))
    zero_w = np.zeros((nz + 1, ny, nx))
    xs = (np.arange(nx) + 0.5) / nx
    b1 = [zero_c.copy(), rho_u * u1, zero_c.copy(), zero_w.copy(), zero_c.copy()]
    b2 = [zero_c.copy(), rho_u * u2, rho_v * v2, zero_w.copy(),
          theta_amp * rho * np.sin(2.0 * math.pi * xs)[None, None, :]]
    return {"nu_lat": np.ascontiguousarray(lat), "nu_top": np.ascontiguousarray(top),
            "bnd1": [np.ascontiguousarray(x) for x in b1],
            "bnd2": [np.ascontiguousarray(x) for x in b2], "t1": float(t1), "t2": float(t2)}


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
C_SOUND = 347.2   # acoustic speed of the isothermal 300 K reference (m/s)


def ensemble_dt(dx: float, dy: float, u_bg: float, n_short: int = 6,
                courant: float = 0.8, cap: float = 10.0) -> float:
    """Long step keeping the horizontal acoustic Courant number of the short
    step below ``courant``: min(cap, floor to 0.25 s of
    courant * n / ((c_s + |u_bg| + 1) * sqrt(1/dx^2 + 1/dy^2)))."""
    raw = courant * n_short / ((C_SOUND + abs(u_bg) + 1.0) * math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2))
    return min(cap, math.floor(raw / 0.25) * 0.25)


def ensemble(count: int = 48, seed: int = 1713, nmin: int = 128, nmax: int = 512,
             nzs=(32, 64), n_short: int = 6, n_long: int = 20) -> List[State]:
    """Independent members of uneven sizes, each drawn from its own seed
    seed*1000 + m: nx, ny ~ U{nmin..nmax}, nz from ``nzs``, dx = dy ~ U[1, 4] km,
    u_bg ~ U[0, 30] m/s, one bubble (r = 4 km at 5 km, random x, y) and noise."""
    out = []
    for m in range(count):
        ms = seed * 1000 + m
        rng = np.random.default_rng(ms)
        nx = int(rng.integers(nmin, nmax + 1))
        ny = int(rng.integers(nmin, nmax + 1))
        nz = int(nzs[int(rng.integers(0, len(nzs)))])
        dx = float(rng.uniform(1000.0, 4000.0))
        u_bg = float(rng.uniform(0.0, 30.0))
        xb, yb = float(rng.uniform(0.0, nx * dx)), float(rng.uniform(0.0, ny * dx))
        dt = ensemble_dt(dx, dx, u_bg, n_short)
        out.append(make_state(nx, ny, nz, dx=dx, dy=dx, seed=ms, bubbles=[(xb, yb, 5000.0, 4000.0)],
                              u_bg=u_bg, dt=dt, n_short=n_short, n_long=n_long,
                              name=f"member{m}"))
    return out


def workload(name: str) -> State:
    """The synthetic single-domain workloads used by tests and the benchmark.

    small       64x64x32, dx = 2 km, one bubble (r = 4 km, centre 5 km), FP64 run
                of 10 long steps with 4 short steps per stage, dt = 10 s.
    large       1024x1024x64, 16 bubbles (r in 2..8 km), 100 long steps, n = 6.
    large_sub   128x128x64 sub-run of the same generator (oracle-sized).
    xl          2048x2048x64, the same generator with 16 bubbles over 8 Gaussian
                hills (max 2 km), u = 10 m/s, 30 long steps, n = 6 (the
                layout-comparison domain).
    terrain     1600x1280x64 over 8 Gaussian hills (max 2 km), 16 bubbles, wind
                shear u = 30 z/H, 50 long steps, n = 6.
    terrain_sub 160x128x64 sub-run of the same generator (oracle-sized; hills
                and bubbles drawn for that domain).
    """
    if name == "small":
        return make_state(64, 64, 32, seed=1710, dt=10.0, n_short=4, n_long=10, name=name)
    if name == "xl":
        seed = 1714
        h = orography(2048, 2048, 2000.0, 2000.0, seed)
        bub = random_bubbles(seed, 16, 2048 * 2000.0, 2048 * 2000.0)
        return make_state(2048, 2048, 64, seed=seed, bubbles=bub, terrain=h, dt=10.0,
                          n_short=6, n_long=30, name=name)
    if name in ("terrain", "terrain_sub"):
        nx, ny = (1600, 1280) if name == "terrain" else (160, 128)
        seed = 1712
        h = orography(nx, ny, 2000.0, 2000.0, seed)
        bub = random_bubbles(seed, 16, nx * 2000.0, ny * 2000.0)
        return make_state(nx, ny, 64, seed=seed, bubbles=bub, u_bg=0.0, shear=30.0,
                          terrain=h, dt=10.0, n_short=6, n_long=50, name=name)
    if name in ("large", "large_sub"):
        n = 1024 if name == "large" else 128
        seed = 1711
        bub = random_bubbles(seed, 16, n * 2000.0, n * 2000.0)
        return make_state(n, n, 64, seed=seed, bubbles=bub, dt=10.0, n_short=6,
                          n_long=100, name=name)
    raise KeyError(name)
