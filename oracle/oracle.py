"""ctypes binding of the FP64 CPU oracle (hevi_oracle.c).

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only callers.  It imports nothing from the product
package; states are passed in as any object carrying the grid attributes
(nx, ny, nz, dx, dy, zf, rho_ref, rt_ref, p_ref, beta) and the five fields
(rho', U, V, W, Theta') in canonical i-fastest float64 layout.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hevi_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
GRAV = 9.80665

LIM_NONE = 0
LIM_KOREN = 1
OK, EARG, ENOMEM, ENOTDOM = 0, -1, -2, -3

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (contraction off, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("donor_cell", ctypes.c_int32), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("beta", ctypes.c_double), ("grav", ctypes.c_double),
                ("zf", _dp), ("rho_ref", _dp), ("rt_ref", _dp), ("p_ref", _dp),
                ("terrain", _dp), ("short_rk2", ctypes.c_int32),
                ("nu_lat", _dp), ("nu_top", _dp), ("bnd1", _dp * 5), ("bnd2", _dp * 5),
                ("t1", ctypes.c_double), ("t2", ctypes.c_double), ("time0", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.or_koren_phi.restype = ctypes.c_double
        L.or_koren_phi.argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_face.restype = ctypes.c_double
        L.or_face.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int]
        L.or_advect_fe.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, ctypes.c_double,
                                   ctypes.c_int, _dp]
        L.or_slow_sweep.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.or_short_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_double, ctypes.c_void_p]
        L.or_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                              ctypes.c_int, ctypes.c_int]
        L.or_thomas.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        col = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
               ctypes.c_double, _dp] + [_dp] * 9
        L.or_vi_assemble.argtypes = col + [_dp] * 4
        L.or_vi_residual.argtypes = col + [_dp, _dp]
        L.or_mass.restype = ctypes.c_double
        L.or_mass.argtypes = [ctypes.c_void_p, _dp]
        L.or_energy.restype = ctypes.c_double
        L.or_energy.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.or_diffuse.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [_dp, _dp]
        L.or_damp.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
        L.or_threads.restype = ctypes.c_int
        L.or_threads.argtypes = []
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class _GridHolder:
    """A filled or_grid plus the arrays it points into (kept alive)."""

    def __init__(self, s, grav: float = GRAV, beta=None, donor_cell: bool = False,
                 short_rk2: bool = False, time0: float = 0.0):
        self.zf = _f64(s.zf)
        self.rho_ref = _f64(s.rho_ref)
        self.rt_ref = _f64(s.rt_ref)
        self.p_ref = _f64(s.p_ref)
        h = getattr(s, "terrain", None)
        self.terrain = None if h is None else _f64(h)
        if self.terrain is not None:
            assert self.terrain.shape == (s.ny, s.nx)
            for r in (self.rho_ref, self.rt_ref, self.p_ref):
                assert r.shape == (s.nz, s.ny, s.nx)
        else:
            for r in (self.rho_ref, self.rt_ref, self.p_ref):
                assert r.shape == (s.nz,)
        self.g = _Grid(int(s.nx), int(s.ny), int(s.nz), 1 if donor_cell else 0,
                       float(s.dx), float(s.dy),
                       float(s.beta if beta is None else beta), float(grav),
                       _ptr(self.zf), _ptr(self.rho_ref), _ptr(self.rt_ref), _ptr(self.p_ref),
                       _dp() if self.terrain is None else _ptr(self.terrain),
                       1 if short_rk2 else 0)
        self.g.time0 = float(time0)
        dmp = getattr(s, "damping", None)
        if dmp is not None:
            self.nu_lat = _f64(dmp["nu_lat"])
            self.nu_top = _f64(dmp["nu_top"])
            assert self.nu_lat.shape == (s.ny, s.nx) and self.nu_top.shape == (s.nz,)
            self.bnd = [[_f64(x) for x in dmp["bnd1"]], [_f64(x) for x in dmp["bnd2"]]]
            for b in self.bnd:
                assert [x.shape for x in b] == [f.shape for f in s.fields]
            self.g.nu_lat = _ptr(self.nu_lat)
            self.g.nu_top = _ptr(self.nu_top)
            for f in range(5):
                self.g.bnd1[f] = _ptr(self.bnd[0][f])
                self.g.bnd2[f] = _ptr(self.bnd[1][f])
            self.g.t1 = float(dmp["t1"])
            self.g.t2 = float(dmp["t2"])

    @property
    def ref(self):
        return ctypes.byref(self.g)


def _ptr_array(arrs: Sequence[np.ndarray]):
    return (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])


def _shapes(s):
    c = (s.nz, s.ny, s.nx)
    w = (s.nz + 1, s.ny, s.nx)
    return [c, c, c, w, c]


def step(s, dt=None, n_long=None, n_short=None, f32_storage=False, grav: float = GRAV,
         check=True, donor_cell: bool = False, short_rk2: bool = False,
         time0: float = 0.0) -> List[np.ndarray]:
    """Advance a copy of the state's fields; returns the new five fields.

    donor_cell=True swaps the Koren face values for first-order upwind ones, a
    linear operator that exposes the RK3 stage structure in closed form (tests
    only; the model itself always uses the Koren limiter).  short_rk2=True
    takes the two-stage Runge-Kutta short step instead of the
    forward-backward one.  A state with a ``damping`` dict (nu_lat, nu_top,
    bnd1, bnd2, t1, t2) is damped after every short step; time0 is the model
    time at the start."""
    dt = s.dt if dt is None else dt
    n_long = s.n_long if n_long is None else n_long
    n_short = s.n_short if n_short is None else n_short
    gh = _GridHolder(s, grav, donor_cell=donor_cell, short_rk2=short_rk2, time0=time0)
    f = [_f64(x).copy() for x in s.fields]
    rc = lib().or_step(gh.ref, _ptr_array(f), float(dt), int(n_long), int(n_short),
                       1 if f32_storage else 0)
    if check and rc != OK:
        raise RuntimeError(f"or_step failed: {rc}")
    return f


def slow_sweep(s, fields=None, grav: float = GRAV, donor_cell: bool = False) -> List[np.ndarray]:
    """{S_U, S_V, S_W, R_Theta, theta_s, P0_s, C_s} of the given stage-input state
    (donor_cell: first-order upwind face values instead of Koren's, tests only)."""
    gh = _GridHolder(s, grav, donor_cell=donor_cell)
    f = [_f64(x) for x in (s.fields if fields is None else fields)]
    c = (s.nz, s.ny, s.nx)
    out = [np.zeros(c), np.zeros(c), np.zeros((s.nz + 1, s.ny, s.nx)), np.zeros(c),
           np.zeros(c), np.zeros(c), np.zeros(c)]
    rc = lib().or_slow_sweep(gh.ref, _ptr_array(f), _ptr_array(out))
    if rc != OK:
        raise RuntimeError(f"or_slow_sweep failed: {rc}")
    return out


def short_step(s, slow, dtau, fields=None, grav: float = GRAV) -> List[np.ndarray]:
    gh = _GridHolder(s, grav)
    f = [_f64(x) for x in (s.fields if fields is None else fields)]
    sl = [_f64(x) for x in slow]
    out = [np.zeros(sh) for sh in _shapes(s)]
    rc = lib().or_short_step(gh.ref, _ptr_array(sl), _ptr_array(f), float(dtau), _ptr_array(out))
    if rc != OK:
        raise RuntimeError(f"or_short_step failed: {rc}")
    return out


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().or_threads())


def set_threads(n: int) -> None:
    """Number of OpenMP threads for the following calls (bitwise the same results)."""
    lib().or_set_threads(int(n))


def koren_phi(dm: float, dp: float) -> float:
    return lib().or_koren_phi(float(dm), float(dp))


def face(qLL, qL, qR, qRR, m, lim=LIM_KOREN) -> float:
    return lib().or_face(float(qLL), float(qL), float(qR), float(qRR), float(m), int(lim))


def advect_fe(s, q, u, v, w, dt, lim) -> np.ndarray:
    gh = _GridHolder(s)
    q, u, v, w = (_f64(x) for x in (q, u, v, w))
    out = np.zeros_like(q)
    rc = lib().or_advect_fe(gh.ref, _ptr(q), _ptr(u), _ptr(v), _ptr(w), float(dt), int(lim),
                            _ptr(out))
    if rc != OK:
        raise RuntimeError(rc)
    return out


def thomas(a, b, c, d):
    a, b, c, d = (_f64(x) for x in (a, b, c, d))
    n = len(b)
    x = np.zeros(n)
    work = np.zeros(2 * n)
    rc = lib().or_thomas(n, _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(x), _ptr(work))
    return x, rc


def _col_args(zf, beta, dtau, grav, col, jac=1.0, E=None):
    keys = ("rt", "tt", "rp", "pp", "P0", "Cs", "ths", "W", "SW")
    arrs = [_f64(col[k]) for k in keys]
    zf = _f64(zf)
    arrs.append(zf)
    e = _dp()
    if E is not None:
        E = _f64(E)
        assert E.shape == (len(zf),)
        arrs.append(E)
        e = _ptr(E)
    return arrs, [len(zf) - 1, _ptr(zf), float(beta), float(dtau), float(grav), float(jac), e] + \
        [_ptr(a) for a in arrs[:9]]


def vi_assemble(zf, beta, dtau, grav, col, jac=1.0, E=None):
    """(A, B, C, D) indexed by level face (nz+1 entries, 1..nz-1 meaningful).

    jac: the column's Jacobian J (thicknesses J dzeta); E: the slope part of
    the flux through the zeta surfaces per level face (None: zero)."""
    zf = _f64(zf)
    nz = len(zf) - 1
    out = [np.zeros(nz + 1) for _ in range(4)]
    keep, args = _col_args(zf, beta, dtau, grav, col, jac, E)
    rc = lib().or_vi_assemble(*args, *[_ptr(o) for o in out])
    if rc != OK:
        raise RuntimeError(rc)
    return out


def vi_residual(zf, beta, dtau, grav, col, Wp, jac=1.0, E=None):
    zf = _f64(zf)
    nz = len(zf) - 1
    R = np.zeros(nz + 1)
    Wp = _f64(Wp)
    keep, args = _col_args(zf, beta, dtau, grav, col, jac, E)
    rc = lib().or_vi_residual(*args, _ptr(Wp), _ptr(R))
    if rc != OK:
        raise RuntimeError(rc)
    return R


def mass(s, rho_p=None) -> float:
    gh = _GridHolder(s)
    rp = _f64(s.fields[0] if rho_p is None else rho_p)
    return lib().or_mass(gh.ref, _ptr(rp))


def energy(s, fields=None, grav: float = GRAV) -> float:
    gh = _GridHolder(s, grav)
    f = [_f64(x) for x in (s.fields if fields is None else fields)]
    return lib().or_energy(gh.ref, _ptr_array(f))


def diffuse(q, kx, ky, kz, steps: int = 1) -> np.ndarray:
    """`steps` seven-point diffusion steps of q (shape (nz, ny, nx))."""
    cur = _f64(q).copy()
    nz, ny, nx = cur.shape
    nxt = np.empty_like(cur)
    for _ in range(steps):
        rc = lib().or_diffuse(nx, ny, nz, float(kx), float(ky), float(kz), _ptr(cur), _ptr(nxt))
        if rc != OK:
            raise RuntimeError(rc)
        cur, nxt = nxt, cur
    return cur


def damp(s, fields, dtau: float, t: float) -> List[np.ndarray]:
    """The damping of one short step's end (state s must carry ``damping``)."""
    gh = _GridHolder(s)
    f = [_f64(x).copy() for x in fields]
    rc = lib().or_damp(gh.ref, _ptr_array(f), float(dtau), float(t))
    if rc != OK:
        raise RuntimeError(rc)
    return f
