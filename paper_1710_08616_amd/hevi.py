"""Python binding of libhevi.so (the C ABI in include/hevi.h).

Argument marshalling only: every step of the time integration runs in the
HIP kernels of the library.  PyTorch supplies the device workspace (one
uint8 tensor owned by the Domain) and the stream handle.  If the library is
not built this module raises on first use; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhevi.so")

HV_OK, HV_ERR_ARG, HV_ERR_HIP, HV_ERR_STATE, HV_ERR_NONFINITE, HV_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
HV_ERR_DRIFT = -6
FP64, FP32, MIXED = 0, 1, 2
IJK, KIJ = 0, 1
RHO_PTB, RHOU, RHOV, RHOW, RHOTHETA_PTB = 0, 1, 2, 3, 4

PRECISIONS = {"fp64": FP64, "fp32": FP32, "mixed": MIXED}
LAYOUTS = {"ijk": IJK, "kij": KIJ}
SHORT_FB, SHORT_RK2 = 0, 1
SHORT_SCHEMES = {"fb": SHORT_FB, "rk2": SHORT_RK2}

EXPORTS = ("hv_workspace_bytes", "hv_grid_create", "hv_state_init", "hv_step", "hv_state_read",
           "hv_mass", "hv_tune", "hv_trace", "hv_trace_read", "hv_grid_destroy", "hv_last_error",
           "hv_ens_workspace_bytes", "hv_ens_create", "hv_ens_state_init", "hv_ens_step",
           "hv_ens_state_read", "hv_ens_mass", "hv_ens_tune", "hv_ens_trace", "hv_ens_trace_read",
           "hv_ens_destroy", "hv_ens_last_error", "hv_diffuse", "hv_damping", "hv_ens_damping", "hv_mass_noalloc", "hv_configure",
           "hv_ens_configure")
K_SLOW_PREP, K_SLOW_FLUX, K_SHORT_STEP, K_MASS = 0, 1, 2, 3
KERNEL_KINDS = {"slow_prep": K_SLOW_PREP, "slow_flux": K_SLOW_FLUX, "short_step": K_SHORT_STEP,
                "mass": K_MASS}

_dp = ctypes.POINTER(ctypes.c_double)


class HvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hevi error {code}: {msg}")
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("zeta_faces", _dp), ("terrain", _dp),
                ("precision", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("beta", ctypes.c_double), ("div_damp", ctypes.c_double),
                ("short_scheme", ctypes.c_int32), ("damping", ctypes.c_int32),
                ("mass_drift_bound", ctypes.c_double)]


_lib = None


def load():
    """Load libhevi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(or python -m paper_1710_08616_amd.build_lib)")
    # torch first: its HIP runtime (same soname) is then the one the library
    # binds to, so workspace, streams and kernels share one runtime
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.hv_workspace_bytes.restype = ctypes.c_size_t
    L.hv_workspace_bytes.argtypes = [ctypes.POINTER(GridDesc)]
    L.hv_grid_create.restype = ctypes.c_int
    L.hv_grid_create.argtypes = [ctypes.POINTER(GridDesc), ctypes.c_void_p, ctypes.c_size_t,
                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    L.hv_state_init.restype = ctypes.c_int
    L.hv_state_init.argtypes = [ctypes.c_void_p, ctypes.POINTER(_dp), _dp, _dp, _dp]
    L.hv_step.restype = ctypes.c_int
    L.hv_step.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int32]
    L.hv_state_read.restype = ctypes.c_int
    L.hv_state_read.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp]
    L.hv_mass.restype = ctypes.c_int
    L.hv_mass.argtypes = [ctypes.c_void_p, _dp, _dp]
    L.hv_mass_noalloc.restype = ctypes.c_int
    L.hv_mass_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.hv_trace.restype = ctypes.c_int
    L.hv_trace.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.hv_trace_read.restype = ctypes.c_int
    L.hv_trace_read.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp,
                                ctypes.POINTER(ctypes.c_int64)]
    _ip = ctypes.POINTER(ctypes.c_int32)
    L.hv_tune.restype = ctypes.c_int
    L.hv_tune.argtypes = [ctypes.c_void_p, _ip, _ip]
    L.hv_configure.restype = ctypes.c_int
    L.hv_configure.argtypes = [ctypes.c_void_p, _ip, _ip, _ip, _ip]
    L.hv_ens_configure.restype = ctypes.c_int
    L.hv_ens_configure.argtypes = [ctypes.c_void_p, ctypes.c_int32, _ip, _ip, _ip, _ip, _ip]
    L.hv_ens_workspace_bytes.restype = ctypes.c_size_t
    L.hv_ens_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.POINTER(GridDesc)]
    L.hv_ens_create.restype = ctypes.c_int
    L.hv_ens_create.argtypes = [ctypes.c_int32, ctypes.POINTER(GridDesc), ctypes.c_void_p,
                                ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    L.hv_ens_state_init.restype = ctypes.c_int
    L.hv_ens_state_init.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(_dp), _dp, _dp,
                                    _dp]
    L.hv_ens_step.restype = ctypes.c_int
    L.hv_ens_step.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int32, ctypes.c_int32]
    L.hv_ens_state_read.restype = ctypes.c_int
    L.hv_ens_state_read.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, _dp]
    L.hv_ens_mass.restype = ctypes.c_int
    L.hv_ens_mass.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp, _dp]
    L.hv_ens_tune.restype = ctypes.c_int
    L.hv_ens_tune.argtypes = [ctypes.c_void_p, _ip, _ip, _ip]
    L.hv_ens_trace.restype = ctypes.c_int
    L.hv_ens_trace.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.hv_ens_trace_read.restype = ctypes.c_int
    L.hv_ens_trace_read.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp,
                                    ctypes.POINTER(ctypes.c_int64)]
    L.hv_ens_destroy.restype = None
    L.hv_ens_destroy.argtypes = [ctypes.c_void_p]
    L.hv_ens_last_error.restype = ctypes.c_char_p
    L.hv_ens_last_error.argtypes = [ctypes.c_void_p]
    L.hv_damping.restype = ctypes.c_int
    L.hv_damping.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.POINTER(_dp), ctypes.POINTER(_dp),
                             ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.hv_ens_damping.restype = ctypes.c_int
    L.hv_ens_damping.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp, _dp, ctypes.POINTER(_dp),
                                 ctypes.POINTER(_dp), ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double]
    L.hv_diffuse.restype = ctypes.c_int
    L.hv_diffuse.argtypes = [ctypes.c_int32] * 5 + [ctypes.c_double] * 3 + [
        ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.hv_grid_destroy.restype = None
    L.hv_grid_destroy.argtypes = [ctypes.c_void_p]
    L.hv_last_error.restype = ctypes.c_char_p
    L.hv_last_error.argtypes = [ctypes.c_void_p]
    _lib = L
    return L


def make_desc(nx, ny, nz, dx, dy, zf, precision="fp32", layout="kij", beta=0.55, terrain=None,
              short="fb", damping=False, drift_bound=0.0):
    """A filled hv_grid_desc plus the arrays it points into (keep them alive
    until the grid is created).  terrain: (ny, nx) surface heights or None;
    short: "fb" (forward-backward) or "rk2" (two-stage Runge-Kutta) short step;
    damping: reserve workspace for lateral / upper damping data; drift_bound: the
    relative mass drift bound of the failure check (0: library default, < 0: off)."""
    zf = np.ascontiguousarray(zf, dtype=np.float64)
    keep = [zf]
    tp = None
    if terrain is not None:
        t = np.ascontiguousarray(terrain, dtype=np.float64)
        if t.shape != (int(ny), int(nx)):
            raise ValueError(f"terrain must have shape (ny, nx) = ({ny}, {nx})")
        keep.append(t)
        tp = t.ctypes.data_as(_dp)
    d = GridDesc(int(nx), int(ny), int(nz), float(dx), float(dy),
                 zf.ctypes.data_as(_dp), tp,
                 PRECISIONS[precision] if isinstance(precision, str) else int(precision),
                 LAYOUTS[layout] if isinstance(layout, str) else int(layout),
                 float(beta), 0.0, SHORT_SCHEMES[short] if isinstance(short, str) else int(short),
                 1 if damping else 0, float(drift_bound))
    return d, keep


def _damping_args(d):
    """Marshal a damping dict (nu_lat, nu_top, bnd1, bnd2, t1, t2) for the ABI."""
    keep = [np.ascontiguousarray(d["nu_lat"], dtype=np.float64),
            np.ascontiguousarray(d["nu_top"], dtype=np.float64)]
    b1 = [np.ascontiguousarray(x, dtype=np.float64) for x in d["bnd1"]]
    b2 = [np.ascontiguousarray(x, dtype=np.float64) for x in d["bnd2"]]
    keep += b1 + b2
    p1 = (_dp * 5)(*[x.ctypes.data_as(_dp) for x in b1])
    p2 = (_dp * 5)(*[x.ctypes.data_as(_dp) for x in b2])
    return keep, [keep[0].ctypes.data_as(_dp), keep[1].ctypes.data_as(_dp), p1, p2,
                  float(d["t1"]), float(d["t2"])]


def workspace_bytes(desc: GridDesc) -> int:
    return int(load().hv_workspace_bytes(ctypes.byref(desc)))


def last_error(handle=None) -> str:
    return load().hv_last_error(handle).decode()


class Domain:
    """One grid on the GPU: workspace, state, stepping and read-back.

    ``state`` is any object with nx, ny, nz, dx, dy, zf, beta attributes, an
    optional ``terrain`` ((ny, nx) surface heights), and rho_ref, rt_ref,
    p_ref, fields when it is also used to initialise (reference columns of nz
    values on flat ground, per-cell (nz, ny, nx) arrays over terrain).
    """

    def __init__(self, state, precision="fp32", layout="kij", device="cuda", stream=None,
                 init=True, short="fb", drift_bound=0.0):
        import torch
        self._torch = torch
        L = load()
        self.nx, self.ny, self.nz = int(state.nx), int(state.ny), int(state.nz)
        dmp = getattr(state, "damping", None)
        self.desc, self._keep = make_desc(state.nx, state.ny, state.nz, state.dx, state.dy,
                                          state.zf, precision, layout, getattr(state, "beta", 0.55),
                                          getattr(state, "terrain", None), short, dmp is not None,
                                          drift_bound)
        nbytes = workspace_bytes(self.desc)
        if nbytes == 0:
            raise HvError(HV_ERR_ARG, last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        h = ctypes.c_void_p()
        rc = L.hv_grid_create(ctypes.byref(self.desc), ctypes.c_void_p(self.workspace.data_ptr()),
                              nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != HV_OK:
            raise HvError(rc, last_error())
        self.handle = h
        if init:
            self.init(state.fields, state.rho_ref, state.rt_ref, state.p_ref)
            if dmp is not None:
                self.set_damping(dmp)

    # -- ABI wrappers -------------------------------------------------------
    def set_damping(self, d, time_now: float = 0.0):
        """hv_damping with a dict of nu_lat, nu_top, bnd1, bnd2, t1, t2."""
        keep, args = _damping_args(d)
        return self._check(load().hv_damping(self.handle, *args, float(time_now)))

    def _check(self, rc):
        if rc != HV_OK:
            raise HvError(rc, last_error(self.handle))
        return rc

    def init(self, fields: Sequence[np.ndarray], rho_ref, rt_ref, p_ref):
        arrs = [np.ascontiguousarray(f, dtype=np.float64) for f in fields]
        ptrs = (_dp * 5)(*[a.ctypes.data_as(_dp) for a in arrs])
        refs = [np.ascontiguousarray(r, dtype=np.float64) for r in (rho_ref, rt_ref, p_ref)]
        return self._check(load().hv_state_init(self.handle, ptrs,
                                                *[r.ctypes.data_as(_dp) for r in refs]))

    def step(self, dt: float, n_long: int, n_short: int):
        return self._check(load().hv_step(self.handle, float(dt), int(n_long), int(n_short)))

    def read(self, field: int) -> np.ndarray:
        nzf = self.nz + 1 if field == RHOW else self.nz
        out = np.empty((nzf, self.ny, self.nx), dtype=np.float64)
        self._check(load().hv_state_read(self.handle, int(field), out.ctypes.data_as(_dp)))
        return out

    def read_all(self):
        return [self.read(f) for f in range(5)]

    def mass(self, energy: bool = False):
        m = ctypes.c_double()
        e = ctypes.c_double()
        self._check(load().hv_mass(self.handle, ctypes.byref(m),
                                   ctypes.byref(e) if energy else None))
        return (m.value, e.value) if energy else m.value

    def mass_noalloc(self, dev_out):
        """hv_mass_noalloc: enqueue the mass and energy sums of the current state
        into dev_out (a device float64 tensor of at least 2 values) on the grid's
        stream; nothing is allocated and nothing waits."""
        import torch
        if dev_out.dtype != torch.float64 or dev_out.numel() < 2 or not dev_out.is_cuda:
            raise ValueError("dev_out must be a device float64 tensor of >= 2 values")
        return self._check(load().hv_mass_noalloc(self.handle, ctypes.c_void_p(dev_out.data_ptr())))

    def tune(self):
        """Autotune the launch configurations; returns the chosen tile x-extent
        per kernel kind (slow prep, slow flux, short step), negative where the
        XCD-chunked block order won, and the lanes per column of each kind."""
        out = (ctypes.c_int32 * 3)()
        lanes = (ctypes.c_int32 * 3)()
        self._check(load().hv_tune(self.handle, out, lanes))
        return list(out), list(lanes)

    def configure(self, config=None):
        """hv_configure: set (config = 3 indices) and/or report the launch
        configurations in force, as (indices, tile x-extents, lanes per column)."""
        idx = (ctypes.c_int32 * 3)()
        out = (ctypes.c_int32 * 3)()
        lanes = (ctypes.c_int32 * 3)()
        cfg = None if config is None else (ctypes.c_int32 * 3)(*[int(c) for c in config])
        self._check(load().hv_configure(self.handle, cfg, idx, out, lanes))
        return list(idx), list(out), list(lanes)

    def pin_default_short_width(self):
        """Keep the tuned tiles and block orders but the short step's default
        lanes per column (whose column solve rounds like an untuned run)."""
        idx, _t, _l = self.configure()
        self.configure([idx[0], idx[1], idx[2] % 6])

    def trace(self, on: bool):
        return self._check(load().hv_trace(self.handle, 1 if on else 0))

    def trace_read(self):
        """{kind: (total ms, launches)} of the kernels recorded since trace(True)."""
        out = {}
        for name, kind in KERNEL_KINDS.items():
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            self._check(load().hv_trace_read(self.handle, kind, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def close(self):
        if getattr(self, "handle", None):
            load().hv_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptrs5(fields):
    arrs = [np.ascontiguousarray(f, dtype=np.float64) for f in fields]
    return arrs, (_dp * 5)(*[a.ctypes.data_as(_dp) for a in arrs])


class Ensemble:
    """Independent domains of uneven sizes advanced together (hv_ens_*).

    ``states``: sequence of objects like the ones Domain takes.  All members
    share precision and layout; each keeps its own dt (``state.dt``).
    """

    def __init__(self, states, precision="fp32", layout="kij", device="cuda", stream=None,
                 init=True, short="fb"):
        import torch
        L = load()
        self.n = len(states)
        self.shapes = [(int(s.nz), int(s.ny), int(s.nx)) for s in states]
        self._keep = []
        descs = (GridDesc * self.n)()
        for q, s in enumerate(states):
            d, keep = make_desc(s.nx, s.ny, s.nz, s.dx, s.dy, s.zf, precision, layout,
                                getattr(s, "beta", 0.55), getattr(s, "terrain", None), short,
                                getattr(s, "damping", None) is not None)
            descs[q] = d
            self._keep.append(keep)
        self._descs = descs
        nbytes = int(L.hv_ens_workspace_bytes(self.n, descs))
        if nbytes == 0:
            raise HvError(HV_ERR_ARG, L.hv_ens_last_error(None).decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        h = ctypes.c_void_p()
        rc = L.hv_ens_create(self.n, descs, ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != HV_OK:
            raise HvError(rc, L.hv_ens_last_error(None).decode())
        self.handle = h
        self.dts = np.array([float(getattr(s, "dt", 10.0)) for s in states])
        if init:
            for q, s in enumerate(states):
                self.init(q, s.fields, s.rho_ref, s.rt_ref, s.p_ref)
                if getattr(s, "damping", None) is not None:
                    self.set_damping(q, s.damping)

    def set_damping(self, member, d, time_now: float = 0.0):
        keep, args = _damping_args(d)
        return self._check(load().hv_ens_damping(self.handle, int(member), *args,
                                                 float(time_now)))

    def _check(self, rc):
        if rc != HV_OK:
            raise HvError(rc, load().hv_ens_last_error(self.handle).decode())
        return rc

    def init(self, member, fields, rho_ref, rt_ref, p_ref):
        keep, ptrs = _ptrs5(fields)
        refs = [np.ascontiguousarray(r, dtype=np.float64) for r in (rho_ref, rt_ref, p_ref)]
        return self._check(load().hv_ens_state_init(self.handle, int(member), ptrs,
                                                    *[r.ctypes.data_as(_dp) for r in refs]))

    def step(self, n_long: int, n_short: int, dts=None):
        d = np.ascontiguousarray(self.dts if dts is None else dts, dtype=np.float64)
        return self._check(load().hv_ens_step(self.handle, d.ctypes.data_as(_dp), int(n_long),
                                              int(n_short)))

    def read(self, member: int, field: int) -> np.ndarray:
        nz, ny, nx = self.shapes[member]
        out = np.empty((nz + 1 if field == RHOW else nz, ny, nx), dtype=np.float64)
        self._check(load().hv_ens_state_read(self.handle, int(member), int(field),
                                             out.ctypes.data_as(_dp)))
        return out

    def read_all(self, member: int):
        return [self.read(member, f) for f in range(5)]

    def mass(self, member: int, energy: bool = False):
        m = ctypes.c_double()
        e = ctypes.c_double()
        self._check(load().hv_ens_mass(self.handle, int(member), ctypes.byref(m),
                                       ctypes.byref(e) if energy else None))
        return (m.value, e.value) if energy else m.value

    def tune(self):
        """Autotune per launch group; returns per group (at most 6: flat and
        terrain, nz = 32, 64, 128) the [prep, flux, short] tile x-extents and
        lanes per column."""
        out = (ctypes.c_int32 * (3 * 6))()
        lanes = (ctypes.c_int32 * (3 * 6))()
        ng = ctypes.c_int32()
        self._check(load().hv_ens_tune(self.handle, out, lanes, ctypes.byref(ng)))
        return [(list(out[3 * g:3 * g + 3]), list(lanes[3 * g:3 * g + 3])) for g in range(ng.value)]

    def configure(self, group=0, config=None):
        """hv_ens_configure for one launch group; returns every group's
        (indices, tile x-extents, lanes per column)."""
        idx = (ctypes.c_int32 * (3 * 6))()
        out = (ctypes.c_int32 * (3 * 6))()
        lanes = (ctypes.c_int32 * (3 * 6))()
        ng = ctypes.c_int32()
        cfg = None if config is None else (ctypes.c_int32 * 3)(*[int(c) for c in config])
        self._check(load().hv_ens_configure(self.handle, int(group), cfg, idx, out, lanes,
                                            ctypes.byref(ng)))
        return [(list(idx[3 * g:3 * g + 3]), list(out[3 * g:3 * g + 3]), list(lanes[3 * g:3 * g + 3]))
                for g in range(ng.value)]

    def pin_default_short_width(self):
        """Keep every group's tuned tiles and block orders but the short
        step's default lanes per column (whose column solve rounds like an
        untuned run)."""
        for g, (idx, _t, _l) in enumerate(self.configure()):
            self.configure(g, [idx[0], idx[1], idx[2] % 6])

    def trace(self, on: bool):
        return self._check(load().hv_ens_trace(self.handle, 1 if on else 0))

    def trace_read(self):
        out = {}
        for name, kind in KERNEL_KINDS.items():
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            self._check(load().hv_ens_trace_read(self.handle, kind, ctypes.byref(ms),
                                                 ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def close(self):
        if getattr(self, "handle", None):
            load().hv_ens_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def diffuse(q_in, q_out, kx: float, ky: float, kz: float, layout="kij", tile_x: int = 16,
            stream=None):
    """One seven-point diffusion step (hv_diffuse) from device tensor q_in into
    q_out (same shape and dtype, float32 or float64).  Shapes: (ny, nx, nz)
    for the column-fastest layout, (nz, ny, nx) for the i-fastest one."""
    import torch
    if q_in.dtype != q_out.dtype or q_in.shape != q_out.shape:
        raise ValueError("q_in and q_out must match")
    if not (q_in.is_contiguous() and q_out.is_contiguous()):
        raise ValueError("tensors must be contiguous")
    lay = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
    if lay == KIJ:
        ny, nx, nz = q_in.shape
    else:
        nz, ny, nx = q_in.shape
    prec = {torch.float64: FP64, torch.float32: FP32}.get(q_in.dtype)
    if prec is None:
        raise ValueError("dtype must be float32 or float64")
    s = stream if stream is not None else torch.cuda.current_stream(q_in.device)
    rc = load().hv_diffuse(nx, ny, nz, prec, lay, float(kx), float(ky), float(kz), int(tile_x),
                           ctypes.c_void_p(q_in.data_ptr()), ctypes.c_void_p(q_out.data_ptr()),
                           ctypes.c_void_p(s.cuda_stream))
    if rc != HV_OK:
        raise HvError(rc, last_error())
    return q_out
