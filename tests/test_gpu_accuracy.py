"""Reduced-precision accuracy on the oracle-sized sub-runs of the two large
single-domain workloads, against per-field bars frozen in
tests/golden/twin_tolerances.json (written by make_twin_tolerances.py beside
it from the oracle alone):

- 128x128x64, 16 bubbles, u = 10 m/s, 100 long steps, n = 6 (the sub-run of
  the 1024x1024x64 workload): float32 and mixed;
- 160x128x64 over Gaussian hills with shear 0-30 m/s, 50 long steps, n = 6
  (the sub-run of the 1600x1280x64 workload): mixed and float64.

The bar of a reduced-precision path is, per field and separately for the max
and the RMS of (gpu - oracle) / range(oracle), 10x the divergence of the
oracle's binary32-storage twin (a float64 run from fl32 of the initial state
and of the reference state that rounds every stored field, slow array and
Runge-Kutta intermediate to binary32 after each sweep).  The float64 path
matches the oracle within 1e-11 of the range.  Mass: the total drifts by at
most 1e-11 of itself in float32 / mixed (binary32 storage of rho') and
1e-13 in float64 over the whole run.
"""
import json
import os

import numpy as np
import pytest

from paper_1710_08616_amd import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = json.load(open(os.path.join(HERE, "golden", "twin_tolerances.json")))["cases"]


@pytest.fixture(scope="module")
def hv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_08616_amd import hevi
    hevi.load()
    return hevi


_REF = {}


def _ref(oracle, case):
    if case not in _REF:
        s = inputs.workload(case)
        print(f"oracle: {case} {s.nx}x{s.ny}x{s.nz}, {s.n_long} long steps", flush=True)
        _REF[case] = (s, oracle.step(s))
    return _REF[case]


def _errors(got, ref):
    out = {}
    for name, a, b in zip(inputs.FIELD_NAMES, got, ref):
        rng = float(np.ptp(b)) or 1.0
        d = a - b
        out[name] = (float(np.abs(d).max()) / rng, float(np.sqrt(np.mean(d * d))) / rng)
    return out


@pytest.mark.parametrize("case,prec", [("large_sub", "fp32"), ("large_sub", "mixed"),
                                       ("terrain_sub", "mixed"), ("terrain_sub", "fp64")])
def test_sub_run_within_frozen_per_field_tolerance(hv, oracle, case, prec):
    s, ref = _ref(oracle, case)
    print(f"case: accuracy {case} {prec}", flush=True)
    d = hv.Domain(s, precision=prec)
    m0 = d.mass()
    d.step(s.dt, s.n_long, s.n_short)
    got = d.read_all()
    m1 = d.mass()
    d.close()
    err = _errors(got, ref)
    tol = TOL[case]["tolerance"]
    for name, (mx, rms) in err.items():
        print(f"  {name}: max {mx:.3e} rms {rms:.3e}", flush=True)
        if prec == "fp64":
            assert mx <= 1e-11, (name, mx)
        else:
            assert mx <= tol[name]["max_rel"], (name, "max", mx, tol[name]["max_rel"])
            assert rms <= tol[name]["rms_rel"], (name, "rms", rms, tol[name]["rms_rel"])
    assert abs(m1 - m0) <= (1e-13 if prec == "fp64" else 1e-11) * m0, (m0, m1)
