"""GPU edge cases of the step: the smallest grids the stencils allow (4
columns along an axis, so the 5-point Koren stencil wraps onto itself), one
short step per stage, zero long steps, and a wind that reverses with height.

Parity bar: float64 within 1e-11 of the field range of the FP64 oracle, as in
the other parity tests.
"""
import numpy as np
import pytest

from paper_1710_08616_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_08616_amd import hevi
    hevi.load()
    return hevi


def _rel(a, b):
    r = np.ptp(b)
    return np.abs(a - b).max() / (r if r > 0 else 1.0)


def _run(hv, s, prec, n_long, n_short, layout="kij"):
    d = hv.Domain(s, precision=prec, layout=layout)
    d.step(s.dt, n_long, n_short)
    out = d.read_all()
    d.close()
    return out


@pytest.mark.parametrize("nx,ny,nz,layout", [(4, 4, 32, "kij"), (4, 7, 64, "ijk"),
                                              (9, 4, 128, "kij"), (5, 5, 32, "ijk")])
def test_smallest_grids_match_oracle(hv, oracle, nx, ny, nz, layout):
    s = inputs.make_state(nx, ny, nz, seed=nx * ny + nz, noise=0.8, u_bg=7.0, v_bg=-3.0,
                          bubbles=[(nx * 1000.0, ny * 1000.0, 4000.0, 3000.0)], n_short=3)
    print(f"case: minimum grid {nx}x{ny}x{nz} {layout} fp64", flush=True)
    ref = oracle.step(s, n_long=3, n_short=3)
    got = _run(hv, s, "fp64", 3, 3, layout)
    for name, a, b in zip(inputs.FIELD_NAMES, got, ref):
        assert _rel(a, b) <= 1e-11, (name, _rel(a, b))


def test_smallest_terrain_grid_matches_oracle(hv, oracle):
    h = inputs.orography(4, 5, 2000.0, 2000.0, 3, hmax=400.0, hills=1, smin=3000.0, smax=5000.0)
    s = inputs.make_state(4, 5, 32, seed=8, terrain=h, u_bg=4.0, shear=10.0, noise=0.5, n_short=2)
    print("case: minimum terrain grid 4x5x32 fp64", flush=True)
    ref = oracle.step(s, n_long=2, n_short=2)
    got = _run(hv, s, "fp64", 2, 2)
    for name, a, b in zip(inputs.FIELD_NAMES, got, ref):
        assert _rel(a, b) <= 1e-11, (name, _rel(a, b))


@pytest.mark.parametrize("short", ["fb", "rk2"])
def test_one_short_step_per_stage_matches_oracle(hv, oracle, short):
    s = inputs.make_state(24, 20, 64, seed=55, noise=0.5, u_bg=12.0, n_short=1, dt=4.0)
    print(f"case: n_short = 1 ({short}) fp64", flush=True)
    ref = oracle.step(s, n_long=4, n_short=1, short_rk2=(short == "rk2"))
    d = hv.Domain(s, precision="fp64", short=short)
    d.step(s.dt, 4, 1)
    got = d.read_all()
    d.close()
    for name, a, b in zip(inputs.FIELD_NAMES, got, ref):
        assert _rel(a, b) <= 1e-11, (name, _rel(a, b))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_zero_long_steps_leave_the_state(hv, prec):
    s = inputs.make_state(20, 13, 32, seed=4, noise=0.5)
    print(f"case: n_long = 0 {prec}", flush=True)
    d = hv.Domain(s, precision=prec)
    before = d.read_all()
    d.step(s.dt, 0, 4)
    after = d.read_all()
    d.close()
    for name, a, b in zip(inputs.FIELD_NAMES, before, after):
        assert np.array_equal(a, b), name
    if prec == "fp64":
        for name, a, b in zip(inputs.FIELD_NAMES, before, s.fields):
            assert np.array_equal(a, b), name


def test_wind_reversing_with_height_matches_oracle(hv, oracle):
    """The x-faces of every column see both upwind directions: the zonal wind
    is -15 m/s at the ground and +15 m/s at the lid (shear 30 m/s over the
    depth), so the sign-symmetric face form is taken on both branches."""
    s = inputs.make_state(16, 12, 64, seed=90, u_bg=-15.0, v_bg=-15.0, shear=30.0, noise=0.3,
                          n_short=4)
    print("case: wind reversal fp64", flush=True)
    ref = oracle.step(s, n_long=3)
    got = _run(hv, s, "fp64", 3, s.n_short)
    for name, a, b in zip(inputs.FIELD_NAMES, got, ref):
        assert _rel(a, b) <= 1e-11, (name, _rel(a, b))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_unstable_run_reports_a_non_finite_mass(hv, prec):
    """Failure detection: a short step far beyond the acoustic limit (c dtau /
    dx ~ 100 with one short step per stage; the oracle refuses the first
    column system, which is no longer diagonally dominant) grows by orders of
    magnitude per long step and overflows well within 200 of them, in float64
    too; the kernels keep running on the non-finite values, and hv_mass
    reports HV_ERR_NONFINITE instead of a number."""
    s = inputs.make_state(16, 16, 32, seed=77, noise=0.5, u_bg=5.0, n_short=1, dt=600.0)
    print(f"case: unstable run {prec}", flush=True)
    d = hv.Domain(s, precision=prec)
    d.step(s.dt, 200, 1)
    with pytest.raises(hv.HvError) as e:
        d.mass()
    assert e.value.code == hv.HV_ERR_NONFINITE
    d.close()
