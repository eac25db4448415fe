"""GPU parity of the float64 energy diagnostic (hv_mass's second output)
against the oracle's energy of the same state read back from the device.

The device sums the stored fields converted to float64, so the two agree up
to summation order (1e-12 relative), except that over terrain the reduced-
precision paths keep the 3D reference fields in binary32 (about 1e-7).
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


def _state(terrain):
    nx, ny, nz = 24, 20, 64
    h = None
    if terrain:
        h = inputs.orography(nx, ny, 2000.0, 2000.0, 17, hmax=1500.0, hills=2, smin=4000.0,
                             smax=8000.0)
    return inputs.make_state(nx, ny, nz, seed=19, terrain=h, u_bg=9.0, v_bg=-5.0, shear=10.0,
                             noise=0.6, n_short=4)


@pytest.mark.parametrize("terrain,prec,tol", [(False, "fp64", 1e-12), (True, "fp64", 1e-12),
                                              (False, "fp32", 1e-12), (False, "mixed", 1e-12),
                                              (True, "mixed", 1e-6)])
def test_energy_matches_oracle_on_the_device_state(hv, oracle, terrain, prec, tol):
    s = _state(terrain)
    print(f"case: energy terrain={terrain} {prec}", flush=True)
    d = hv.Domain(s, precision=prec)
    d.step(s.dt, 2, s.n_short)
    m, e = d.mass(energy=True)
    s2 = s.copy()
    s2.fields = d.read_all()
    d.close()
    want = oracle.energy(s2)
    assert np.isfinite(e)
    assert abs(e / want - 1.0) <= tol, (e, want)
    assert abs(m / oracle.mass(s2) - 1.0) <= 1e-13
