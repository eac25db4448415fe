"""GPU test of hv_mass_noalloc, the allocation-free variant of hv_mass: its
sums go through the library's static device scratch instead of the grid's
workspace and land in caller-owned device memory without a synchronisation.

Both entry points run the same kernels in the same fixed order on the same
state, so the values must be bitwise equal.  Two grids in a row, the second
smaller (fewer partial sums, the rest of the scratch holds stale values of
the first), in two precisions; the first grid is then read again to show
that a call does not depend on what an earlier one left in the scratch.
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


def _both(hv, d):
    import torch
    want = d.mass(energy=True)
    out = torch.full((2,), float("nan"), dtype=torch.float64, device=d.workspace.device)
    d.mass_noalloc(out)
    d.stream.synchronize()
    got = tuple(out.cpu().numpy().tolist())
    return want, got


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_sums_equal_hv_mass_on_two_grids(hv, prec):
    big = inputs.make_state(96, 80, 64, seed=31, noise=0.4, n_short=4)
    small = inputs.make_state(20, 12, 32, seed=32, noise=0.4, n_short=4)
    print(f"case: noalloc {prec} 96x80x64 then 20x12x32", flush=True)
    d1 = hv.Domain(big, precision=prec)
    d1.step(big.dt, 2, big.n_short)
    w1, g1 = _both(hv, d1)
    d2 = hv.Domain(small, precision=prec)
    d2.step(small.dt, 1, small.n_short)
    w2, g2 = _both(hv, d2)
    assert np.isfinite(w1).all() and np.isfinite(w2).all()
    assert g1 == w1, (g1, w1)
    assert g2 == w2, (g2, w2)
    # the first grid again, after the smaller one overwrote part of the scratch
    w1b, g1b = _both(hv, d1)
    assert g1b == w1b == w1
    d1.close()
    d2.close()


def test_noalloc_rejects_bad_arguments(hv):
    import torch
    s = inputs.make_state(16, 16, 32, seed=33, n_short=4)
    d = hv.Domain(s, precision="fp32", init=False)
    out = torch.zeros(2, dtype=torch.float64, device=d.workspace.device)
    with pytest.raises(hv.HvError) as ei:
        d.mass_noalloc(out)
    assert ei.value.code == hv.HV_ERR_STATE
    L = hv.load()
    assert L.hv_mass_noalloc(None, None) == hv.HV_ERR_ARG
    assert L.hv_mass_noalloc(d.handle, None) == hv.HV_ERR_ARG
    d.close()
