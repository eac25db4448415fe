"""Invariants the full oracle step must keep, each fixed by the scheme's
mathematics rather than by the oracle's own code.

- rest stays exactly at rest (p' = 0 exactly when Theta' = 0),
- a horizontally uniform flow over flat ground is bitwise steady,
- total mass is conserved (flux form, periodic sides, rigid lids),
- a uniform potential temperature stays uniform under any flow,
- a column in discrete hydrostatic balance stays at rest,
- a warm bubble is buoyant (rises),
- results do not depend on the OpenMP thread count.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1710_08616_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_rest_state_stays_exactly_zero(oracle):
    s = inputs.rest_state(8, 6, 16, n_short=4)
    out = oracle.step(s, dt=10.0, n_long=3, n_short=4)
    for f in out:
        assert np.all(f == 0.0)


def test_uniform_flow_is_bitwise_steady(oracle):
    nx, ny, nz = 8, 5, 12
    s = inputs.rest_state(nx, ny, nz)
    s.fields[1][:] = (s.rho_ref * 10.0)[:, None, None]
    s.fields[2][:] = (s.rho_ref * -3.0)[:, None, None]
    out = oracle.step(s, dt=10.0, n_long=3, n_short=4)
    for f0, f1 in zip(s.fields, out):
        assert np.array_equal(f0, f1)


def test_mass_is_conserved_per_long_step(oracle):
    s = inputs.workload("small")
    m0 = oracle.mass(s)
    dz = np.diff(s.zf)[:, None, None]
    pm0 = (s.fields[0] * dz).sum()
    scale = (np.abs(s.fields[0]) * dz).sum()
    f = s.fields
    for _ in range(3):
        s.fields = f
        f = oracle.step(s, n_long=1)
        s2 = s.copy()
        s2.fields = f
        m1 = oracle.mass(s2)
        assert abs(m1 - m0) <= 1e-14 * m0
        # the perturbation mass itself is conserved to rounding of the increments
        assert abs((f[0] * dz).sum() - pm0) <= 1e-12 * scale
    assert not np.allclose(f[0], inputs.workload("small").fields[0])


def test_uniform_theta_is_preserved(oracle):
    """Neutral reference (theta = 300 K everywhere) with divergent noise:
    Theta and rho are advected by the same mass fluxes, so theta stays 300 K."""
    nx, ny, nz = 16, 12, 16
    s = inputs.make_state(nx, ny, nz, seed=21, bubbles=[], noise=2.0, u_bg=5.0,
                          reference="neutral", n_short=4)
    theta0 = s.rt_ref[0] / s.rho_ref[0]
    out = oracle.step(s, dt=10.0, n_long=10, n_short=4)
    rho = s.rho_ref[:, None, None] + out[0]
    th = (s.rt_ref[:, None, None] + out[4]) / rho
    assert np.abs(out[0]).max() > 1e-6            # the flow really moved mass around
    assert np.max(np.abs(th / theta0 - 1.0)) <= 1e-13


def test_discrete_hydrostatic_balance_stays_at_rest(oracle):
    """A horizontally uniform Theta' with rho' chosen so that
    (p'_k - p'_{k-1}) / dzf_k = -g (a_k rho'_k + b_k rho'_{k-1})
    (linear interpolation of rho' to level faces) is a steady state."""
    nx, ny, nz = 4, 3, 16
    s = inputs.rest_state(nx, ny, nz)
    zf = s.zf
    dz = np.diff(zf)
    zc = inputs.centres(zf)
    tp = 0.8 * np.sin(zc / 3000.0)
    pp = s.p_ref * np.expm1(1.4 * np.log1p(tp / s.rt_ref))
    rp = np.zeros(nz)
    rp[0] = -2e-3
    for k in range(1, nz):
        dzf = zc[k] - zc[k - 1]
        a = dz[k - 1] / (dz[k - 1] + dz[k])
        b = dz[k] / (dz[k - 1] + dz[k])
        rp[k] = (-(pp[k] - pp[k - 1]) / (inputs.GRAV * dzf) - b * rp[k - 1]) / a
    s.fields[0][:] = rp[:, None, None]
    s.fields[4][:] = tp[:, None, None]
    out = oracle.step(s, dt=10.0, n_long=2, n_short=4)
    assert np.abs(out[3]).max() <= 1e-10
    assert np.abs(out[1]).max() <= 1e-10 and np.abs(out[2]).max() <= 1e-10
    assert np.max(np.abs(out[0] - s.fields[0])) <= 1e-12 * np.abs(rp).max()
    assert np.max(np.abs(out[4] - s.fields[4])) <= 1e-12 * np.abs(tp).max()
    # the same Theta' without its balancing rho' is not steady
    s.fields[0][:] = 0.0
    out = oracle.step(s, dt=10.0, n_long=1, n_short=4)
    assert np.abs(out[3]).max() > 1e-3


def test_warm_bubble_rises(oracle):
    s = inputs.make_state(32, 32, 32, noise=0.0, u_bg=0.0, n_short=4)
    out = oracle.step(s, dt=10.0, n_long=3, n_short=4)
    wcol = out[3][:, 16, 16]
    kmax = int(np.argmax(wcol))
    assert wcol[kmax] > 0.05                        # upward mass flux through the bubble
    assert abs(s.zf[kmax] - 5000.0) < 4000.0        # peaking inside the bubble (r = 4 km)
    assert wcol.min() >= 0.0


def test_thread_count_does_not_change_results(oracle, tmp_path):
    code = (
        "import sys, numpy as np; sys.path.insert(0, %r)\n"
        "from paper_1710_08616_amd import inputs\n"
        "from oracle import oracle as O\n"
        "s = inputs.make_state(24, 20, 16, seed=4, n_short=3)\n"
        "f = O.step(s, n_long=2)\n"
        "np.savez(sys.argv[1], *f)\n" % ROOT)
    outs = []
    for nt in ("1", "3"):
        p = tmp_path / f"o{nt}.npz"
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        subprocess.check_call([sys.executable, "-c", code, str(p)], env=env)
        outs.append(np.load(p))
    for key in outs[0].files:
        assert np.array_equal(outs[0][key], outs[1][key])


def test_f32_storage_model_is_close_but_not_equal(oracle):
    s = inputs.workload("small")
    a = oracle.step(s, n_long=2)
    b = oracle.step(s.as_f32(), n_long=2, f32_storage=True)
    for x, y in zip(a, b):
        rng_ = np.ptp(x) or 1.0
        assert np.max(np.abs(x - y)) <= 1e-4 * rng_
    assert any(not np.array_equal(x, y) for x, y in zip(a, b))
