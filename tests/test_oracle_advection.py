"""Pins of the oracle's flux-limited finite-volume advection.

The paper only names finite-volume discretisation (Sect. 1.1); the limiter is
the Koren (1993) kappa = 1/3 limiter.  These tests hold the oracle to values
fixed by that definition and by the mathematics of flux-form advection.
"""
import numpy as np
import pytest

from paper_1710_08616_amd import inputs

# psi(r) = max(0, min(2r, (1+2r)/3, 2)) evaluated by hand at these ratios
KOREN_TABLE = [(-1.0, 0.0), (0.0, 0.0), (0.25, 0.5), (0.5, 2.0 / 3.0), (1.0, 1.0),
               (2.5, 2.0), (4.0, 2.0)]


def test_koren_table(oracle):
    for r, psi in KOREN_TABLE:
        # Phi(D-, D+) = psi(D+/D-) D-, for both signs of D-
        assert oracle.koren_phi(1.0, r) == pytest.approx(psi, rel=0, abs=1e-15)
        assert oracle.koren_phi(-1.0, -r) == pytest.approx(-psi, rel=0, abs=1e-15)
        assert oracle.koren_phi(4.0, 4.0 * r) == pytest.approx(4.0 * psi, rel=0, abs=1e-14)
    # no upwind gradient: no correction, whatever the downwind one is
    for dp in (-3.0, 0.0, 2.0):
        assert oracle.koren_phi(0.0, dp) == 0.0


def test_smooth_regime_is_third_order_upwind(oracle):
    """For 1/4 <= r <= 5/2 the face value is (-q_LL + 5 q_L + 2 q_R)/6."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        qll = rng.uniform(-2, 2)
        dm = rng.uniform(0.1, 1.0) * rng.choice([-1.0, 1.0])
        r = rng.uniform(0.26, 2.49)
        ql = qll + dm
        qr = ql + r * dm
        want = (-qll + 5.0 * ql + 2.0 * qr) / 6.0
        got = oracle.face(qll, ql, qr, 123.0, 1.0)
        assert abs(got - want) <= 4 * np.spacing(max(abs(want), abs(ql), abs(qr)))
        # mirrored flow direction reads the stencil the other way round
        got_m = oracle.face(123.0, qr, ql, qll, -1.0)
        assert got_m == got


def test_linear_data_reproduced_exactly(oracle):
    for q0, d in ((1.0, 0.25), (-3.0, 0.5), (2.0, -1.0)):
        ql, qr = q0 + d, q0 + 2 * d
        assert oracle.face(q0, ql, qr, q0 + 3 * d, 2.0) == 0.5 * (ql + qr)
        assert oracle.face(q0, ql, qr, q0 + 3 * d, -2.0) == 0.5 * (ql + qr)


def test_limiter_clips_extrema(oracle):
    # at a local extremum the limited value is the upwind value (first order)
    assert oracle.face(0.0, 1.0, 0.5, 0.0, 1.0) == 1.0
    assert oracle.face(2.0, 1.0, 1.5, 9.0, 1.0) == 1.0
    # and it never leaves the interval spanned by q_L and q_R
    rng = np.random.default_rng(5)
    for _ in range(500):
        q = rng.normal(size=4)
        m = rng.normal()
        f = oracle.face(*q, m)
        assert min(q[1], q[2]) - 1e-15 <= f <= max(q[1], q[2]) + 1e-15


def _grid(nx, ny, nz, dx=1.0, dy=1.0, dzc=1.0):
    s = inputs.rest_state(nx, ny, nz, dx=dx, dy=dy, zf=np.arange(nz + 1) * dzc)
    return s


@pytest.mark.parametrize("axis,sign", [("x", 1), ("x", -1), ("y", 1), ("y", -1)])
def test_donor_cell_shift_at_courant_one(oracle, axis, sign):
    """Forward Euler + donor cell at C = 1 is an exact one-cell shift.

    dx = 0.5, dt = 0.25 and |u| = 2 are powers of two and q lies in [1, 2), so
    every subtraction is exact (Sterbenz) and the result must be bitwise.
    """
    nx, ny, nz = 16, 8, 3
    s = _grid(nx, ny, nz, dx=0.5, dy=0.5)
    rng = np.random.default_rng(11)
    q = rng.uniform(1.0, 2.0, size=(nz, ny, nx))
    u = np.zeros((nz, ny, nx))
    v = np.zeros((nz, ny, nx))
    w = np.zeros((nz + 1, ny, nx))
    if axis == "x":
        u[:] = 2.0 * sign
    else:
        v[:] = 2.0 * sign
    out = oracle.advect_fe(s, q, u, v, w, 0.25, oracle.LIM_NONE)
    want = np.roll(q, sign, axis=2 if axis == "x" else 1)
    assert np.array_equal(out, want)


def test_vertical_donor_cell_interior_shift(oracle):
    """Upward flow at C = 1: interior cells take their lower neighbour's value;
    the bottom cell empties and the top cell accumulates (rigid lids)."""
    nz = 6
    s = _grid(2, 2, nz, dzc=0.5)
    rng = np.random.default_rng(2)
    q = rng.uniform(1.0, 2.0, size=(nz, 2, 2))
    w = np.zeros((nz + 1, 2, 2))
    w[1:nz] = 2.0
    z = np.zeros((nz, 2, 2))
    out = oracle.advect_fe(s, q, z, z, w, 0.25, oracle.LIM_NONE)
    assert np.array_equal(out[1:nz - 1], q[0:nz - 2])
    assert np.array_equal(out[0], np.zeros((2, 2)))
    assert np.allclose(out[nz - 1], q[nz - 1] + q[nz - 2], rtol=0, atol=1e-15)


@pytest.mark.parametrize("lim", [0, 1])
def test_flux_form_conserves_total(oracle, lim):
    """Fluxes telescope on a periodic domain with lids: sum(q dz) is invariant."""
    nx, ny, nz = 12, 10, 7
    s = inputs.rest_state(nx, ny, nz, dx=300.0, dy=250.0, zf=inputs.levels(nz, 3000.0))
    rng = np.random.default_rng(7)
    q = rng.uniform(0.5, 2.0, size=(nz, ny, nx))
    u = rng.normal(size=(nz, ny, nx)) * 3.0
    v = rng.normal(size=(nz, ny, nx)) * 3.0
    w = rng.normal(size=(nz + 1, ny, nx))
    w[0] = w[nz] = 0.0
    dz = np.diff(s.zf)[:, None, None]
    out = oracle.advect_fe(s, q, u, v, w, 5.0, lim)
    before = (q * dz).sum()
    after = (out * dz).sum()
    assert abs(after - before) <= 1e-13 * before
    assert not np.allclose(out, q)


def test_koren_step_keeps_bounds_at_half_courant(oracle):
    """In 1D with C <= 1/2 the Koren limiter makes forward Euler bounded:
    no new extrema appear (psi <= 2 and psi(r)/r <= 2)."""
    nx = 64
    s = _grid(nx, 1, 1)
    rng = np.random.default_rng(9)
    q = np.where(rng.uniform(size=nx) < 0.5, 1.0, 0.0)[None, None, :]
    q = q + 0.3 * np.sin(np.arange(nx) / 3.0)[None, None, :]
    z = np.zeros((1, 1, nx))
    for c in (0.5, -0.45, 0.3):
        u = np.full((1, 1, nx), c)
        out = oracle.advect_fe(s, q, u, z, np.zeros((2, 1, nx)), 1.0, oracle.LIM_KOREN)
        assert out.max() <= q.max() + 1e-14
        assert out.min() >= q.min() - 1e-14
    # without the limiter's bound (C = 1.5) the same step does overshoot
    u = np.full((1, 1, nx), 1.5)
    out = oracle.advect_fe(s, q, u, z, np.zeros((2, 1, nx)), 1.0, oracle.LIM_KOREN)
    assert out.max() > q.max() + 1e-3 or out.min() < q.min() - 1e-3
