"""Pins of the oracle's terrain-following form, each fixed by geometry or
by the continuous equations rather than by the oracle's own code.

Reading held to here: height z = zeta + h (1 - zeta/H), Jacobian J = 1 - h/H
per column, J on x- and y-faces the mean of the two columns, face slopes
dh/dx and dh/dy as one-sided differences of h, the flux through the zeta
surfaces Omega = W - (1 - zeta/H) (slope-weighted momenta, averaged to the
level face), zero on both lids.

- zero terrain is the flat model, bitwise;
- a raised plateau (constant h) is the flat model on levels compressed by J;
- a pressure perturbation linear in true height, in hydrostatic balance,
  stays at rest over hills (the metric correction of the horizontal pressure
  gradient cancels the along-zeta gradient exactly);
- a flow that follows the zeta surfaces (J U constant, Omega = 0) stays
  steady in the short step and gives no Theta residual over a stratified
  theta(zeta) in the slow sweep;
- total mass J (rho_ref + rho') dx dy dzeta is conserved, and the slow
  momentum tendencies are in conservative form;
- a uniform potential temperature stays uniform under any flow over hills;
- rest over terrain stays exactly at rest.
"""
import numpy as np
import pytest

from paper_1710_08616_amd import inputs

GRAV = inputs.GRAV
H = inputs.H_TOP


def _hills(nx, ny, dx, seed=7, hmax=1500.0):
    return inputs.orography(nx, ny, dx, dx, seed, hmax=hmax, hills=3, smin=3 * dx, smax=6 * dx)


def _terrain_state(nx=20, ny=16, nz=16, seed=3, terrain=None, reference="isothermal", **kw):
    h = _hills(nx, ny, 2000.0, seed) if terrain is None else terrain
    kw.setdefault("bubbles", [(nx * 1000.0, ny * 1000.0, 5000.0, 4000.0)])
    kw.setdefault("u_bg", 5.0)
    kw.setdefault("shear", 10.0)
    return inputs.make_state(nx, ny, nz, seed=seed, terrain=h, dt=10.0, n_short=4, n_long=2,
                             reference=reference, **kw)


def _faces(h, dx, dy):
    """J, Ju, Jv, dh/dx on x-faces, dh/dy on y-faces (the reading above)."""
    J = 1.0 - h / H
    Ju = 0.5 * ((1.0 - np.roll(h, 1, axis=1) / H) + (1.0 - h / H))
    Jv = 0.5 * ((1.0 - np.roll(h, 1, axis=0) / H) + (1.0 - h / H))
    su = (h - np.roll(h, 1, axis=1)) / dx
    sv = (h - np.roll(h, 1, axis=0)) / dy
    return J, Ju, Jv, su, sv


def test_zero_terrain_is_the_flat_model_bitwise(oracle):
    nx, ny, nz = 14, 10, 16
    kw = dict(seed=5, bubbles=[(14000.0, 10000.0, 5000.0, 4000.0)], u_bg=8.0, noise=0.5,
              dt=10.0, n_short=3, n_long=2)
    flat = inputs.make_state(nx, ny, nz, **kw)
    zero = inputs.make_state(nx, ny, nz, terrain=np.zeros((ny, nx)), **kw)
    assert zero.rho_ref.shape == (nz, ny, nx)
    for a, b in zip(flat.fields, zero.fields):
        assert np.array_equal(a, b)
    for a, b in zip(oracle.slow_sweep(flat), oracle.slow_sweep(zero)):
        assert np.array_equal(a, b)
    for a, b in zip(oracle.step(flat), oracle.step(zero)):
        assert np.array_equal(a, b)
    assert oracle.mass(flat) == oracle.mass(zero)
    assert oracle.energy(flat) == oracle.energy(zero)


def test_raised_plateau_is_the_flat_model_on_compressed_levels(oracle):
    """h = h0 everywhere: z = h0 + J zeta with J = 1 - h0/H constant, so the
    model is the flat one on levels J zeta with the same reference values
    (the shift h0 enters only through them)."""
    nx, ny, nz = 12, 10, 16
    h0 = 1500.0
    t = _terrain_state(nx, ny, nz, seed=9, terrain=np.full((ny, nx), h0), noise=0.5)
    J = 1.0 - h0 / H
    flat = inputs.State(nx, ny, nz, t.dx, t.dy, t.zf * J,
                        np.ascontiguousarray(t.rho_ref[:, 0, 0]),
                        np.ascontiguousarray(t.rt_ref[:, 0, 0]),
                        np.ascontiguousarray(t.p_ref[:, 0, 0]),
                        [f.copy() for f in t.fields], dt=t.dt, n_short=t.n_short,
                        n_long=t.n_long, beta=t.beta)
    a = oracle.step(t)
    b = oracle.step(flat)
    for f0, x, y in zip(t.fields, a, b):
        scale = max(np.abs(x).max(), np.abs(f0).max(), 1e-30)
        assert np.max(np.abs(x - y)) <= 1e-11 * scale
        assert not np.array_equal(x, f0) or np.abs(f0).max() == 0.0
    assert abs(oracle.mass(t) - oracle.mass(flat)) <= 1e-14 * oracle.mass(flat)


def test_hydrostatic_pressure_linear_in_height_stays_at_rest_over_hills(oracle):
    """p' = alpha z (true height) with rho' = -alpha/g is at rest: along a zeta
    surface dp'/dx = alpha dz/dx, which the metric term (z_x/J) dp'/dzeta
    cancels exactly for a linear profile; vertically -dp'/dz - g rho' = 0."""
    nx, ny, nz = 20, 16, 16
    s = _terrain_state(nx, ny, nz, seed=11)
    h = s.terrain
    z3 = inputs.true_heights(inputs.centres(s.zf), h)
    alpha = 0.05
    fields = [np.full((nz, ny, nx), -alpha / GRAV), np.zeros((nz, ny, nx)),
              np.zeros((nz, ny, nx)), np.zeros((nz + 1, ny, nx)), np.zeros((nz, ny, nx))]
    c = (nz, ny, nx)
    slow = [np.zeros(c), np.zeros(c), np.zeros((nz + 1, ny, nx)), np.zeros(c),
            s.rt_ref / s.rho_ref, alpha * z3, 1.4 * s.p_ref / s.rt_ref]
    dtau = 2.5
    out = oracle.short_step(s, slow, dtau, fields=fields)
    _, _, _, su, sv = _faces(h, s.dx, s.dy)
    # size of each of the two cancelling pressure-gradient terms
    scale_u = dtau * alpha * np.abs(su).max()
    scale_v = dtau * alpha * np.abs(sv).max()
    assert scale_u > 1e-3 and scale_v > 1e-3
    assert np.abs(out[1]).max() <= 1e-11 * scale_u
    assert np.abs(out[2]).max() <= 1e-11 * scale_v
    assert np.abs(out[3]).max() <= 1e-11 * dtau * alpha
    assert np.max(np.abs(out[0] - fields[0])) <= 1e-12 * alpha / GRAV
    assert np.abs(out[4]).max() <= 1e-10
    # without the metric term the same state accelerates along the slopes
    flat_like = s.copy()
    flat_like.terrain = np.zeros_like(h)
    out2 = oracle.short_step(flat_like, slow, dtau, fields=fields)
    assert np.abs(out2[1]).max() > 0.1 * scale_u


def _following_flow(s, u0=12.0, theta_lapse=4e-3):
    """rho' = 0, theta = theta(zeta) stratified, J U = u0 rho_0, V = 0, and W
    on every interior level face such that Omega = 0 (flow along the zeta
    surfaces)."""
    nx, ny, nz = s.nx, s.ny, s.nz
    h = s.terrain
    J, Ju, Jv, su, sv = _faces(h, s.dx, s.dy)
    zc = inputs.centres(s.zf)
    th = (300.0 + theta_lapse * zc)[:, None, None] * np.ones((nz, ny, nx))
    rp = np.zeros((nz, ny, nx))
    tp = s.rho_ref * th - s.rt_ref
    U = np.broadcast_to(u0 * 1.1 / Ju, (nz, ny, nx)).copy()
    V = np.zeros((nz, ny, nx))
    dz = np.diff(s.zf)
    a = dz[:-1] / (dz[:-1] + dz[1:])
    b = dz[1:] / (dz[:-1] + dz[1:])
    df = 1.0 - s.zf / H
    W = np.zeros((nz + 1, ny, nx))
    mx = 0.5 * (su * U + np.roll(su * U, -1, axis=2))         # slope-weighted U at the centre
    for k in range(1, nz):
        W[k] = df[k] * (a[k - 1] * mx[k] + b[k - 1] * mx[k - 1])
    return [rp, U, V, W, tp], th


def test_terrain_following_flow_is_steady_in_the_short_step(oracle):
    s = _terrain_state(20, 16, 16, seed=13)
    fields, th = _following_flow(s)
    nz, ny, nx = th.shape
    c = (nz, ny, nx)
    Cs = 1.4 * s.p_ref / s.rt_ref
    slow = [np.zeros(c), np.zeros(c), np.zeros((nz + 1, ny, nx)), np.zeros(c),
            th, -Cs * fields[4], Cs]                  # p' = P0 + C Theta' = 0
    dtau = 2.5
    out = oracle.short_step(s, slow, dtau, fields=fields)
    wmax = np.abs(fields[3]).max()
    assert wmax > 0.05
    assert np.array_equal(out[1], fields[1]) and np.array_equal(out[2], fields[2])
    assert np.max(np.abs(out[3] - fields[3])) <= 1e-12 * wmax
    # each cell's vertical flux change, had Omega* not vanished, would be ~dtau W/dz
    scale = dtau * wmax / np.diff(s.zf).min()
    assert np.abs(out[0]).max() <= 1e-11 * scale
    assert np.max(np.abs(out[4] - fields[4])) <= 1e-11 * scale * 600.0
    # the same W with the slope term of Omega dropped is far from steady
    wrong = [f.copy() for f in fields]
    wrong[3][:] = 0.0
    out2 = oracle.short_step(s, slow, dtau, fields=wrong)
    assert np.abs(out2[3]).max() > 0.01 * wmax


def test_terrain_following_flow_gives_no_theta_residual(oracle):
    """Omega = 0 and theta uniform along each zeta surface: every flux of
    (limited - centred) theta vanishes, while the same state with W = 0 (so
    Omega = -slope term) has a clear residual."""
    s = _terrain_state(20, 16, 16, seed=17)
    fields, th = _following_flow(s, theta_lapse=6e-3)
    # curvature in theta(zeta) so the limited and centred face values differ
    zc = inputs.centres(s.zf)
    th = (300.0 + 6e-3 * zc + 2.0 * np.sin(zc / 1500.0))[:, None, None] * np.ones_like(th)
    fields[4] = s.rho_ref * th - s.rt_ref
    RT = oracle.slow_sweep(s, fields)[3]
    wrong = [f.copy() for f in fields]
    wrong[3][:] = 0.0
    RT0 = oracle.slow_sweep(s, wrong)[3]
    assert np.abs(RT0).max() > 1e-6
    assert np.abs(RT).max() <= 1e-9 * np.abs(RT0).max()


def test_mass_is_conserved_over_terrain(oracle):
    s = _terrain_state(20, 16, 16, seed=19, noise=0.5)
    J = 1.0 - s.terrain / H
    dz = np.diff(s.zf)[:, None, None]
    m0 = oracle.mass(s)
    pm0 = (s.fields[0] * dz * J).sum()
    scale = (np.abs(s.fields[0]) * dz * J).sum()
    f = s.fields
    for _ in range(3):
        s2 = s.copy()
        s2.fields = f
        f = oracle.step(s2, n_long=1)
        s3 = s.copy()
        s3.fields = f
        assert abs(oracle.mass(s3) - m0) <= 1e-14 * m0
        assert abs((f[0] * dz * J).sum() - pm0) <= 1e-12 * scale
    assert np.max(np.abs(f[0] - s.fields[0])) > 1e-5


def test_slow_momentum_tendencies_are_conservative_over_terrain(oracle):
    """Sum over all control volumes of J_face S dzeta vanishes: flux form,
    periodic sides, no flux through the lids."""
    s = _terrain_state(20, 16, 16, seed=23, noise=1.0)
    J, Ju, Jv, su, sv = _faces(s.terrain, s.dx, s.dy)
    dz = np.diff(s.zf)[:, None, None]
    out = oracle.slow_sweep(s)
    for S, Jf in ((out[0], Ju), (out[1], Jv)):
        terms = S * Jf * dz
        assert np.abs(terms).sum() > 0.0
        assert abs(terms.sum()) <= 1e-12 * np.abs(terms).sum()
    # the same sum weighted with the cell Jacobian does not vanish
    terms = out[0] * J * dz
    assert abs(terms.sum()) > 1e-9 * np.abs(terms).sum()


def test_uniform_theta_is_preserved_over_terrain(oracle):
    nx, ny, nz = 16, 12, 16
    s = _terrain_state(nx, ny, nz, seed=29, reference="neutral", bubbles=[], noise=2.0)
    theta0 = s.rt_ref[0, 0, 0] / s.rho_ref[0, 0, 0]
    assert np.allclose(s.rt_ref / s.rho_ref, theta0, rtol=1e-15)
    out = oracle.step(s, dt=10.0, n_long=6, n_short=4)
    rho = s.rho_ref + out[0]
    th = (s.rt_ref + out[4]) / rho
    assert np.abs(out[0]).max() > 1e-6
    assert np.max(np.abs(th / theta0 - 1.0)) <= 1e-13


def test_rest_over_terrain_stays_exactly_at_rest(oracle):
    s = _terrain_state(12, 10, 16, seed=31)
    s.fields = [np.zeros_like(f) for f in s.fields]
    for f in oracle.step(s, n_long=2):
        assert np.all(f == 0.0)
