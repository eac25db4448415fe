"""Pins of the two-stage Runge-Kutta short step.

Reading: with Phi(X_b, X_e, d) the short step whose increments are added to
X_b and whose explicit and old-time (1 - beta) terms come from X_e, one
Runge-Kutta short step is X* = Phi(X, X, dtau/2), X+ = Phi(X, X*, dtau).

Closed forms (g = 0, height-independent reference, amplitude 1e-8, so the
slow terms are second order and one long step is n short steps of dt/n):
- horizontal mode: X* = M(a/2) X with the forward-backward matrix
  M(a) = [[1, -i a], [-i c^2 a, 1 - c^2 a^2]], then
  U+ = U - i a p*,  p+ = p - i c^2 a U+;
- vertical mode: G = (I - beta dtau L)^-1 (I + (1 - beta) dtau L G1) with
  G1 = (I - beta dtau/2 L)^-1 (I + (1 - beta) dtau/2 L).
Both damp: |lambda| < 1 for 0 < c a < 2, against the neutral forward-backward
step.  Steady states of the forward-backward step are steady here too, and
the flux form still conserves mass and a uniform theta.
"""
import math

import numpy as np
import pytest

from paper_1710_08616_amd import inputs

GAMMA = 1.4


def _uniform_state(nx, ny, nz, dx, top, beta):
    rho, rt, p = inputs.reference_uniform(nz, 1.0, 300.0, GAMMA)
    zf = inputs.uniform_levels(nz, top)
    f = [np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx)),
         np.zeros((nz + 1, ny, nx)), np.zeros((nz, ny, nx))]
    return inputs.State(nx, ny, nz, dx, dx, zf, rho, rt, p, f, beta=beta)


def _pprime(s, tp):
    return s.p_ref[:, None, None] * np.expm1(GAMMA * np.log1p(tp / s.rt_ref[:, None, None]))


def _m_fb(a, c2):
    return np.array([[1.0, -1j * a], [-1j * c2 * a, 1.0 - c2 * a * a]])


def _m_rk2(a, c2):
    mh = _m_fb(0.5 * a, c2)
    row_u = np.array([1.0, 0.0]) - 1j * a * mh[1, :]
    row_p = np.array([0.0, 1.0]) - 1j * c2 * a * row_u
    return np.array([row_u, row_p])


@pytest.mark.parametrize("axis", ["x", "y"])
@pytest.mark.parametrize("mode", [1, 5, 16])
def test_horizontal_acoustic_mode_rk2(oracle, axis, mode):
    n, dt, dx, nn = 64, 10.0, 2000.0, 4
    s = _uniform_state(n if axis == "x" else 1, 1 if axis == "x" else n, 4, dx, 4000.0, 0.5)
    c2 = GAMMA * s.p_ref[0] / s.rho_ref[0]
    c = math.sqrt(c2)
    amp = 1e-8 * s.rho_ref[0] * c
    k = 2.0 * math.pi * mode / (n * dx)
    xf = np.arange(n) * dx
    xc = xf + 0.5 * dx
    u0 = amp * np.cos(k * xf)
    if axis == "x":
        s.fields[1][:] = u0[None, None, :]
    else:
        s.fields[2][:] = u0[None, :, None]
    out = oracle.step(s, dt=dt, n_long=1, n_short=nn, grav=0.0, short_rk2=True)
    dtau = dt / nn
    a = 2.0 * dtau / dx * math.sin(0.5 * k * dx)
    M = _m_rk2(a, c2)
    uh, ph = np.linalg.matrix_power(M, nn) @ np.array([amp, 0.0])
    u_want = np.real(uh * np.exp(1j * k * xf))
    p_want = np.real(ph * np.exp(1j * k * xc))
    if axis == "x":
        u_got, p_got, other = out[1][:, 0, :], _pprime(s, out[4])[:, 0, :], out[2]
    else:
        u_got, p_got, other = out[2][:, :, 0], _pprime(s, out[4])[:, :, 0], out[1]
    assert np.max(np.abs(u_got - u_want[None, :])) <= 1e-6 * amp
    assert np.max(np.abs(p_got - p_want[None, :])) <= 1e-6 * amp * c
    assert np.max(np.abs(other)) <= 1e-6 * amp
    # damping, and the forward-backward result differs
    lam = np.abs(np.linalg.eigvals(M))
    assert np.all(lam < 1.0) and np.all(lam > 0.0)
    fb = oracle.step(s, dt=dt, n_long=1, n_short=nn, grav=0.0)
    assert np.max(np.abs(fb[1] - out[1]) + np.abs(fb[2] - out[2])) > 1e-4 * amp


@pytest.mark.parametrize("beta", [0.5, 0.55, 0.7])
@pytest.mark.parametrize("mode", [1, 3, 15])
def test_vertical_acoustic_mode_rk2(oracle, beta, mode):
    nz, top, dt, nn = 16, 4000.0, 10.0, 4
    s = _uniform_state(1, 1, nz, 2000.0, top, beta)
    c2 = GAMMA * s.p_ref[0] / s.rho_ref[0]
    c = math.sqrt(c2)
    amp = 1e-8 * s.rho_ref[0] * c
    dz = top / nz
    kk = np.arange(nz + 1)
    sk = np.sin(mode * math.pi * kk / nz)
    cm = np.cos(mode * math.pi * (np.arange(nz) + 0.5) / nz)
    s.fields[3][:, 0, 0] = amp * sk
    out = oracle.step(s, dt=dt, n_long=1, n_short=nn, grav=0.0, short_rk2=True)
    dtau = dt / nn
    K = 2.0 / dz * math.sin(mode * math.pi / (2 * nz))
    L = np.array([[0.0, K], [-c2 * K, 0.0]])
    I = np.eye(2)
    G1 = np.linalg.solve(I - beta * 0.5 * dtau * L, I + (1.0 - beta) * 0.5 * dtau * L)
    G = np.linalg.solve(I - beta * dtau * L, I + (1.0 - beta) * dtau * L @ G1)
    wh, ph = np.linalg.matrix_power(G, nn) @ np.array([amp, 0.0])
    assert np.max(np.abs(out[3][:, 0, 0] - wh * sk)) <= 1e-6 * amp
    assert np.max(np.abs(_pprime(s, out[4])[:, 0, 0] - ph * cm)) <= 1e-6 * amp * c
    assert np.all(np.abs(np.linalg.eigvals(G)) < 1.0)


def test_rk2_rest_and_uniform_flow_are_steady(oracle):
    s = inputs.rest_state(8, 6, 16, n_short=4)
    for f in oracle.step(s, dt=10.0, n_long=2, n_short=4, short_rk2=True):
        assert np.all(f == 0.0)
    s.fields[1][:] = (s.rho_ref * 10.0)[:, None, None]
    s.fields[2][:] = (s.rho_ref * -3.0)[:, None, None]
    out = oracle.step(s, dt=10.0, n_long=2, n_short=4, short_rk2=True)
    for f0, f1 in zip(s.fields, out):
        assert np.array_equal(f0, f1)


def test_rk2_mass_and_uniform_theta_conserved(oracle):
    s = inputs.make_state(16, 12, 16, seed=21, bubbles=[], noise=2.0, u_bg=5.0,
                          reference="neutral", n_short=4)
    theta0 = s.rt_ref[0] / s.rho_ref[0]
    m0 = oracle.mass(s)
    out = oracle.step(s, dt=10.0, n_long=4, n_short=4, short_rk2=True)
    s2 = s.copy()
    s2.fields = out
    assert abs(oracle.mass(s2) - m0) <= 1e-14 * m0
    th = (s.rt_ref[:, None, None] + out[4]) / (s.rho_ref[:, None, None] + out[0])
    assert np.abs(out[0]).max() > 1e-6
    assert np.max(np.abs(th / theta0 - 1.0)) <= 1e-13


def test_rk2_over_terrain_keeps_the_terrain_pins(oracle):
    """Mass over hills and rest over hills under the Runge-Kutta short step."""
    nx, ny, nz = 20, 16, 16
    h = inputs.orography(nx, ny, 2000.0, 2000.0, 7, hmax=1500.0, hills=3, smin=6000.0,
                         smax=12000.0)
    s = inputs.make_state(nx, ny, nz, seed=3, terrain=h, u_bg=5.0, shear=10.0, noise=0.5,
                          n_short=4)
    m0 = oracle.mass(s)
    out = oracle.step(s, dt=10.0, n_long=3, n_short=4, short_rk2=True)
    s2 = s.copy()
    s2.fields = out
    assert abs(oracle.mass(s2) - m0) <= 1e-14 * m0
    s.fields = [np.zeros_like(f) for f in s.fields]
    for f in oracle.step(s, dt=10.0, n_long=2, n_short=4, short_rk2=True):
        assert np.all(f == 0.0)


def test_rk2_warm_bubble_close_to_forward_backward(oracle):
    """Both short-step integrators carry the same slow, buoyant dynamics: the
    rising plume of a noise-free warm bubble (vertical momentum) after three
    long steps differs by a small fraction of its size, while the sound
    waves the start excites are damped only by the Runge-Kutta form."""
    s = inputs.make_state(48, 48, 32, seed=1710, noise=0.0, u_bg=0.0, n_short=4)
    a = oracle.step(s, n_long=3)
    b = oracle.step(s, n_long=3, short_rk2=True)
    wa, wb = a[3][:, 24, 24], b[3][:, 24, 24]
    assert wa.max() > 0.05
    assert np.abs(wa - wb).max() <= 0.05 * wa.max()
    assert not np.array_equal(a[3], b[3])
