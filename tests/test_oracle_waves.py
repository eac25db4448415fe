"""Closed-form acoustic modes of the HEVI short step.

With g = 0, a height-independent reference state and a perturbation of
relative size 1e-8, the slow tendencies are second order in the amplitude.
The third RK3 stage restarts from the start state, so to first order one long
step is n short steps of length dt/n, and a single Fourier mode evolves by the
n-th power of a 2x2 amplification matrix that follows from the linearised
equations alone:

- horizontally (forward-backward): U+ = U - dtau dx p, p+ = p - c^2 dtau dx U+
  gives M = [[1, -i a], [-i c^2 a, 1 - c^2 a^2]], a = (2 dtau/dx) sin(k dx/2),
  whose eigenvalues satisfy cos(w dtau) = 1 - 2 (c dtau/dx)^2 sin^2(k dx/2);
- vertically (beta-trapezoidal): (I - beta dtau L) x+ = (I + (1-beta) dtau L) x
  with L = [[0, K], [-c^2 K, 0]], K = (2/dz) sin(m pi / (2 nz)); for beta = 1/2
  tan(w dtau / 2) = c dtau K / 2 and |G| = 1, for beta > 1/2 |G| < 1.

The oracle's full 3D step must follow these to 1e-6 of the amplitude.
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


@pytest.mark.parametrize("axis", ["x", "y"])
@pytest.mark.parametrize("mode", [1, 5, 16])
def test_horizontal_acoustic_mode(oracle, axis, mode):
    n, dt, dx, nn = 64, 10.0, 2000.0, 4
    s = _uniform_state(n if axis == "x" else 1, 1 if axis == "x" else n, 4, dx, 4000.0, 0.5)
    c2 = GAMMA * s.p_ref[0] / s.rho_ref[0]
    c = math.sqrt(c2)
    amp = 1e-8 * s.rho_ref[0] * c
    k = 2.0 * math.pi * mode / (n * dx)
    xf = np.arange(n) * dx                  # west/south faces
    xc = xf + 0.5 * dx                      # centres
    u0 = amp * np.cos(k * xf)
    if axis == "x":
        s.fields[1][:] = u0[None, None, :]
    else:
        s.fields[2][:] = u0[None, :, None]
    out = oracle.step(s, dt=dt, n_long=1, n_short=nn, grav=0.0)
    dtau = dt / nn
    a = 2.0 * dtau / dx * math.sin(0.5 * k * dx)
    M = np.array([[1.0, -1j * a], [-1j * c2 * a, 1.0 - c2 * a * a]])
    uh, ph = np.linalg.matrix_power(M, nn) @ np.array([amp, 0.0])
    u_want = np.real(uh * np.exp(1j * k * xf))
    p_want = np.real(ph * np.exp(1j * k * xc))
    if axis == "x":
        u_got = out[1][:, 0, :]
        p_got = _pprime(s, out[4])[:, 0, :]
        other = out[2]
    else:
        u_got = out[2][:, :, 0]
        p_got = _pprime(s, out[4])[:, :, 0]
        other = out[1]
    assert np.max(np.abs(u_got - u_want[None, :])) <= 1e-6 * amp
    assert np.max(np.abs(p_got - p_want[None, :])) <= 1e-6 * amp * c
    assert np.max(np.abs(other)) <= 1e-6 * amp
    assert np.max(np.abs(out[3])) <= 1e-6 * amp
    # the discrete dispersion relation (eigen-phase of M) vs its closed form
    lam = np.linalg.eigvals(M)
    cos_w = 1.0 - 2.0 * (c * dtau / dx) ** 2 * math.sin(0.5 * k * dx) ** 2
    assert np.allclose(np.abs(lam), 1.0, atol=1e-12)
    assert np.allclose(np.real(lam), cos_w, atol=1e-12)


@pytest.mark.parametrize("beta", [0.5, 0.55, 0.7])
@pytest.mark.parametrize("mode", [1, 3, 15])
def test_vertical_acoustic_mode(oracle, beta, mode):
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
    out = oracle.step(s, dt=dt, n_long=1, n_short=nn, grav=0.0)
    dtau = dt / nn
    K = 2.0 / dz * math.sin(mode * math.pi / (2 * nz))
    L = np.array([[0.0, K], [-c2 * K, 0.0]])
    I = np.eye(2)
    G = np.linalg.solve(I - beta * dtau * L, I + (1.0 - beta) * dtau * L)
    wh, ph = np.linalg.matrix_power(G, nn) @ np.array([amp, 0.0])
    assert np.max(np.abs(out[3][:, 0, 0] - wh * sk)) <= 1e-6 * amp
    assert np.max(np.abs(_pprime(s, out[4])[:, 0, 0] - ph * cm)) <= 1e-6 * amp * c
    lam = np.linalg.eigvals(G)
    if beta == 0.5:
        assert np.allclose(np.abs(lam), 1.0, atol=1e-12)
        w = np.abs(np.angle(lam[0]))
        assert math.tan(0.5 * w) == pytest.approx(0.5 * c * dtau * K, rel=1e-12)
    else:
        assert np.all(np.abs(lam) < 1.0)
        # |G|^2 = (1 + (1-b)^2 x^2) / (1 + b^2 x^2), x = c dtau K
        x = c * dtau * K
        g2 = (1.0 + (1.0 - beta) ** 2 * x * x) / (1.0 + beta * beta * x * x)
        assert np.allclose(np.abs(lam) ** 2, g2, rtol=1e-12)


@pytest.mark.parametrize("mode", [1, 4, 9])
@pytest.mark.parametrize("dt", [10.0, 25.0])
def test_rk3_stage_structure_closed_form(oracle, mode, dt):
    """With a linear (donor-cell) slow operator and vanishing fast terms, the
    long step is the Wicker-Skamarock RK3 map: stages of length dt/3, dt/2 and
    dt, each restarting from the start state, give
        G = 1 + z + z^2/2 + z^3/6,  z = dt * lambda,
    for a Fourier mode with donor-cell eigenvalue
        lambda = -(u0/dx) (1 - exp(-i k dx)).
    Case: y-momentum V(x) advected by a uniform x-flow on a grid with ny = 1,
    so no pressure gradient, divergence or Theta change is ever produced.
    """
    nx, dx, u0 = 48, 2000.0, 20.0
    rho, rt, p = inputs.reference_uniform(4, 1.0, 300.0, GAMMA)
    zf = inputs.uniform_levels(4, 4000.0)
    f = [np.zeros((4, 1, nx)), np.full((4, 1, nx), u0), np.zeros((4, 1, nx)),
         np.zeros((5, 1, nx)), np.zeros((4, 1, nx))]
    k = 2.0 * math.pi * mode / (nx * dx)
    xc = (np.arange(nx) + 0.5) * dx
    amp = 0.3
    f[2][:] = amp * np.cos(k * xc)[None, None, :]
    s = inputs.State(nx, 1, 4, dx, dx, zf, rho, rt, p, f, beta=0.55)
    out = oracle.step(s, dt=dt, n_long=1, n_short=3, grav=0.0, donor_cell=True)
    lam = -(u0 / dx) * (1.0 - np.exp(-1j * k * dx))
    z = dt * lam
    G = 1.0 + z + z * z / 2.0 + z ** 3 / 6.0
    want = np.real(amp * G * np.exp(1j * k * xc))
    assert np.max(np.abs(out[2][:, 0, :] - want[None, :])) <= 1e-12 * amp
    assert np.array_equal(out[1], f[1])
    for q in (out[0], out[3], out[4]):
        assert np.max(np.abs(q)) == 0.0
