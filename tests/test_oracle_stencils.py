"""Closed forms of single stencil terms, each holding one interpolation or
control-volume detail of the oracle to what the discretisation says it is.

- A uniform specific velocity u0 (the same in every cell) makes every Koren
  face value u0, so flux-form momentum advection reduces to u0 times the mass
  convergence of its control volume.  With U = u0 rho_u (rho_u the two-point
  mean of the full density on the x-face), V = 0 and W = 0 that is
  S_U[i] = -u0 (U[i+1] - U[i-1]) / (2 dx), whatever the density does in x,
  y and z; likewise for V and, on level faces whose stencil stays off the
  lids, for W = w0 rho_w (rho_w linear in z between the two cell centres),
  S_W[k] = -w0 (W[k+1] - W[k-1]) / (2 dzf_k) with dzf_k the centre-to-centre
  distance of the W control volume.
- A potential temperature linear in height, theta = t0 + G z, is
  interpolated exactly by the linear centre-to-face weights: on stretched
  levels the short step's Theta flux through level face k is
  (t0 + G zf_k) W_k, and the slow sweep's centred face value is t0 + G zf_k,
  so the Theta residual takes a closed form from the limited face values
  (upwind, or Koren's third-order value in its smooth range).
- Flux-form Theta transport conserves the total sum(Theta' J dV) per long
  step to rounding on a periodic domain with rigid lids.
"""
import math

import numpy as np
import pytest

from paper_1710_08616_amd import inputs


def _varying_density_state(nx, ny, nz, seed=5):
    """Isothermal reference over stretched levels with a density perturbation
    that varies in x, y and z (about 3% of the reference) and Theta' = 0."""
    s = inputs.rest_state(nx, ny, nz)
    rng = np.random.default_rng(seed)
    s.fields[0][:] = 0.03 * s.rho_ref[:, None, None] * rng.uniform(-1.0, 1.0, (nz, ny, nx))
    return s


def _full_rho(s):
    return s.rho_ref[:, None, None] + s.fields[0]


@pytest.mark.parametrize("axis", ["x", "y"])
def test_uniform_horizontal_velocity_advects_like_mass(oracle, axis):
    nx, ny, nz = 12, 10, 16
    s = _varying_density_state(nx, ny, nz)
    rho = _full_rho(s)
    ax = 2 if axis == "x" else 1
    q0 = 8.0                          # a power of two: U / rho_u == q0 exactly
    rho_f = 0.5 * (np.roll(rho, 1, axis=ax) + rho)
    M = q0 * rho_f
    s.fields[1 if axis == "x" else 2][:] = M
    sl = oracle.slow_sweep(s)
    S = sl[0] if axis == "x" else sl[1]
    h = s.dx if axis == "x" else s.dy
    want = -q0 * (np.roll(M, -1, axis=ax) - np.roll(M, 1, axis=ax)) / (2.0 * h)
    scale = q0 * np.abs(M).max() / h
    assert np.max(np.abs(S - want)) <= 1e-13 * scale
    # the density variation is large enough for a different face density to show
    assert np.max(np.abs(want)) > 1e-3 * scale


def test_uniform_vertical_velocity_advects_like_mass(oracle):
    nx, ny, nz = 6, 5, 16
    s = _varying_density_state(nx, ny, nz, seed=6)
    rho = _full_rho(s)
    zf = s.zf
    zc = inputs.centres(zf)
    dz = np.diff(zf)
    w0 = 0.25
    # rho on level face k, linear in z between the centres of cells k-1 and k
    lam = ((zf[1:nz] - zc[:nz - 1]) / (zc[1:] - zc[:nz - 1]))[:, None, None]
    rho_w = rho[:nz - 1] + lam * (rho[1:] - rho[:nz - 1])
    W = np.zeros((nz + 1, ny, nx))
    W[1:nz] = w0 * rho_w
    # W / rho_w must give back w0 exactly for the closed form to hold bitwise in
    # the face values; the interpolation weights may round differently from
    # lam, so the check below allows for a few ulp of w0 in the face value
    s.fields[3][:] = W
    SW = oracle.slow_sweep(s)[2]
    dzf = np.zeros(nz + 1)
    dzf[1:nz] = zc[1:] - zc[:-1]
    ks = np.arange(2, nz - 1)                 # stencils clear of both lids
    want = -w0 * (W[ks + 1] - W[ks - 1]) / (2.0 * dzf[ks][:, None, None])
    scale = w0 * np.abs(W).max() / dzf[1:nz].min()
    assert np.max(np.abs(SW[ks] - want)) <= 1e-12 * scale
    assert np.max(np.abs(want)) > 1e-3 * scale
    assert np.all(SW[0] == 0.0) and np.all(SW[nz] == 0.0)
    # the stretched levels make dzf differ from the cell thickness
    assert np.max(np.abs(dzf[ks] - dz[ks]) / dz[ks]) > 1e-3


def test_short_step_theta_flux_uses_the_face_height(oracle):
    """One short step with only vertical transport switched on (C_s = 0 and
    g = 0 decouple W, so W* = W): rho'+_k = -(dtau/dz_k)(W_{k+1} - W_k) and
    Theta'+_k = -(dtau/dz_k)(theta(zf_{k+1}) W_{k+1} - theta(zf_k) W_k)."""
    nx, ny, nz = 3, 2, 32
    s = inputs.rest_state(nx, ny, nz)
    zf, zc = s.zf, inputs.centres(s.zf)
    dz = np.diff(zf)
    t0, G = 300.0, 0.004
    rng = np.random.default_rng(9)
    W = np.zeros((nz + 1, ny, nx))
    W[1:nz] = rng.uniform(-1.0, 1.0, (nz - 1, ny, nx))
    s.fields[3][:] = W
    c3 = (nz, ny, nx)
    slow = [np.zeros(c3), np.zeros(c3), np.zeros((nz + 1, ny, nx)), np.zeros(c3),
            np.broadcast_to((t0 + G * zc)[:, None, None], c3).copy(), np.zeros(c3), np.zeros(c3)]
    dtau = 2.5
    out = oracle.short_step(s, slow, dtau, grav=0.0)
    assert np.array_equal(out[3], W)
    thf = (t0 + G * zf)[:, None, None]
    r = (dtau / dz)[:, None, None]
    want_r = -r * (W[1:] - W[:-1])
    want_t = -r * (thf[1:] * W[1:] - thf[:-1] * W[:-1])
    assert np.max(np.abs(out[0] - want_r)) <= 1e-13 * np.abs(want_r).max()
    assert np.max(np.abs(out[4] - want_t)) <= 1e-12 * np.abs(want_t).max()


def _linear_theta_column_state(nx, ny, nz, t0, G, w0):
    """rho' = 0, Theta' such that theta = t0 + G z at the cell centres, U = V
    = 0, W = w0 on every interior level face."""
    s = inputs.rest_state(nx, ny, nz)
    zc = inputs.centres(s.zf)
    th = t0 + G * zc
    s.fields[4][:] = (s.rho_ref * th - s.rt_ref)[:, None, None]
    s.fields[3][1:nz] = w0
    return s


@pytest.mark.parametrize("donor_cell", [True, False])
@pytest.mark.parametrize("w0", [0.5, -0.5])
def test_theta_residual_closed_form_for_linear_theta(oracle, donor_cell, w0):
    """R_Theta = -d/dz(W (limited face theta - centred face theta)) for
    theta = t0 + G z and a uniform W on the interior faces.  The centred
    value is theta(zf_k); the limited one is upwind (donor cell) or, with the
    Koren limiter, q_up + (D- + 2 D+)/6 wherever the ratio of successive
    differences lies in Koren's smooth range (it is near 1 on these levels),
    and the upwind value next to a lid, where the zero-gradient ghost makes
    D- = 0."""
    nx, ny, nz = 3, 2, 32
    t0, G = 300.0, 0.004
    s = _linear_theta_column_state(nx, ny, nz, t0, G, w0)
    zf, zc = s.zf, inputs.centres(s.zf)
    dz = np.diff(zf)
    RT = oracle.slow_sweep(s, donor_cell=donor_cell)[3]
    th = t0 + G * zc
    F = np.zeros(nz + 1)
    for k in range(1, nz):
        up = w0 >= 0.0
        if donor_cell:
            q = th[k - 1] if up else th[k]
        else:
            if up:
                qL, qLL, qR = th[k - 1], th[max(k - 2, 0)], th[k]
            else:
                qL, qLL, qR = th[k], th[min(k + 1, nz - 1)], th[k - 1]
            dm, dp = qL - qLL, qR - qL
            if dm == 0.0:
                q = qL
            else:
                r = dp / dm
                assert 0.25 <= r <= 2.5       # Koren's smooth branch
                q = qL + (dm + 2.0 * dp) / 6.0
        F[k] = w0 * (q - (t0 + G * zf[k]))
    want = -(F[1:] - F[:-1]) / dz
    got = RT[:, 0, 0]
    assert np.all(RT == RT[:, :1, :1])           # horizontally uniform
    assert np.max(np.abs(got - want)) <= 1e-9 * np.abs(want).max()
    assert np.abs(want).max() > 1e-4


@pytest.mark.parametrize("terrain", [False, True])
def test_total_theta_is_conserved_per_long_step(oracle, terrain):
    """sum((Theta_ref + Theta') J dx dy dzeta) is invariant: the Theta
    residual, the short step's horizontal Theta divergence and its vertical
    Theta flux are all in flux form."""
    nx, ny, nz = 24, 20, 16
    h = inputs.orography(nx, ny, 2000.0, 2000.0, seed=77, hmax=1500.0) if terrain else None
    s = inputs.make_state(nx, ny, nz, seed=33, noise=1.0, u_bg=6.0, v_bg=-4.0,
                          bubbles=[(0.4 * nx * 2000.0, 0.6 * ny * 2000.0, 4000.0, 6000.0)],
                          terrain=h, n_short=4)
    dz = np.diff(s.zf)
    J = np.ones((ny, nx)) if h is None else 1.0 - h / s.zf[-1]
    vol = (s.dx * s.dy) * dz[:, None, None] * J[None, :, :]
    rt_ref = s.rt_ref if h is not None else np.broadcast_to(s.rt_ref[:, None, None], (nz, ny, nx))

    def total(tp):
        return math.fsum(((rt_ref + tp) * vol).ravel())

    def ptb(tp):
        return math.fsum((tp * vol).ravel())

    t0, p0 = total(s.fields[4]), ptb(s.fields[4])
    scale = math.fsum((np.abs(s.fields[0]) * vol).ravel()) * 300.0
    f = s.fields
    for _ in range(2):
        s.fields = f
        f = oracle.step(s, n_long=1)
        assert abs(total(f[4]) - t0) <= 1e-14 * t0
        assert abs(ptb(f[4]) - p0) <= 1e-11 * scale
    assert np.abs(f[4]).max() > 1e-3              # Theta' really changed
