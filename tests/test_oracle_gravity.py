"""Linear gravity and acoustic waves of the full step against the dispersion
relation of the compressible isothermal atmosphere.

The paper integrates sound and gravity waves on the finer (short) time step
(Sect. 1.1).  Linearised about the hydrostatic isothermal reference at rest
(temperature T0, scale height Hs = R T0 / g, sound speed c^2 = gamma R T0,
buoyancy frequency N^2 = g^2 / (c_p T0), acoustic cut-off
wa = c / (2 Hs)), the compressible equations in an x-z slab between two rigid
lids have the normal modes
    W = rho w ~ exp(-z / (2 Hs)) sin(m z) cos(k x - w t),  m = n pi / H,
with
    w^4 - (c^2 (k^2 + m^2) + wa^2) w^2 + c^2 N^2 k^2 = 0
(the textbook result for an isothermal atmosphere, e.g. Gill 1982, ch. 6):
a slow gravity branch and a fast acoustic one.
A small W of that shape (relative amplitude 1e-6, so every nonlinear and
slow-tendency term is negligible) excites both.  The projection of the
model's W on the mode shape, sampled every long step, is a sum of damped
oscillations; a matrix-pencil fit gives their frequencies.  The scheme is
second order in space and time: with k dx <= 0.3 and m dz <= 0.3 on the
stretched levels its truncation error is of order (0.3)^2 / 24 ~ 0.4%, so
both branches must match the continuous relation within 1%.
"""
import math

import numpy as np
import pytest

from paper_1710_08616_amd import inputs

T0 = 300.0
GAMMA = 1.4


def _dispersion(k, m):
    hs = inputs.R_DRY * T0 / inputs.GRAV
    c2 = GAMMA * inputs.R_DRY * T0
    n2 = inputs.GRAV ** 2 / (inputs.CP_DRY * T0)
    b = c2 * (k * k + m * m) + c2 / (4.0 * hs * hs)
    d = math.sqrt(b * b - 4.0 * c2 * n2 * k * k)
    return math.sqrt(0.5 * (b - d)), math.sqrt(0.5 * (b + d)), math.sqrt(n2), math.sqrt(c2) / (2.0 * hs)


def _pencil(x, dt, order):
    """Frequencies, decay rates and amplitudes of the `order` damped complex
    exponentials that best represent the samples x (matrix-pencil method)."""
    n = len(x)
    L = n // 2
    Y = np.array([x[i:i + L + 1] for i in range(n - L)])
    _, _, vh = np.linalg.svd(Y, full_matrices=False)
    V = vh[:order].T
    z = np.linalg.eigvals(np.linalg.pinv(V[:-1]) @ V[1:])
    Z = np.vander(z, n, increasing=True).T
    amp = np.linalg.lstsq(Z, x.astype(complex), rcond=None)[0]
    return np.angle(z) / dt, np.log(np.abs(z)) / dt, np.abs(amp)


@pytest.mark.parametrize("mx,mz,n_long", [(1, 1, 250), (2, 1, 200), (3, 1, 200), (1, 2, 300)])
def test_gravity_and_acoustic_modes_follow_the_isothermal_dispersion_relation(oracle, mx, mz, n_long):
    nx, nz, dx, dt = 64, 32, 2000.0, 10.0
    s = inputs.rest_state(nx, 1, nz, dx=dx, n_short=4)
    zf = s.zf
    H = zf[-1]
    hs = inputs.R_DRY * T0 / inputs.GRAV
    k = 2.0 * math.pi * mx / (nx * dx)
    m = math.pi * mz / H
    shape = (np.exp(-zf / (2.0 * hs)) * np.sin(m * zf))[:, None] * \
        np.cos(k * (np.arange(nx) + 0.5) * dx)[None, :]
    shape[0] = 0.0
    shape[-1] = 0.0
    s.fields[3][:, 0, :] = 1e-6 * shape
    samples = []
    f = s.fields
    for n in range(n_long + 1):
        samples.append(float((f[3][:, 0, :] * shape).sum()))
        if n < n_long:
            s.fields = f
            f = oracle.step(s, dt=dt, n_long=1, n_short=4)
    w, sig, amp = _pencil(np.array(samples), dt, 6)
    wg, ws, N, wa = _dispersion(k, m)
    grav = [i for i in range(len(w)) if 0.0 < w[i] < N]
    sound = [i for i in range(len(w)) if w[i] > wa]
    assert grav and sound
    ig = max(grav, key=lambda i: amp[i])
    isd = max(sound, key=lambda i: amp[i])
    assert w[ig] == pytest.approx(wg, rel=1e-2)
    assert w[isd] == pytest.approx(ws, rel=1e-2)
    # the gravity wave is nearly neutral (the off-centring damps sound waves)
    assert abs(sig[ig]) < 1e-3 * wg
    assert sig[isd] < 0.0
