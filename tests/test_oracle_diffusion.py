"""Pins of the seven-point diffusion step (the bandwidth-model stencil of the
paper's reduced weather application, Sect. 4).

- a constant field is a fixed point, bitwise;
- the sum is conserved (periodic sides, no flux through the lids);
- a separable cosine mode decays by exactly
  1 - 4 kx sin^2(ax/2) - 4 ky sin^2(ay/2) - 4 kz sin^2(az/2) per step
  (vertical modes cos(m pi (k + 1/2) / nz) satisfy the no-flux lids);
- the result equals a 7-point correlation with scipy.ndimage (wrap in x, y,
  nearest = mirrored ghost in z);
- with kx + ky + kz <= 1/2 no new extrema appear.
"""
import math

import numpy as np
import pytest


def _rand(shape, seed):
    return np.random.default_rng(seed).normal(size=shape)


def test_constant_field_is_fixed_point(oracle):
    q = np.full((8, 6, 10), 3.25)
    out = oracle.diffuse(q, 0.1, 0.12, 0.2, steps=3)
    assert np.array_equal(out, q)


def test_sum_is_conserved(oracle):
    q = _rand((16, 12, 20), 1)
    out = oracle.diffuse(q, 0.1, 0.15, 0.2, steps=5)
    assert abs(out.sum() - q.sum()) <= 1e-12 * np.abs(q).sum()
    assert not np.allclose(out, q)


@pytest.mark.parametrize("mx,my,mz", [(1, 0, 0), (0, 2, 0), (0, 0, 3), (3, 1, 2), (8, 6, 7)])
def test_cosine_mode_decay_closed_form(oracle, mx, my, mz):
    nx, ny, nz = 16, 12, 14
    kx, ky, kz = 0.11, 0.07, 0.2
    ax, ay, az = 2 * math.pi * mx / nx, 2 * math.pi * my / ny, math.pi * mz / nz
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = (np.arange(nz) + 0.5)[:, None, None]
    q = np.cos(ax * i) * np.cos(ay * j) * np.cos(az * k)
    g = 1.0 - 4 * kx * math.sin(ax / 2) ** 2 - 4 * ky * math.sin(ay / 2) ** 2 \
        - 4 * kz * math.sin(az / 2) ** 2
    steps = 4
    out = oracle.diffuse(q, kx, ky, kz, steps=steps)
    assert np.max(np.abs(out - g ** steps * q)) <= 1e-13


def test_matches_scipy_correlation(oracle):
    from scipy import ndimage
    q = _rand((10, 9, 11), 2)
    kx, ky, kz = 0.13, 0.09, 0.17
    w = np.zeros((3, 3, 3))
    w[1, 1, 1] = 1.0 - 2 * (kx + ky + kz)
    w[1, 1, 0] = w[1, 1, 2] = kx
    w[1, 0, 1] = w[1, 2, 1] = ky
    w[0, 1, 1] = w[2, 1, 1] = kz
    # wrap in x and y; the lids mirror the boundary cell ("nearest" ghost)
    padded = np.pad(q, ((1, 1), (0, 0), (0, 0)), mode="edge")
    ref = ndimage.correlate(padded, w, mode="wrap")[1:-1]
    out = oracle.diffuse(q, kx, ky, kz)
    assert np.max(np.abs(out - ref)) <= 1e-14 * 10


def test_no_new_extrema_when_stable(oracle):
    q = _rand((12, 10, 14), 3)
    out = oracle.diffuse(q, 0.15, 0.15, 0.2, steps=6)
    assert out.max() <= q.max() + 1e-15 and out.min() >= q.min() - 1e-15
