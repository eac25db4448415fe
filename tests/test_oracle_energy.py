"""Pins of the oracle's diagnostic total energy (kinetic + internal +
potential), summed over cells of volume J dx dy dzeta.

Closed forms:
- rest state in the isothermal reference p = p0 exp(-z/Hs), rho g = p/Hs:
  per unit area, E = integral over [h, H] of p/(gamma-1) + rho g z dz
    = p0 Hs [(e^(-h/Hs) - e^(-H/Hs))/(gamma-1)
             + (1 + h/Hs) e^(-h/Hs) - (1 + H/Hs) e^(-H/Hs)],
  which the midpoint sums over the cells approach to O((dz/Hs)^2): with
  128 levels over 20 km about 1e-5 relative.  Over terrain each column
  integrates from its own surface height h (true heights, volumes J dzeta);
- a uniform flow u in a horizontally uniform density adds exactly
  (1/2) u^2 M (M the total mass, pinned in the mass tests), v likewise;
- with g = 0 only the internal energy p/(gamma-1) remains.
"""
import math

import numpy as np
import pytest

from paper_1710_08616_amd import inputs

GAMMA = 1.4
T0, P0 = 300.0, 1.0e5
HS = inputs.R_DRY * T0 / inputs.GRAV


def _rest(nx, ny, nz, terrain=None, dx=2000.0):
    zf = inputs.uniform_levels(nz, inputs.H_TOP)
    z = inputs.true_heights(inputs.centres(zf), terrain)
    rho, rt, p = inputs.reference_isothermal(z if terrain is not None else z[:, 0, 0], T0, P0)
    f = [np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx)),
         np.zeros((nz + 1, ny, nx)), np.zeros((nz, ny, nx))]
    return inputs.State(nx, ny, nz, dx, dx, zf, rho, rt, p, f, terrain=terrain)


def _column_energy(h, grav=True):
    a, b = h / HS, inputs.H_TOP / HS
    internal = P0 * HS * (math.exp(-a) - math.exp(-b)) / (GAMMA - 1.0)
    potential = P0 * HS * ((1.0 + a) * math.exp(-a) - (1.0 + b) * math.exp(-b)) if grav else 0.0
    return internal + potential


@pytest.mark.parametrize("grav", [True, False])
def test_rest_energy_of_the_isothermal_column(oracle, grav):
    s = _rest(6, 5, 128)
    e = oracle.energy(s, grav=inputs.GRAV if grav else 0.0)
    want = _column_energy(0.0, grav) * s.nx * s.ny * s.dx * s.dy
    assert abs(e / want - 1.0) <= 1e-4, (e, want)


def test_rest_energy_over_terrain_integrates_from_the_ground(oracle):
    nx, ny = 8, 6
    h = inputs.orography(nx, ny, 2000.0, 2000.0, 11, hmax=2500.0, hills=3, smin=3000.0,
                         smax=6000.0)
    s = _rest(nx, ny, 128, terrain=h)
    e = oracle.energy(s)
    want = sum(_column_energy(float(x)) for x in h.ravel()) * s.dx * s.dy
    assert abs(e / want - 1.0) <= 1e-4, (e, want)
    # and the terrain term matters: flat ground would be far off
    flat = _column_energy(0.0) * nx * ny * s.dx * s.dy
    assert abs(flat / want - 1.0) > 1e-2


@pytest.mark.parametrize("axis", [1, 2])
def test_uniform_flow_adds_half_u_squared_times_mass(oracle, axis):
    s = _rest(7, 6, 32)
    e0 = oracle.energy(s)
    m = oracle.mass(s)
    u = 13.0
    s.fields[axis][:] = (s.rho_ref * u)[:, None, None]
    e1 = oracle.energy(s)
    assert abs((e1 - e0) / (0.5 * u * u * m) - 1.0) <= 1e-9
