"""Pins of the oracle's vertically implicit column solve.

The HEVI short step (paper Sect. 1.1) couples W, rho' and Theta' implicitly
in the vertical; substituting the cell updates into the W equation gives one
tridiagonal system per column.  The oracle assembles it in closed form and
solves it with the Thomas algorithm.  Here the solve is held to a dense LU
(numpy.linalg.solve), and the assembled matrix and right-hand side are held to
the brute-force Jacobian of the update equations themselves.
"""
import numpy as np
import pytest

from paper_1710_08616_amd import inputs

GRAV = 9.80665


@pytest.mark.parametrize("n", [1, 2, 3, 7, 31, 63, 64])
def test_thomas_matches_dense_lu(oracle, n):
    rng = np.random.default_rng(n)
    for _ in range(5):
        a = rng.normal(size=n)
        c = rng.normal(size=n)
        b = np.abs(a) + np.abs(c) + rng.uniform(0.1, 2.0, size=n)
        b *= rng.choice([-1.0, 1.0], size=n)
        d = rng.normal(size=n) * 10.0
        M = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        want = np.linalg.solve(M, d)
        got, rc = oracle.thomas(a, b, c, d)
        assert rc == 0
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_thomas_flags_non_dominant_rows(oracle):
    a = np.array([0.0, 1.0, 1.0])
    b = np.array([1.0, 1.5, 3.0])
    c = np.array([0.5, 1.0, 0.0])
    _, rc = oracle.thomas(a, b, c, np.ones(3))
    assert rc == oracle.ENOTDOM


def _column(nz, seed, zf, scale=1.0):
    """A realistic random column: reference-like stage coefficients and
    perturbations of the size seen in the warm-bubble runs."""
    rng = np.random.default_rng(seed)
    zc = inputs.centres(zf)
    rho, rt, p = inputs.reference_isothermal(zc)
    th = rt / rho + rng.normal(size=nz)
    Cs = 1.4 * p / rt * (1.0 + 1e-3 * rng.normal(size=nz))
    col = dict(
        rt=scale * 1e-3 * rng.normal(size=nz),
        tt=scale * 0.5 * rng.normal(size=nz),
        rp=scale * 1e-3 * rng.normal(size=nz),
        pp=scale * 50.0 * rng.normal(size=nz),
        P0=scale * 20.0 * rng.normal(size=nz),
        Cs=Cs,
        ths=th,
        W=np.concatenate([[0.0], scale * 0.5 * rng.normal(size=nz - 1), [0.0]]),
        SW=np.concatenate([[0.0], scale * 1e-3 * rng.normal(size=nz - 1), [0.0]]),
    )
    return col


@pytest.mark.parametrize("nz,stretched,beta,dtau,terrain",
                         [(8, True, 0.55, 2.5, False), (8, False, 0.5, 1.0, False),
                          (32, True, 0.55, 2.5, False), (64, True, 0.7, 1.6, False),
                          (8, True, 0.55, 2.5, True), (32, True, 0.6, 2.0, True)])
def test_assembly_is_jacobian_of_update_equations(oracle, nz, stretched, beta, dtau, terrain):
    """Over terrain the column has J < 1 and a nonzero slope flux E."""
    zf = inputs.levels(nz) if stretched else inputs.uniform_levels(nz, 8000.0)
    col = _column(nz, nz * 7 + 1, zf)
    jac, E = 1.0, None
    if terrain:
        jac = 0.9
        E = np.concatenate([[0.0], 0.3 * np.random.default_rng(nz).normal(size=nz - 1), [0.0]])
    A, B, C, D = oracle.vi_assemble(zf, beta, dtau, GRAV, col, jac, E)
    r0 = oracle.vi_residual(zf, beta, dtau, GRAV, col, np.zeros(nz + 1), jac, E)
    # the residual is affine in W+: R(W+) = M W+ - D
    assert np.allclose(-r0[1:nz], D[1:nz], rtol=1e-12, atol=1e-12 * np.abs(D).max())
    M = np.zeros((nz - 1, nz - 1))
    for jcol in range(1, nz):
        e = np.zeros(nz + 1)
        e[jcol] = 1.0
        M[:, jcol - 1] = (oracle.vi_residual(zf, beta, dtau, GRAV, col, e, jac, E) - r0)[1:nz]
    T = np.diag(B[1:nz]) + np.diag(A[2:nz], -1) + np.diag(C[1:nz - 1], 1)
    assert np.max(np.abs(M - T)) <= 1e-11 * np.max(np.abs(T))
    # nothing outside the three diagonals
    off = M.copy()
    for d in (-1, 0, 1):
        off -= np.diag(np.diag(M, d), d)
    assert np.max(np.abs(off)) <= 1e-12 * np.max(np.abs(T))


def test_solved_column_satisfies_update_equations(oracle):
    nz = 32
    zf = inputs.levels(nz)
    col = _column(nz, 99, zf)
    A, B, C, D = oracle.vi_assemble(zf, 0.55, 2.5, GRAV, col)
    x, rc = oracle.thomas(A[1:nz], B[1:nz], C[1:nz], D[1:nz])
    assert rc == 0
    Wp = np.concatenate([[0.0], x, [0.0]])
    R = oracle.vi_residual(zf, 0.55, 2.5, GRAV, col, Wp)
    assert np.max(np.abs(R)) <= 1e-12 * np.max(np.abs(Wp))


@pytest.mark.parametrize("nz", [32, 64])
def test_columns_are_diagonally_dominant(oracle, nz):
    """Row margin B - |A| - |C| stays near 1 for the paper-scale short steps."""
    zf = inputs.levels(nz)
    col = _column(nz, 5, zf)
    for dtau in (10.0 / 3 / 4, 10.0 / 4, 10.0 / 6):
        A, B, C, D = oracle.vi_assemble(zf, 0.55, dtau, GRAV, col)
        margin = B[1:nz] - np.abs(A[1:nz]) - np.abs(C[1:nz])
        margin[0] = B[1] - np.abs(C[1])
        assert margin.min() > 0.5
