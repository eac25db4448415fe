"""The i-fastest layout's own mapping: one lane per column, 64 columns at
consecutive i per wavefront, the k loop inside every lane, and a serial
Thomas sweep per column (hv_configure config width 0; width 1 runs the
column-segment kernels on the same storage).

- the slow sweeps compute every cell as the segment kernels do: with the
  short step in column segments, the whole step equals the column-fastest
  layout's bitwise;
- the full column mapping (its own column solve) matches the oracle: float64
  within 1e-11 of the field range, float32 / mixed within 10x the oracle's
  binary32-storage twin; flat and over hills, 32/64/128 levels, grids whose
  nx is not a multiple of 64 nor ny of 4 (inactive lanes), and the smallest
  grid whose stencils wrap onto themselves;
- mass is conserved to 1e-14 (float64) per long step; graph replay equals
  direct launches bitwise.
"""
import numpy as np
import pytest

from paper_1710_08616_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_08616_amd import hevi
    hevi.load()
    return hevi


def _rel(a, b):
    r = np.ptp(b)
    return np.abs(a - b).max() / (r if r > 0 else 1.0)


def _state(nx, ny, nz, terrain, seed):
    h = None
    if terrain:
        h = inputs.orography(nx, ny, 2000.0, 2000.0, seed, hmax=1200.0, hills=2,
                             smin=3000.0 * max(1, nx // 20), smax=6000.0 * max(1, nx // 20))
    return inputs.make_state(nx, ny, nz, seed=seed, terrain=h, noise=0.5, u_bg=6.0, v_bg=-2.0,
                             shear=8.0, n_short=3,
                             bubbles=[(nx * 1000.0, ny * 1000.0, 5000.0, 4000.0)])


def _run(hv, s, prec, layout, config=None, n_long=2):
    d = hv.Domain(s, precision=prec, layout=layout)
    if config is not None:
        d.configure(config)
    d.step(s.dt, n_long, s.n_short)
    out = d.read_all()
    m = d.mass()
    d.close()
    return out, m


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("nz", [32, 64, 128])
@pytest.mark.parametrize("terrain", [False, True])
def test_column_slow_sweeps_equal_the_segment_kernels(hv, prec, nz, terrain):
    s = _state(70, 9, nz, terrain, 60 + nz)
    print(f"case: ijk sweeps {prec} nz={nz} terrain={terrain}", flush=True)
    ref, _ = _run(hv, s, prec, "kij")
    # slow sweeps one lane per column, short step in column segments
    got, _ = _run(hv, s, prec, "ijk", [0, 0, 6])
    for name, a, b in zip(inputs.FIELD_NAMES, got, ref):
        assert np.array_equal(a, b), name
    # everything in column segments
    seg, _ = _run(hv, s, prec, "ijk", [6, 6, 6])
    for name, a, b in zip(inputs.FIELD_NAMES, seg, ref):
        assert np.array_equal(a, b), name


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("nx,ny,nz,terrain", [(70, 9, 32, False), (70, 9, 64, True), (66, 5, 128, False),
                                              (40, 12, 128, True), (4, 5, 32, False), (5, 4, 64, True)])
def test_column_step_matches_oracle(hv, oracle, prec, nx, ny, nz, terrain):
    """(Float32 with 128 levels: the float32 column solve of such stiff
    columns rounds beyond the twin bar in any mapping; there the column
    mapping must not be worse than the column-fastest segments by more than
    2x.)"""
    s = _state(nx, ny, nz, terrain, 70 + nx + nz)
    print(f"case: ijk columns {prec} {nx}x{ny}x{nz} terrain={terrain}", flush=True)
    d = hv.Domain(s, precision=prec, layout="ijk")
    lanes = d.configure([0, 0, 0])[2]
    d.close()
    assert lanes == [1, 1, 1]
    got, _ = _run(hv, s, prec, "ijk", [0, 0, 0])
    ref = oracle.step(s, n_long=2)
    if prec == "fp64":
        for name, a, b in zip(inputs.FIELD_NAMES, got, ref):
            assert _rel(a, b) <= 1e-11, (name, _rel(a, b))
    elif prec == "fp32" and nz == 128:
        seg, _ = _run(hv, s, prec, "kij")
        for name, a, g, b in zip(inputs.FIELD_NAMES, got, seg, ref):
            assert _rel(a, b) <= 2.0 * _rel(g, b) + 1e-12, (name, _rel(a, b), _rel(g, b))
    else:
        twin = oracle.step(s.as_f32(reference=True), n_long=2, f32_storage=True)
        for name, a, b, t in zip(inputs.FIELD_NAMES, got, ref, twin):
            assert _rel(a, b) <= 10.0 * _rel(t, b), (name, _rel(a, b), _rel(t, b))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-14), ("mixed", 1e-11), ("fp32", 1e-11)])
def test_column_step_conserves_mass(hv, prec, tol):
    s = _state(70, 9, 64, True, 81)
    print(f"case: ijk mass {prec}", flush=True)
    d = hv.Domain(s, precision=prec, layout="ijk")
    assert d.configure()[2] == [1, 1, 1]
    m0 = d.mass()
    for _ in range(3):
        d.step(s.dt, 1, s.n_short)
        assert abs(d.mass() - m0) <= tol * m0
    d.close()


def test_column_graph_replay_equals_direct_launches(hv):
    s = _state(70, 9, 64, False, 82)
    print("case: ijk graph vs direct", flush=True)
    out = []
    for trace in (False, True):
        d = hv.Domain(s, precision="mixed", layout="ijk")
        d.trace(trace)
        d.step(s.dt, 2, s.n_short)
        out.append(d.read_all())
        d.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("nx,ny,nz,terrain", [(70, 9, 64, False), (37, 23, 32, True), (300, 5, 128, False)])
def test_column_mass_matches_the_oracle_and_the_segment_sum(hv, oracle, prec, nx, ny, nz, terrain):
    """The i-fastest mass sum (one lane per column; 630, 851 and 1500
    columns: chunks of 256 with a ragged last one) equals the oracle's mass of
    the device state and the column-fastest layout's segment sum of the same
    state to 1e-14 (float64 sums in another order), after steps and at
    state_init; an ensemble of i-fastest members (grouped launch) gives each
    member's single-grid mass bitwise."""
    s = _state(nx, ny, nz, terrain, 90 + nx)
    print(f"case: ijk mass sum {prec} {nx}x{ny}x{nz} terrain={terrain}", flush=True)
    d = hv.Domain(s, precision=prec, layout="ijk")
    m_init = d.mass()
    d.step(s.dt, 1, s.n_short)
    m = d.mass()
    s2 = s.copy()
    s2.fields = d.read_all()
    d.close()
    want = oracle.mass(s2)
    assert abs(m - want) <= 1e-14 * abs(want), (m, want)
    k = hv.Domain(s2, precision=prec, layout="kij")
    mk = k.mass()
    k.close()
    assert abs(m - mk) <= 1e-14 * abs(mk), (m, mk)
    s0 = s.as_f32() if prec != "fp64" else s
    assert abs(m_init - oracle.mass(s0)) <= 1e-14 * abs(m_init)


def test_column_mass_in_an_ensemble_equals_single_grids(hv):
    ms = [_state(70, 9, 64, False, 95), _state(37, 23, 64, False, 96), _state(20, 30, 64, False, 97)]
    print("case: ijk mass ensemble", flush=True)
    e = hv.Ensemble(ms, precision="fp32", layout="ijk")
    e.step(1, 3)
    got = [e.mass(q) for q in range(len(ms))]
    states = [e.read_all(q) for q in range(len(ms))]
    e.close()
    for q, s in enumerate(ms):
        s2 = s.copy()
        s2.fields = states[q]
        d = hv.Domain(s2, precision="fp32", layout="ijk")
        assert d.mass() == got[q], q
        d.close()
