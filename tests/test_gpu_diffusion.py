"""GPU parity of the seven-point diffusion step (hv_diffuse) with the oracle.

The kernel evaluates the oracle's expression in the oracle's order with
contraction off, so float64 results are bitwise equal; float32 is compared
with the oracle run on the binary32-rounded input, within 4 ulps of the
field's magnitude per step.  Layouts and tile shapes agree bitwise.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

K = (0.11, 0.09, 0.21)


@pytest.fixture(scope="module")
def hv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_08616_amd import hevi
    hevi.load()
    return hevi


def _gpu(hv, q, steps, dtype, layout="kij", tile_x=16):
    """q canonical (nz, ny, nx) float64; returns canonical float64."""
    import torch
    host = np.ascontiguousarray(np.transpose(q, (1, 2, 0)) if layout == "kij" else q)
    a = torch.from_numpy(host).to(dtype).cuda()
    b = torch.empty_like(a)
    for _ in range(steps):
        hv.diffuse(a, b, *K, layout=layout, tile_x=tile_x)
        a, b = b, a
    torch.cuda.synchronize()
    out = a.double().cpu().numpy()
    return np.ascontiguousarray(np.transpose(out, (2, 0, 1))) if layout == "kij" else out


def _field(nz, ny, nx, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(nz, ny, nx)) + 5.0


@pytest.mark.parametrize("nz,ny,nx", [(32, 13, 7), (64, 20, 33), (128, 9, 16)])
@pytest.mark.parametrize("layout", ["kij", "ijk"])
def test_fp64_bitwise_equal_to_oracle(hv, oracle, nz, ny, nx, layout):
    import torch
    q = _field(nz, ny, nx, nz + nx)
    print(f"case: diffusion fp64 {nz}x{ny}x{nx} {layout}", flush=True)
    ref = oracle.diffuse(q, *K, steps=3)
    got = _gpu(hv, q, 3, torch.float64, layout)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("layout", ["kij", "ijk"])
def test_fp32_within_rounding_of_oracle(hv, oracle, layout):
    import torch
    q = _field(64, 24, 40, 5)
    q32 = q.astype(np.float32).astype(np.float64)
    steps = 4
    ref = oracle.diffuse(q32, *K, steps=steps)
    got = _gpu(hv, q, steps, torch.float32, layout)
    assert np.abs(got - ref).max() <= steps * 4 * 2.0 ** -24 * np.abs(q).max()


def test_tiles_and_layouts_bitwise(hv):
    import torch
    q = _field(32, 17, 21, 9)
    a = _gpu(hv, q, 2, torch.float32, "kij", 16)
    for lay, t in (("kij", 8), ("kij", 4), ("ijk", 16), ("ijk", 4)):
        assert np.array_equal(_gpu(hv, q, 2, torch.float32, lay, t), a), (lay, t)


def test_full_size_step_matches_oracle(hv, oracle):
    """1024 x 1024 x 64, the size of the benchmark, one float32 step."""
    import torch
    print("case: diffusion 1024x1024x64 fp32", flush=True)
    rng = np.random.default_rng(11)
    q = (rng.random((64, 1024, 1024)) + 1.0).astype(np.float32).astype(np.float64)
    ref = oracle.diffuse(q, *K, steps=1)
    got = _gpu(hv, q, 1, torch.float32, "kij")
    assert np.abs(got - ref).max() <= 4 * 2.0 ** -24 * 2.0
