"""AddressSanitizer builds of the host code, run on the CPU:

- the oracle (plain C) built with gcc -fsanitize=address,undefined and driven
  through its Python binding over every exported routine on small grids
  (flat and over hills, forward-backward and Runge-Kutta short steps,
  damping, the binary32-storage twin, sums, diffusion, single faces, the
  Thomas solver, forward-Euler advection);
- the library's host runtime (argument checking and workspace planning of
  the C ABI) built with hipcc, sanitizer on the host code only, with the
  kernel launchers replaced by failing stubs, driven by
  tests/asan/host_abi_main.cpp through calls that return before any device
  call.
A sanitizer report aborts the child process, which fails the test.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))

ORACLE_SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
from oracle import oracle
oracle.LIB = {lib!r}
from paper_1710_08616_amd import inputs
s = inputs.make_state(8, 6, 32, seed=3, noise=0.5, n_short=2)
oracle.step(s, n_long=2)
oracle.step(s, n_long=1, short_rk2=True)
oracle.step(s.as_f32(reference=True), n_long=1, f32_storage=True, short_rk2=True)
h = inputs.orography(8, 6, 2000.0, 2000.0, 3, hmax=800.0, hills=2, smin=4000.0, smax=6000.0)
t = inputs.make_state(8, 6, 64, seed=4, terrain=h, noise=0.5, shear=10.0, n_short=2)
oracle.step(t, n_long=2)
oracle.step(t, n_long=1, short_rk2=True)
t.damping = inputs.damping(t, width=2, t2=40.0)
oracle.step(t, n_long=1)
oracle.step(t, n_long=1, short_rk2=True)
sl = oracle.slow_sweep(s)
oracle.short_step(s, sl, 1.0)
oracle.slow_sweep(s, donor_cell=True)
assert np.isfinite(oracle.mass(s)) and np.isfinite(oracle.energy(s)) and np.isfinite(oracle.energy(t))
q = np.random.default_rng(0).random((32, 6, 8)) + 1.0
oracle.diffuse(q, 0.1, 0.1, 0.1, steps=2)
n = 9
x, rc = oracle.thomas(np.full(n, -1.0), np.full(n, 4.0), np.full(n, -1.0), np.arange(n, dtype=float))
assert rc == 0
u = np.full((32, 6, 8), 1.0)
w = np.zeros((33, 6, 8))
oracle.advect_fe(s, q, u, u, w, 10.0, oracle.LIM_KOREN)
for r in (-1.0, 0.0, 0.5, 4.0):
    oracle.koren_phi(1.0, r)
    oracle.face(0.0, 1.0, 2.0 + r, 3.0, -1.0)
print("ok")
"""


def _run(cmd, env=None, timeout=600):
    return subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=timeout)


def test_oracle_under_address_sanitizer(tmp_path):
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc has no AddressSanitizer runtime")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                           "-shared", "-fPIC", "-o", lib, os.path.join(ROOT, "oracle", "hevi_oracle.c"),
                           "-lm"])
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = _run([sys.executable, "-c", ORACLE_SCRIPT.format(root=ROOT, lib=lib)], env=env)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-4000:]


def test_host_runtime_under_address_sanitizer(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc):
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "host_abi_asan")
    csrc = os.path.join(ROOT, "paper_1710_08616_amd", "csrc")
    r = _run([hipcc, "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address",
              "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
              "-I", csrc, "-o", exe, os.path.join(csrc, "hevi_runtime.cpp"),
              os.path.join(HERE, "asan", "host_abi_main.cpp")])
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = _run([exe], env=env, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().startswith("ok"), (r.stdout + r.stderr)[-4000:]
