"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle source is built into a small driver (tests/oracle_sanitize_driver.c)
with gcc's address and undefined-behaviour checks, run on small D2Q9 and
D3Q19 fields for each cubic, and its densities compared with the regular
oracle library on the same input: any out-of-bounds access, use after free
or undefined arithmetic aborts the driver.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from inputs import components as C
from tests import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "oracle_sanitize_driver.c")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("san") / "oracle_san")
    cmd = [gcc, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fopenmp"] + SAN + [DRIVER, "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-300:])
    return exe


@pytest.mark.parametrize("eos", ["PR", "SRK", "vdW"])
@pytest.mark.parametrize("lattice,shape,N", [(0, (13, 7), 3), (1, (6, 5, 4), 2)])
def test_oracle_clean_under_sanitizers(driver, eos, lattice, shape, N):
    from oracle.lbm import EOS_CODE
    wl = W.random_droplet(N, shape, seed=3, lattice=lattice, eos=eos)
    o = wl.oracle()
    m = o.mix
    steps = 20
    nx, ny, nz = (tuple(shape) + (1, 1))[:3]
    vals = [lattice, N, nx, ny, nz, EOS_CODE[eos], m.tau, m.RT, m.pr.d1, m.pr.d2, steps]
    vals += list(m.pr.b) + list(m.M) + list(m.sqk) + list(m.pr.aij.ravel())
    vals += list(np.asarray(wl.rho, dtype=np.float64).ravel())
    inp = "\n".join("%.17g" % v for v in vals) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([driver], input=inp, capture_output=True, text=True, env=env, timeout=120)
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    assert r.returncode == 0, r.stderr[-2000:]
    got = np.array([float(v) for v in r.stdout.split()])
    assert o.run(steps) == 0
    np.testing.assert_allclose(got, o.rho().ravel(), rtol=1e-13, atol=0)
