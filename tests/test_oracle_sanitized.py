"""The C oracle under the host sanitizers: oracle/lqoracle.c built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code only) into a
small driver that computes the clover field, D, D^dag, H and the site-block
inverses on lattices with L_mu = 2 directions (coincident neighbours) and
on a larger one.  The run must end cleanly (any report aborts it) and give
the values of the ordinary oracle build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from lattice_inputs import ANTIPERIODIC_T, gauge_exp, gaussian_spinor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_driver")
    cmd = [gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", os.path.join(HERE, "sanitize", "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "lqoracle.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("dims,kappa,csw", [((2, 2, 2, 2), 0.12, 1.0), ((2, 4, 2, 6), 0.13, 1.7),
                                            ((4, 4, 4, 8), 0.1355, 1.7)])
def test_oracle_under_asan_ubsan(driver, tmp_path, dims, kappa, csw):
    U = gauge_exp(dims, 0.5, 1401)
    psi = gaussian_spinor(dims, 2401)
    V = int(np.prod(dims))
    src = tmp_path / "in.bin"
    with open(src, "wb") as f:
        f.write(np.asarray(dims, dtype=np.int32).tobytes())
        f.write(np.asarray([kappa, csw], dtype=np.float64).tobytes())
        f.write(np.asarray([(c.real, c.imag) for c in np.asarray(ANTIPERIODIC_T, dtype=complex)],
                           dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(U, dtype=np.complex128).tobytes())
        f.write(np.ascontiguousarray(psi, dtype=np.complex128).tobytes())
    out = tmp_path / "out.bin"
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, str(src), str(out)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    raw = np.fromfile(out, dtype=np.complex128, count=V * (144 + 12 * 3 + 144))
    F, rest = raw[:V * 144], raw[V * 144:]
    d, dd, h, Ainv = rest[:V * 12], rest[V * 12:2 * V * 12], rest[2 * V * 12:3 * V * 12], rest[3 * V * 12:]
    Fr = oracle.clover(dims, U, csw, kappa)
    assert np.allclose(F, Fr.reshape(-1), rtol=0, atol=1e-14)
    for got, want in ((d, oracle.dirac(dims, U, ANTIPERIODIC_T, kappa, psi, F=Fr)),
                      (dd, oracle.dirac(dims, U, ANTIPERIODIC_T, kappa, psi, F=Fr, dagger=True)),
                      (h, oracle.hop(dims, U, ANTIPERIODIC_T, psi))):
        want = np.asarray(want).reshape(-1)
        assert np.linalg.norm(got - want) <= 1e-14 * np.linalg.norm(want)
    # (1 + F)^-1 (1 + F) = 1 block by block
    A = Fr.reshape(V, 12, 12) + np.eye(12)
    assert np.abs(np.einsum("xij,xjk->xik", Ainv.reshape(V, 12, 12), A) - np.eye(12)).max() < 1e-12
