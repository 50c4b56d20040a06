"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle4.c is built with gcc together with a small driver (tests/oracle_asan_driver.c) that
reads the arguments of oracle_rates4 from files, so that no Python process has to load the
sanitizer runtimes.  The driver runs on sampled modes of the 3x3x3 workload and on a ragged
2x3x2 grid; the run must end with no sanitizer report (errors are fatal, leaks reported) and
give the same counts and rates as the regular build called through ctypes.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fcx-limited-range", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "oracle4.c"),
           os.path.join(HERE, "oracle_asan_driver.c"), "-o", out, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtimes not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return out


def _write(d, name, arr, dtype):
    np.ascontiguousarray(arr, dtype=dtype).tofile(os.path.join(d, name))


@pytest.mark.parametrize("case", ["small", "ragged"])
def test_oracle_clean_under_sanitizers(driver, tmp_path, case):
    if case == "small":
        inst = synth.small()
        targets = np.arange(3, inst.nmodes, 7, dtype=np.int32)
        T, sb, mask = [300.0], 1.0, 7
    else:
        inst = synth.diamond_instance((2, 3, 2), synth.configs.RC_SECOND, seed=5, T=(300.0, 900.0))
        targets = np.arange(3, inst.nmodes, dtype=np.int32)
        T, sb, mask = [300.0, 900.0], 0.8, 5
    m = oracle.Model.from_instance(inst)
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    d = str(tmp_path)
    _write(d, "grid.i32", m.grid, np.int32)
    _write(d, "ints.i32", [m.natoms, m.atoms.shape[0], len(T), mask, targets.size], np.int32)
    _write(d, "scal.f64", [sb, 2.0, 1e-4, dq], np.float64)
    for name, arr, dt in (("mass.f64", m.mass, np.float64), ("omega.f64", m.omega, np.float64),
                          ("evec.f64", m.evec, np.float64), ("vel.f64", m.vel, np.float64),
                          ("atoms.i32", m.atoms, np.int32), ("cells.i32", m.cells, np.int32),
                          ("phi.f64", m.phi, np.float64), ("T.f64", T, np.float64),
                          ("targets.i32", targets, np.int32)):
        _write(d, name, arr, dt)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([driver, d], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    rates = np.fromfile(os.path.join(d, "rates.f64")).reshape(len(T), targets.size)
    counts = np.fromfile(os.path.join(d, "counts.i64"), dtype=np.int64).reshape(targets.size, 3)
    r_ref, _, c_ref = oracle.rates4(m, T, sb, mask, dq, targets)
    assert np.array_equal(counts, c_ref)
    assert counts.sum() > 0
    np.testing.assert_allclose(rates, r_ref, rtol=1e-13, atol=0.0)
