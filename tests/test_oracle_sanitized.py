"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, CPU only): a driver runs its right-hand side, Jacobian-vector product,
production rates and per-cell right-hand side on a small ragged box for each
species-diffusion and stencil option, must finish without a sanitizer
report, and must give exactly the regular build's results."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from synth import fields, mechanism

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    out = tmp_path_factory.mktemp("asan") / "oracle_asan"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "native", "oracle_sanitized_main.cpp"), os.path.join(ROOT, "oracle", "oracle.cpp"),
           "-o", str(out)]
    subprocess.check_call(cmd)
    return str(out)


def _write_case(path, m, U, wU, wA, ref, wide, dx):
    ns, nr = int(m["ns"]), int(m["nr"])
    nz, ny, nx = U.shape[1:]
    with open(path, "wb") as f:
        np.array([ns, nr, nx, ny, nz, ref, int(wide), 0], dtype=np.int32).tofile(f)
        for key in ("W", "nasa", "A", "b", "Ea", "Le"):
            np.ascontiguousarray(m[key], dtype=np.float64).tofile(f)
        np.array([m["Tlo"], m["Thi"], m["mu_ref"], m["T_ref"], m["mu_exp"], m["Pr"], m["bulk_ratio"],
                  m["m47"], m["m48"], dx], dtype=np.float64).tofile(f)
        np.ascontiguousarray(m["nu_f"], dtype=np.int32).tofile(f)
        np.ascontiguousarray(m["nu_r"], dtype=np.int32).tofile(f)
        for a in (U, wU, wA):
            np.ascontiguousarray(a, dtype=np.float64).tofile(f)


@pytest.mark.parametrize("key,ref,wide", [("mech9le", -1, False), ("mech9le", 8, False),
                                          ("mech9le", -1, True), ("mech21", -1, False)])
def test_oracle_under_sanitizers(orc, driver, tmp_path, key, ref, wide):
    m = mechanism.load(key)
    om = orc.Mechanism(m, ref_species=ref, wide=wide)
    shape = (5, 6, 7)
    dx = 1e-4
    U = orc.prim_to_cons(om, fields.sines(shape, dx, om.ns, 9))
    rng = np.random.default_rng(3)
    wU = rng.standard_normal(U.shape) * np.abs(U).max(axis=(1, 2, 3), keepdims=True)
    wA = rng.standard_normal(om.nr)
    inp, outp = tmp_path / "case.bin", tmp_path / "out.bin"
    _write_case(inp, m, U, wU, wA, ref, wide, dx)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([driver, str(inp), str(outp)], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
    got = np.fromfile(outp, dtype=np.float64)
    nU, n = U.shape[0], U[0].size
    rhs, jvp = got[:nU * n].reshape(U.shape), got[nU * n:2 * nU * n].reshape(U.shape)
    prod = got[2 * nU * n:2 * nU * n + om.ns * n].reshape((om.ns,) + shape)
    cells = got[2 * nU * n + om.ns * n:].reshape(4, nU)
    np.testing.assert_array_equal(rhs, orc.rhs(om, U, dx))
    _, jref = orc.rhs_jvp(om, U, dx, wU, wA)
    np.testing.assert_array_equal(jvp, jref)
    np.testing.assert_array_equal(prod, orc.production(om, U))
    nz, ny, nx = shape
    cl = np.array([[0, 0, 0], [nx - 1, ny - 1, nz - 1], [nx // 2, 0, nz - 1], [1, ny // 2, nz // 2]])
    np.testing.assert_array_equal(cells, orc.rhs_cells(om, U, dx, cl))
