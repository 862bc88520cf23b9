"""The oracle's builds: the OpenMP build (the one every test and the CPU
baseline use) equals the serial build bit for bit, and an AddressSanitizer +
UndefinedBehaviorSanitizer build of the C source runs every entry point on
small problems without a finding."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2308_06152_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def both(ora):
    ora.build(force=False)
    ora.build(force=True, serial=True)
    return ora


def _problem(ora, nx, ny, bc, vark, cop, **kw):
    h = 1.0 / (max(nx, ny) - 1)
    k = inputs.random_field(ny, nx, 10.0, 30.0, seed=nx + ny) if vark else None
    return ora.Problem(nx, ny, h, h, bc=bc, k=k, kconst=0.0 if vark else 20.0, coarse_op=cop,
                       **kw)


CASES = [(65, 65, 0, False, 0), (97, 161, 1, True, 1), (129, 97, 1, False, 0),
         (77, 45, 0, True, 3)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}_bc{c[2]}_op{c[4]}" for c in CASES])
def test_threaded_oracle_equals_serial_build(both, case):
    ora = both
    P = _problem(ora, *case, coarse_mode=ora.CMODE_TOL, coarse_iters=200, coarse_restart=10)
    Pf = P.replace(coarse_mode=ora.CMODE_FIXED, coarse_iters=6)
    v = inputs.random_complex((P.ny, P.nx), 91)
    b = inputs.point_source(P.nx, P.ny, P.hx, P.hy, P.nx // 2, P.ny // 2)

    def run():
        out = [ora.helm_apply(P, v), ora.vcycle(P, v), ora.deflate_apply(Pf, v, 2)[0],
               ora.coarse_apply(P, ora.z_restrict(P, v))]
        x, info = ora.fgmres(P, b, restart=20, tol=1e-6, maxit=100)
        out += [x, np.array([info.iters, info.inner_total, info.relres])]
        xg, ig = ora.gcr(P, b, restart=20, tol=1e-6, maxit=100)
        out += [xg, np.array([ig.iters, ig.relres])]
        return out

    threaded = run()
    with ora.serial_build():
        serial = run()
    for a, s in zip(threaded, serial):
        assert np.array_equal(a, s)


@pytest.mark.slow
def test_oracle_sanitizer_build(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = tmp_path / "oracle_san"
    cmd = [gcc, "-O1", "-g", "-std=c99", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "oracle"), "-o", str(exe),
           os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "tests", "csrc", "oracle_sanitize_main.c"), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    assert "PASS: 0 failed calls" in p.stdout
