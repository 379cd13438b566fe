"""The seeded input generator (host C code) built with AddressSanitizer and
UndefinedBehaviorSanitizer: every generator runs clean on a small lattice and gives the same
numbers as the library the tests load."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import gen

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _weighted(a):
    a = np.ascontiguousarray(a).view(np.float64).reshape(-1) if np.iscomplexobj(a) else np.asarray(a).reshape(-1)
    w = (np.arange(a.size) % 7 + 1).astype(np.float64)
    return float(np.sum(a * w))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_generator_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "gen_sanitized")
    cmd = ["gcc", "-O1", "-g", "-fopenmp", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", os.path.join(ROOT, "gen", "gen.c"), os.path.join(HERE, "gen_sanitized_main.c"),
           "-o", exe, "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    env.pop("LD_PRELOAD", None)
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, out.stderr
    got = dict(line.split(" ", 1) for line in out.stdout.strip().splitlines())
    dims = (2, 4, 2, 6)
    assert [int(v) for v in got["philox"].split()] == list(gen.philox4x32_10([1, 2, 3, 4], [5, 6]))
    want = {"su3": _weighted(gen.su3_field(dims, 0.5, 11)), "u1": _weighted(gen.u1_field(dims, 0.3, 11)),
            "spinor": _weighted(gen.gaussian_spinor(dims, 12, 3)),
            "omega": _weighted(gen.gauge_transform(dims, 13)[0]), "lambda": _weighted(gen.gauge_transform(dims, 13)[1]),
            "uniform": _weighted(gen.uniforms(1000, 14, 99))}
    for k, v in want.items():
        assert float(got[k]) == pytest.approx(v, rel=1e-14, abs=1e-12), k
