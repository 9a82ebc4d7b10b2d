"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code
only).  A copy of oracle/st_oracle.c and st_oracle_par.c is compiled with
both sanitizers, every pin runs against it in a child process, and so does a
run of the OpenMP drivers against the serial functions: an out-of-bounds
access, a use after free or undefined behaviour anywhere on those paths ends
the child with a sanitizer report instead of passing."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


PAR_CHECK = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[2])
sys.path.insert(0, sys.argv[3])
from oracle.oracle import MeshParams, load
from workloads import synth
orc = load(sys.argv[1])
w = synth.get("tg32")
x, up, d = w.particles(3000)
U = w.field()
m = MeshParams(**w.mesh_kwargs())
a = orc.run(m, U, x, up, d, w.dt, 3)
b = orc.run_par(m, U, x, up, d, w.dt, 3, threads=4)
assert all(np.allclose(p, q, rtol=0, atol=1e-12 * max(1.0, float(np.abs(p).max())))
           for p, q in zip(a, b))
lam = np.random.default_rng(1).normal(size=(3,) + tuple(w.n[::-1]))
g1 = orc.adjoint(m, U, x, up, d, w.dt, 3, lam)
g2 = orc.adjoint_run_par(m, U[None], np.zeros(3, np.int32), np.full(3, w.dt), 1, x, up, d,
                         lam, threads=4)
for p, q in zip(g1, g2):
    p, q = np.asarray(p).ravel(), np.asarray(q).ravel()
    assert np.allclose(p, q, rtol=1e-12, atol=1e-12 * max(1e-300, float(np.abs(p).max())))
print("PAR_OK")
"""


@pytest.mark.skipif(not (_runtime("libasan.so") and _runtime("libubsan.so")),
                    reason="gcc's sanitizer runtimes are not installed")
def test_oracle_clean_under_sanitizers():
    env = dict(os.environ)
    env["LD_PRELOAD"] = f"{_runtime('libasan.so')} {_runtime('libubsan.so')}"
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    with tempfile.TemporaryDirectory() as tmp:
        shutil.copy(os.path.join(ROOT, "oracle", "st_oracle.h"), tmp)
        lib = os.path.join(tmp, "libst_oracle_san.so")
        subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fopenmp", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                        os.path.join(ROOT, "oracle", "st_oracle.c"),
                        os.path.join(ROOT, "oracle", "st_oracle_par.c"),
                        "-I", tmp, "-o", lib, "-lm"], check=True, capture_output=True)
        r = subprocess.run([sys.executable, os.path.join(HERE, "oracle_pins.py"), lib],
                           capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0 and r.stdout.strip().splitlines()[-1] == "ALL_PASSED", \
            (r.stdout[-2000:], r.stderr[-4000:])
        r = subprocess.run([sys.executable, "-c", PAR_CHECK, lib, ROOT, HERE],
                           capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0 and "PAR_OK" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
