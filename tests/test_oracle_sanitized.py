"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer.

The C oracle is compiled a second time with ``-fsanitize=address,undefined``
(every error fatal) and driven through its Python binding, in a child
process with the sanitizer runtime preloaded, over small inputs that reach
every entry point: keys, stable sort, cell table, brute-force and k-d tree
searches, the band and root solves with their failure flags, exact K, the
scatter form, the adjoint and the pressure force, on periodic and grouped
sets.  A heap overflow, a use after free, a signed overflow, a shift out of
range or a misaligned access ends the child with an error report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sph_oracle.c")

DRIVER = r"""
import numpy as np
import oracle, sphgen
sets = [sphgen.uniform(700, seed=71, n_target=32.0, n_tol=1.0),
        sphgen.plummer_mixture(1500, 4, seed=72, n_target=32.0, n_tol=1.0),
        sphgen.groups(6, seed=73, sizes=np.array([0, 1, 40, 300, 2, 500]), n_target=16.0,
                      n_tol=1.0),
        sphgen.lattice(6, h=0.3, n_target=40.0)]
bad = sphgen.uniform(300, seed=74, n_target=32.0)
bad.x[5] = np.nan
bad.h_init[7] = -1.0
bad.y[9] = 1.5
sets.append(bad)
for ps in sets:
    o = oracle.sort(ps)
    assert o["cell_count"].sum() == ps.n
    for search in (0, 1):
        r = oracle.solve(ps, search=search)
        e = oracle.eval_at_h(ps, r["h"], search=search)
    oracle.solve(ps, mode=oracle.ROOT, root_tol=1e-9)
    oracle.solve(ps, max_iter=2)
    oracle.solve(ps, subset=np.arange(0, ps.n, 7))
    for kern in (oracle.M4, oracle.WENDLAND_C6):
        oracle.eval_at_h(ps, r["h"], kernel=kern)
        oracle.knn(ps, 12, kernel=kern)
        oracle.scatter(ps, r["h"], kernel=kern)
        gr = np.random.default_rng(1).standard_normal(ps.n)
        oracle.backward(ps, r["h"], gr, gr, kernel=kern)
    P = np.abs(r["rho"]) + 1.0
    oracle.pressure_force(ps, r["h"], np.where(np.isfinite(r["rho"]), r["rho"], 1.0), P)
print("sanitized oracle ok")
"""


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_asan_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for gcc on this host")
    lib = str(tmp_path / "liboracle_san.so")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-o", lib, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, LD_PRELOAD=asan, SPH_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", DRIVER], env=env, capture_output=True, text=True,
                       timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
