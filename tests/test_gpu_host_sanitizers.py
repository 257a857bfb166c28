"""The library's host code under UndefinedBehaviorSanitizer on the GPU: a child
process loads libpbdsbi_hostubsan.so (host code built with -fsanitize=undefined
and the minimal runtime, aborting on the first report; device code as in the
product library) and runs every entry point on small inputs: FP64 and
refined-FP32 solves with both preconditioner kernels, forces, a batch with
forces, all FP32 sweep kinds, the treecode, leaves, potentials, and the error
paths (non-finite vertex, coincident centroids, kappa out of range, memory
cap, iteration cap).  A sanitizer report aborts the child; energies are
checked against the oracle."""
import json
import os
import subprocess
import sys

import pytest

import synth
from oracle import dsbi
from test_host_sanitizers import ROOT, sanitized_library_env

pytestmark = pytest.mark.gpu


def test_every_entry_point_under_host_sanitizers():
    w = synth.kirkwood_sphere(freq=8)
    star = synth.star_protein(freq=10, r0=8.0, n_charges=60, seed=43)
    expect = {
        "kirkwood": dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-12).e_solv,
        "star": dsbi.solve(star.verts, star.tris, star.pos, star.q, tol=1e-12).e_solv,
    }
    env = sanitized_library_env("ubsan")
    print(f"host-sanitized library, {w.n_tri} and {star.n_tri} triangles", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "hostsan_driver.py"), "gpu",
                        json.dumps(expect)], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-4000:], r.stderr[-4000:], flush=True)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "gpu ok" in r.stdout
