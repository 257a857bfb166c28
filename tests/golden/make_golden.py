"""Write stored oracle results for the parity tests.

Calls only ``oracle`` and ``synth``: every stored number comes from the FP64
CPU oracle on the seeded synthetic input named in the file, together with the
SHA-256 digest of that input so a test can confirm it regenerated the same
arrays.

    python tests/golden/make_golden.py kirkwood   # 1,280 triangles, seconds
    python tests/golden/make_golden.py star       # 81,920 triangles, ~1-2 h on 8 cores
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import dsbi  # noqa: E402


def _record(w, tol, n_sample, seed):
    t0 = time.time()
    s = dsbi.solve(w.verts, w.tris, w.pos, w.q, eps_in=w.eps_in, eps_out=w.eps_out,
                   kappa=w.kappa, tol=tol, restart=10, max_iter=5000)
    n = s.geom.n
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=min(n_sample, n), replace=False))
    return {
        "workload": w.name,
        "digest": synth.input_digest(w),
        "n_tri": n,
        "n_charges": w.n_charges,
        "eps_in": w.eps_in, "eps_out": w.eps_out, "kappa": w.kappa,
        "gmres": {"restart": 10, "tol": tol, "iters": s.info.iters,
                  "matvecs": s.info.matvecs, "rel_residual": s.info.rel_residual,
                  "converged": s.info.converged},
        "e_solv": s.e_solv,
        "sample_index": idx.tolist(),
        "phi": s.xi[idx].tolist(),
        "dphi": s.xi[n + idx].tolist(),
        "b1": s.b[idx].tolist(),
        "b2": s.b[n + idx].tolist(),
        "oracle_seconds": time.time() - t0,
        "threads": os.environ.get("OMP_NUM_THREADS", str(os.cpu_count())),
    }


def main(which):
    if which == "kirkwood":
        rec = _record(synth.kirkwood_sphere(), 1e-12, 64, 101)
        path = os.path.join(HERE, "kirkwood_f8.json")
    elif which == "star":
        rec = _record(synth.star_protein(), 1e-12, 256, 102)
        path = os.path.join(HERE, "star_f64_s2.json")
    else:
        raise SystemExit("usage: make_golden.py kirkwood|star")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(path, rec["e_solv"], rec["gmres"])


if __name__ == "__main__":
    main(sys.argv[1])
