"""Parity of the whole solve at the largest workload: the 327,680-triangle
star surface with 10,000 interior charges (the benchmark's headline input).

The oracle cannot solve a system of 655,360 unknowns in test time, so the
FP64 GPU solution is checked through properties that hold at any size:
* it satisfies the oracle's own discretised equations (eqs. eqbim_5/eqbim_6,
  oracle matvec and sources) on 64 sampled rows of each block;
* the oracle's energy quadrature (eq. solvation_energy) of it, a full
  N x N_c = 3.3e9-pair sum, equals the GPU energy;
* the refined-FP32 solve (the benchmarked path) gives the same energy within
  1e-6, in both the plain and the preconditioned configuration.
"""
import numpy as np
import pytest

import synth
from oracle import dsbi

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def test_largest_workload_solve_against_oracle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_10044_amd as m

    w = synth.large_star_protein()
    assert w.n_tri == 327680 and w.n_charges == 10000
    _say(f"largest workload: {w.n_tri} triangles, {w.n_charges} charges")
    base = dict(eps_in=w.eps_in, eps_out=w.eps_out, kappa=w.kappa, restart=10, max_iter=3000)
    with m.Context(0) as ctx:
        info64, phi, dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                                         m.Params(tol=1e-12, **base))
        _say(f"  fp64 tol 1e-12: E={info64.e_solv:.12f} iters={info64.iters} "
             f"t={info64.seconds:.2f}s")
        assert info64.status == m.PB_OK
        g = dsbi.geometry(w.verts, w.tris)
        rows = np.sort(np.random.default_rng(33).choice(w.n_tri, 64, replace=False))
        xi = np.concatenate([phi, dphi])
        y1, y2 = dsbi.matvec(g, w.eps_out / w.eps_in, w.kappa, xi, rows=rows)
        b1, b2 = dsbi.source(g, w.pos, w.q, w.eps_in, rows=rows)
        bn = np.abs(np.concatenate([b1, b2])).max()
        res = np.abs(np.concatenate([y1 - b1, y2 - b2])).max() / bn
        _say(f"  oracle residual on {len(rows)} rows per block: {res:.3e} of max|b|")
        assert res <= 1e-9
        e_orc = dsbi.energy(g, w.eps_out / w.eps_in, w.kappa, xi, w.pos, w.q)
        _say(f"  oracle energy of the GPU solution: {e_orc:.12f} "
             f"(rel diff {abs(e_orc - info64.e_solv) / abs(e_orc):.2e})")
        assert abs(e_orc - info64.e_solv) <= 1e-11 * abs(e_orc)
        for leaf in (0, 24):
            info32, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                                          m.Params(tol=1e-7, precision=m.PB_FP32_IR,
                                                   inner_tol=1e-8, precond_leaf=leaf, **base))
            rel = abs(info32.e_solv - info64.e_solv) / abs(info64.e_solv)
            _say(f"  fp32-ir leaf {leaf}: E={info32.e_solv:.12f} rel={rel:.2e} "
                 f"mv32={info32.matvecs_fp32} mv64={info32.matvecs_fp64} "
                 f"t={info32.seconds:.2f}s")
            assert info32.status == m.PB_OK
            assert rel <= 1e-6
