"""The pair sweeps at the paper's largest surface size: a star surface of
1,003,520 triangles (the paper's largest protein surface, Table tb_proteins,
has 993,572 elements), 3,920 tiles, 7.7 million tile pairs.  The default FP32
sweep (XCD-aware plan, 16 strips) and the FP64 sweep, forward, and the FP32
sweep transposed, against the oracle on sampled rows of both blocks.  The
FP64 sweep's partial records alone take 31 GB here."""
import numpy as np
import pytest

import synth
from oracle import dsbi

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-14   # |dy_i| / S_i
FP32_BAR = 5e-5


def test_sweeps_at_the_largest_size():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_10044_amd as m

    w = synth.star_protein(freq=224, r0=70.0, n_charges=200, seed=7)
    assert w.n_tri == 1003520
    print(f"largest size: {w.n_tri} triangles", flush=True)
    g = dsbi.geometry(w.verts, w.tris)
    x = np.random.default_rng(5).normal(size=2 * g.n)
    rows = np.sort(np.random.default_rng(6).choice(g.n, 24, replace=False))
    p = m.Params(eps_in=w.eps_in, eps_out=w.eps_out, kappa=w.kappa)
    eps = w.eps_out / w.eps_in
    with m.Context(0) as ctx:
        for precision, transpose, bar in ((0, False, FP64_BAR), (1, False, FP32_BAR),
                                          (1, True, FP32_BAR)):
            y = ctx.pb_matvec(w.verts, w.tris, x, p, transpose=transpose, precision=precision)
            y1, y2, s1, s2 = dsbi.matvec(g, eps, w.kappa, x, rows=rows, transpose=transpose,
                                         with_abs=True)
            err = max((np.abs(y[rows] - y1) / s1).max(), (np.abs(y[g.n + rows] - y2) / s2).max())
            print(f"  precision={precision} transpose={transpose}: max |dy|/S = {err:.3e} "
                  f"on {len(rows)} rows per block; device memory held "
                  f"{ctx.memory_used() / 1e9:.1f} GB", flush=True)
            assert np.all(np.isfinite(y))
            assert err <= bar
