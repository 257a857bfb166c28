"""pb_matvec_dev_noalloc: the matvec on device arrays with no device
allocation (a fixed library scratch array per GPU), against pb_matvec_dev and
the oracle, on two calls in a row with the second surface smaller.

Bars (as for every matvec): |dy_i| <= bar * S_i with S_i the oracle's sum of
|terms| of row i, bar = 1e-14 (FP64) or 5e-5 (FP32); the two entry points use
different sweeps (per-target against pairwise), so they agree to twice the bar.
The context's device scratch stays at zero bytes: the call takes nothing from
it.
"""
import numpy as np
import pytest

import synth
from oracle import dsbi

pytestmark = pytest.mark.gpu

BARS = {0: 1e-14, 1: 5e-5}


def _say(msg):
    print(msg, flush=True)


def test_noalloc_matvec_matches_the_allocating_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_10044_amd as m

    dev = torch.device("cuda:0")
    big = synth.star_protein(freq=12, r0=10.0, n_charges=1, seed=41)    # 2,880 triangles
    small = synth.kirkwood_sphere(freq=8)                               # 1,280 triangles
    with m.Context(0) as ctx_na, m.Context(0) as ctx_ref:
        assert ctx_na.memory_used() == 0
        for w in (big, small):
            g = dsbi.geometry(w.verts, w.tris)
            tv = torch.from_numpy(w.verts).to(dev)
            tt = torch.from_numpy(w.tris.astype(np.int32)).to(dev)
            x = np.random.default_rng(w.n_tri).normal(size=2 * w.n_tri)
            tx = torch.from_numpy(x).to(dev)
            for precision in (m.PB_FP64, m.PB_FP32_IR):
                for transpose in (False, True):
                    P = m.Params(kappa=w.kappa)
                    _say(f"noalloc: {w.n_tri} triangles precision={precision} "
                         f"transpose={transpose}")
                    y_na = torch.full_like(tx, float("nan"))
                    y_ref = torch.empty_like(tx)
                    torch.cuda.synchronize()
                    ctx_na.pb_matvec_dev_noalloc(tv, tt, tx, y_na, P, transpose=transpose,
                                                 precision=precision)
                    ctx_ref.pb_matvec_dev(tv, tt, tx, y_ref, P, transpose=transpose,
                                          precision=precision)
                    a = y_na.cpu().numpy()
                    b = y_ref.cpu().numpy()
                    y1, y2, s1, s2 = dsbi.matvec(g, w.eps_out / w.eps_in, w.kappa, x,
                                                 rows=np.arange(g.n), transpose=transpose,
                                                 with_abs=True)
                    S = np.concatenate([s1, s2])
                    ref = np.concatenate([y1, y2])
                    bar = BARS[precision]
                    e_ref = np.max(np.abs(a - b) / S)
                    e_orc = np.max(np.abs(a - ref) / S)
                    _say(f"  vs pb_matvec_dev {e_ref:.2e}, vs oracle {e_orc:.2e}")
                    assert np.all(np.isfinite(a))
                    assert e_ref <= 2 * bar
                    assert e_orc <= bar
        # nothing came from the context's own (allocating) scratch
        assert ctx_na.memory_used() == 0
        # beyond the fixed scratch: a clear error, and the next call still works
        over = synth.star_protein(freq=41, r0=20.0, n_charges=1, seed=3)
        assert over.n_tri > 32768
        tv = torch.from_numpy(over.verts).to(dev)
        tt = torch.from_numpy(over.tris.astype(np.int32)).to(dev)
        tx = torch.zeros(2 * over.n_tri, dtype=torch.float64, device=dev)
        ty = torch.empty_like(tx)
        with pytest.raises(m.PbError) as e:
            ctx_na.pb_matvec_dev_noalloc(tv, tt, tx, ty, m.Params())
        assert e.value.status == m.PB_ERR_ARG and "at most 32768" in e.value.message
        tv = torch.from_numpy(small.verts).to(dev)
        tt = torch.from_numpy(small.tris.astype(np.int32)).to(dev)
        tx = torch.ones(2 * small.n_tri, dtype=torch.float64, device=dev)
        ty = torch.empty_like(tx)
        ctx_na.pb_matvec_dev_noalloc(tv, tt, tx, ty, m.Params())
        assert torch.isfinite(ty).all()
        assert ctx_na.memory_used() == 0
