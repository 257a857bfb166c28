"""Adjoint forces on the GPU: transpose matvec, adjoint GMRES and gradient
sweep against the oracle's adjoint, against central finite differences of
the GPU energy, and through torch.autograd."""
import numpy as np
import pytest

import synth
from oracle import dsbi

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def pb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_10044_amd as m
    ctx = m.Context(0, torch.cuda.current_stream())
    yield m, ctx
    ctx.close()


def test_forces_match_oracle_adjoint(pb):
    m, ctx = pb
    w = synth.star_protein(freq=12, r0=10.0, n_charges=300, seed=41)
    _say(f"forces vs oracle: {w.n_tri} triangles, {w.n_charges} charges")
    sol = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-12)
    dpos_ref, dq_ref, _lam, _ = dsbi.forces(sol, w.pos, w.q, tol=1e-12)
    info, dpos, dq = ctx.pb_forces(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-12))
    assert info.status == m.PB_OK and info.adjoint_iters > 0
    assert abs(info.e_solv - sol.e_solv) <= 1e-10 * abs(sol.e_solv)
    assert np.abs(dpos - dpos_ref).max() <= 1e-8 * np.abs(dpos_ref).max()
    assert np.abs(dq - dq_ref).max() <= 1e-8 * np.abs(dq_ref).max()


def test_forces_fp32_ir_close_to_fp64(pb):
    m, ctx = pb
    w = synth.star_protein(freq=12, r0=10.0, n_charges=300, seed=41)
    i64, p64, q64 = ctx.pb_forces(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-12))
    i32, p32, q32 = ctx.pb_forces(w.verts, w.tris, w.pos, w.q,
                                  m.Params(tol=1e-8, precision=m.PB_FP32_IR, inner_tol=1e-4))
    assert i32.status == m.PB_OK and i32.refinements >= 2
    assert np.abs(p32 - p64).max() <= 1e-5 * np.abs(p64).max()
    assert np.abs(q32 - q64).max() <= 1e-5 * np.abs(q64).max()


def test_forces_full_size_against_central_differences(pb):
    """81,920-triangle star, 2,000 charges: dE/dy_k on 16 seeded charges
    against (E(y+h e_c) - E(y-h e_c)) / 2h, h = 1e-4 A, FP64 solves at 1e-12.
    Criterion: max_k |F_adj - F_fd| / max_k |F_fd| <= 1e-4."""
    import torch
    m, ctx = pb
    w = synth.star_protein()
    dev = torch.device("cuda:0")
    tv = torch.from_numpy(w.verts).to(dev)
    tt = torch.from_numpy(w.tris.astype(np.int32)).to(dev)
    tq = torch.from_numpy(w.q).to(dev)
    P = m.Params(tol=1e-12, max_iter=3000)
    tp = torch.from_numpy(w.pos).to(dev)
    gpos = torch.empty_like(tp)
    gq = torch.empty_like(tq)
    info = ctx.pb_forces_dev(tv, tt, tp, tq, P, gpos, gq)
    assert info.status == m.PB_OK
    _say(f"forces full size: E={info.e_solv:.10f} iters={info.iters} adj={info.adjoint_iters} "
         f"t={info.seconds:.2f}s")
    ks = np.random.default_rng(4).choice(w.n_charges, 16, replace=False)
    h = 1e-4
    F_adj = gpos.cpu().numpy()[ks]
    F_fd = np.zeros_like(F_adj)
    for a, k in enumerate(ks):
        for c in range(3):
            pp = w.pos.copy()
            pp[k, c] += h
            ep = ctx.pb_solve_dev(tv, tt, torch.from_numpy(pp).to(dev), tq, P).e_solv
            pp[k, c] -= 2 * h
            em = ctx.pb_solve_dev(tv, tt, torch.from_numpy(pp).to(dev), tq, P).e_solv
            F_fd[a, c] = (ep - em) / (2 * h)
        _say(f"  charge {k}: adj {F_adj[a]} fd {F_fd[a]}")
    err = np.abs(F_adj - F_fd).max() / np.abs(F_fd).max()
    _say(f"  max rel err {err:.2e}")
    assert err <= 1e-4


def test_autograd_function(pb):
    import torch
    from paper_2312_10044_amd.autograd import pb_energy
    m, ctx = pb
    w = synth.star_protein(freq=8, r0=8.0, n_charges=20, seed=12)
    dev = torch.device("cuda:0")
    tv = torch.from_numpy(w.verts).to(dev)
    tt = torch.from_numpy(w.tris.astype(np.int32)).to(dev)
    pos = torch.from_numpy(w.pos).to(dev).requires_grad_(True)
    q = torch.from_numpy(w.q).to(dev).requires_grad_(True)
    P = m.Params(tol=1e-12)
    E = pb_energy(tv, tt, pos, q, ctx, P)
    (2.0 * E).backward()
    info, dpos, dq = ctx.pb_forces(w.verts, w.tris, w.pos, w.q, P)
    assert float(E.detach()) == pytest.approx(info.e_solv, rel=1e-14)
    assert np.allclose(pos.grad.cpu().numpy(), 2.0 * dpos, rtol=1e-13, atol=0)
    assert np.allclose(q.grad.cpu().numpy(), 2.0 * dq, rtol=1e-13, atol=0)
    with torch.no_grad():
        E2 = pb_energy(tv, tt, pos, q, ctx, P)
    assert float(E2) == pytest.approx(info.e_solv, rel=1e-12)


def test_autograd_function_raises_when_not_converged(pb):
    """An unconverged forward or adjoint solve is an error, not an energy."""
    import torch
    from paper_2312_10044_amd.autograd import pb_energy
    m, ctx = pb
    w = synth.star_protein(freq=8, r0=8.0, n_charges=20, seed=12)
    dev = torch.device("cuda:0")
    tv = torch.from_numpy(w.verts).to(dev)
    tt = torch.from_numpy(w.tris.astype(np.int32)).to(dev)
    pos = torch.from_numpy(w.pos).to(dev).requires_grad_(True)
    q = torch.from_numpy(w.q).to(dev)
    _say("autograd: max_iter 1 must raise")
    for grad in (True, False):
        with torch.set_grad_enabled(grad):
            with pytest.raises(m.PbError) as e:
                pb_energy(tv, tt, pos, q, ctx, m.Params(tol=1e-12, max_iter=1))
        assert e.value.status == m.PB_NOT_CONVERGED
    # the context still solves afterwards
    E = pb_energy(tv, tt, pos, q, ctx, m.Params(tol=1e-10))
    assert np.isfinite(float(E.detach()))
