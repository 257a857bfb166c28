"""Block-diagonal leaf preconditioner on the GPU against the oracle.

Leaves of up to 32 elements are inverted by one wave (a row per lane), larger
ones (up to N0 = 100, the paper's leaf size, blocks of 200 x 200) by a whole
workgroup; both kernels are checked."""
import numpy as np
import pytest

import synth
from oracle import dsbi, precond

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_10044_amd as m
    ctx = m.Context(0)
    yield m, ctx
    ctx.close()


@pytest.fixture(scope="module")
def star12():
    return synth.star_protein(freq=12, r0=10.0, n_charges=300, seed=41)


@pytest.mark.parametrize("leaf", [1, 5, 16, 32, 48, 100])
def test_leaves_are_identical_to_the_oracle(pb, star12, leaf):
    m, ctx = pb
    w = star12
    got = ctx.pb_precond_leaves(w.verts, w.tris, leaf)
    ref = precond.leaves(dsbi.geometry(w.verts, w.tris).cen, leaf)
    assert len(got) == len(ref)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("leaf", [16, 48, 100])
def test_apply_matches_oracle(pb, star12, transpose, leaf):
    m, ctx = pb
    w = star12
    g = dsbi.geometry(w.verts, w.tris)
    M = precond.BlockDiagonal(g, 80.0, 0.1257, leaf)
    sizes = [len(idx) for idx in M.leaves]
    print(f"leaf {leaf}: {len(sizes)} leaves, largest {max(sizes)}", flush=True)
    if leaf > 32:
        assert max(sizes) > 32   # the workgroup inversion is exercised
    x = np.random.default_rng(3).normal(size=2 * g.n)
    y = ctx.pb_precond_apply(w.verts, w.tris, x, m.Params(precond_leaf=leaf),
                             transpose=transpose)
    if not transpose:
        ref = M.apply(x)
    else:
        n = g.n
        ref = np.empty_like(x)
        for k, idx in enumerate(M.leaves):
            rows = np.concatenate([idx, n + idx])
            ref[rows] = M.block(k).T @ x[rows]
    assert np.abs(y - ref).max() <= 1e-11 * np.abs(ref).max()


def test_preconditioned_solves_match_unpreconditioned_oracle(pb, star12):
    m, ctx = pb
    w = star12
    ref = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-12)
    i0, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-8))
    info, phi, dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                                   m.Params(tol=1e-12, precond_leaf=16))
    assert info.status == m.PB_OK
    assert abs(info.e_solv - ref.e_solv) <= 1e-10 * abs(ref.e_solv)
    i1, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-8, precond_leaf=16))
    assert i1.iters < i0.iters
    i32, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                               m.Params(tol=1e-8, precond_leaf=16, precision=m.PB_FP32_IR,
                                        inner_tol=1e-5))
    assert i32.status == m.PB_OK
    assert abs(i32.e_solv - ref.e_solv) <= 1e-6 * abs(ref.e_solv)
    ip, dpos, dq = ctx.pb_forces(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-12, precond_leaf=16))
    i0f, dpos0, dq0 = ctx.pb_forces(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-12))
    assert np.abs(dpos - dpos0).max() <= 1e-8 * np.abs(dpos0).max()
    # the paper's leaf size N0 = 100
    i100, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                                m.Params(tol=1e-12, precond_leaf=100))
    assert i100.status == m.PB_OK
    assert abs(i100.e_solv - ref.e_solv) <= 1e-10 * abs(ref.e_solv)
    f100, dpos100, _q = ctx.pb_forces(w.verts, w.tris, w.pos, w.q,
                                      m.Params(tol=1e-12, precond_leaf=100))
    assert np.abs(dpos100 - dpos0).max() <= 1e-8 * np.abs(dpos0).max()


def test_preconditioned_full_size_iterations(pb):
    m, ctx = pb
    w = synth.star_protein()
    a, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-6))
    b, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-6, precond_leaf=16))
    c, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-6, precond_leaf=100))
    print(f"iterations to 1e-6: plain {a.iters}, leaf 16 {b.iters}, leaf 100 {c.iters}",
          flush=True)
    assert b.iters < a.iters and c.iters < a.iters
    assert abs(a.e_solv - b.e_solv) <= 1e-5 * abs(a.e_solv)
    assert abs(a.e_solv - c.e_solv) <= 1e-5 * abs(a.e_solv)
