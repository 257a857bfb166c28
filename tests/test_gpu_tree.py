"""Treecode matvec (pb_matvec_tree) against the treecode oracle and, at
theta = 0, against the direct sum."""
import numpy as np
import pytest

import synth
from oracle import dsbi, treecode as tc

pytestmark = pytest.mark.gpu

EPS, KAPPA = 80.0, 0.1257


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def pb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_10044_amd as m
    ctx = m.Context(0)
    yield m, ctx
    ctx.close()


@pytest.fixture(scope="module")
def star8():
    return synth.star_protein(freq=8, r0=8.0, n_charges=1, seed=7)


@pytest.fixture(scope="module")
def star12():
    return synth.star_protein(freq=12, r0=10.0, n_charges=300, seed=41)


def _scale(g, x):
    """Row scale: the diagonal plus the sum of |pair terms| is bounded by
    this; tolerances are relative to max |y_direct|."""
    return np.abs(dsbi.matvec(g, EPS, KAPPA, x)).max()


@pytest.mark.parametrize("mesh", ["star8", "star12"])
def test_tree_theta_zero_is_the_direct_sum(pb, mesh, request):
    m, ctx = pb
    w = request.getfixturevalue(mesh)
    g = dsbi.geometry(w.verts, w.tris)
    x = np.random.default_rng(0).normal(size=2 * g.n)
    _say(f"tree theta=0: {g.n} triangles")
    y = ctx.pb_matvec_tree(w.verts, w.tris, x, m.Params(), theta=0.0, order=2, leaf_size=20)
    ref = dsbi.matvec(g, EPS, KAPPA, x)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("order", [0, 1, 2, 3, 4])
def test_tree_matches_oracle_treecode(pb, star8, order):
    m, ctx = pb
    w = star8
    g = dsbi.geometry(w.verts, w.tris)
    x = np.random.default_rng(order).normal(size=2 * g.n)
    _say(f"tree theta=0.5 p={order}: {g.n} triangles")
    y, cnt = ctx.pb_matvec_tree(w.verts, w.tris, x, m.Params(), theta=0.5, order=order,
                                leaf_size=20, with_counts=True)
    ref = tc.matvec(g, EPS, KAPPA, x, theta=0.5, p=order, n0=20)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    _say(f"  max |dy| / max |y| = {err:.2e}; counts {cnt}")
    assert err <= 1e-12
    pp, pc = tc.counts(g, 0.5, 20)
    assert cnt[0] == pc and cnt[1] == pp


def test_tree_paper_setting_ragged(pb, star12):
    """theta = 0.8, p = 3, N0 = 100 on 2,880 triangles."""
    m, ctx = pb
    w = star12
    g = dsbi.geometry(w.verts, w.tris)
    x = np.random.default_rng(9).normal(size=2 * g.n)
    y = ctx.pb_matvec_tree(w.verts, w.tris, x, m.Params(), theta=0.8, order=3, leaf_size=100)
    ref = tc.matvec(g, EPS, KAPPA, x, theta=0.8, p=3, n0=100)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    d = dsbi.matvec(g, EPS, KAPPA, x)
    _say(f"  treecode vs direct: {np.abs(y - d).max() / np.abs(d).max():.2e}")


def test_tree_full_size_sampled_rows(pb):
    m, ctx = pb
    w = synth.star_protein()
    g = dsbi.geometry(w.verts, w.tris)
    x = np.random.default_rng(3).normal(size=2 * g.n)
    rows = np.sort(np.random.default_rng(4).choice(g.n, 24, replace=False))
    _say(f"tree full size: {g.n} triangles, {len(rows)} rows")
    y = ctx.pb_matvec_tree(w.verts, w.tris, x, m.Params(), theta=0.8, order=3, leaf_size=100)
    r1, r2 = tc.matvec(g, EPS, KAPPA, x, theta=0.8, p=3, n0=100, rows=rows)
    scale = np.abs(y).max()
    assert np.abs(y[rows] - r1).max() <= 1e-11 * scale
    assert np.abs(y[g.n + rows] - r2).max() <= 1e-11 * scale


def test_tree_rejects_bad_parameters(pb, star8):
    m, ctx = pb
    w = star8
    x = np.zeros(2 * w.n_tri)
    for kw in ({"theta": 1.0}, {"theta": -0.1}, {"order": 6}, {"leaf_size": 0}):
        args = dict(theta=0.5, order=2, leaf_size=20)
        args.update(kw)
        with pytest.raises(m.PbError) as e:
            ctx.pb_matvec_tree(w.verts, w.tris, x, m.Params(), **args)
        assert e.value.status == m.PB_ERR_ARG


def test_tree_solve_theta_zero_is_the_direct_solve(pb, star8):
    m, ctx = pb
    w = synth.star_protein(freq=8, r0=8.0, n_charges=20, seed=7)
    P = m.Params(tol=1e-10)
    i_d, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, P)
    i_t, _p, _d = ctx.pb_solve_tree(w.verts, w.tris, w.pos, w.q, P, theta=0.0, order=2,
                                    leaf_size=20)
    assert i_t.status == m.PB_OK
    assert abs(i_t.e_solv - i_d.e_solv) <= 1e-9 * abs(i_d.e_solv)


def test_tree_solve_matches_oracle_treecode_solve(pb):
    """Both sides solve the same treecode operator (theta 0.5, p 3, N0 20) to
    tol 1e-10: the energies agree far below the treecode's own error."""
    m, ctx = pb
    w = synth.star_protein(freq=8, r0=8.0, n_charges=20, seed=7)
    info, _p, _d = ctx.pb_solve_tree(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-10),
                                     theta=0.5, order=3, leaf_size=20)
    e_ref, _xi, _inf = tc.solve(w.verts, w.tris, w.pos, w.q, theta=0.5, p=3, n0=20, tol=1e-10)
    _say(f"tree solve E = {info.e_solv:.12f}, oracle {e_ref:.12f}")
    assert info.status == m.PB_OK
    assert abs(info.e_solv - e_ref) <= 1e-8 * abs(e_ref)


def test_tree_solve_with_preconditioner_and_bad_precision(pb, star12):
    m, ctx = pb
    w = star12
    i_d, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-8, precond_leaf=16))
    i_t, _p, _d = ctx.pb_solve_tree(w.verts, w.tris, w.pos, w.q,
                                    m.Params(tol=1e-8, precond_leaf=16), theta=0.5, order=4,
                                    leaf_size=50)
    _say(f"tree solve (theta 0.5, p 4) vs direct: {abs(i_t.e_solv - i_d.e_solv) / abs(i_d.e_solv):.2e}")
    assert i_t.status == m.PB_OK
    assert abs(i_t.e_solv - i_d.e_solv) <= 1e-2 * abs(i_d.e_solv)
    with pytest.raises(m.PbError) as e:
        ctx.pb_solve_tree(w.verts, w.tris, w.pos, w.q, m.Params(precision=m.PB_FP32_IR))
    assert e.value.status == m.PB_ERR_ARG
    # the context's ordinary solves are unaffected afterwards
    i_d2, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-8, precond_leaf=16))
    assert i_d2.e_solv == i_d.e_solv
