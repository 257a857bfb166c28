"""The FP32 sweeps in both kinds (pairwise: each unordered pair once, forward
and transposed; per-target: 1 or 2 targets per thread) and the pairwise FP64
sweep against the oracle's matvec."""
import numpy as np
import pytest

import synth
from oracle import dsbi

pytestmark = pytest.mark.gpu

KAPPA = 0.1257
FP64_BAR = 1e-14   # |dy_i| / S_i for the FP64 sweeps


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
def star12():
    """2,880 triangles: 12 tiles of 256 after padding, the last one ragged."""
    return synth.star_protein(freq=12, r0=10.0, n_charges=300, seed=41)


def _err(m, ctx, w, kappa=KAPPA, rows=None, seed=0, transpose=False):
    g = dsbi.geometry(w.verts, w.tris)
    x = np.random.default_rng(seed).normal(size=2 * g.n)
    y = ctx.pb_matvec(w.verts, w.tris, x, m.Params(kappa=kappa), transpose=transpose,
                      precision=m.PB_FP32_IR)
    if rows is None:
        rows = np.arange(g.n)
    y1, y2, s1, s2 = dsbi.matvec(g, 80.0, kappa, x, rows=rows, transpose=transpose,
                                 with_abs=True)
    return max((np.abs(y[rows] - y1) / s1).max(), (np.abs(y[g.n + rows] - y2) / s2).max()), y


@pytest.mark.parametrize("kind", ["pairwise", "banded", 1, 2])
@pytest.mark.parametrize("kappa", [KAPPA, 0.0])
def test_fp32_sweep_kinds_all_rows(pb, star12, kind, kappa):
    m, ctx = pb
    k = {"pairwise": m.PB_SWEEP_PAIRWISE, "banded": m.PB_SWEEP_BANDED}.get(kind, kind)
    ctx.set_sweep_config(k, 32768)
    _say(f"fp32 sweep kind={kind} kappa={kappa}: {star12.n_tri} triangles")
    err, _y = _err(m, ctx, star12, kappa=kappa)
    _say(f"  max |dy|/S = {err:.3e}")
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 131072)
    assert err <= 5e-5


@pytest.mark.parametrize("kappa", [KAPPA, 0.0])
def test_fp32_pairwise_transposed_all_rows(pb, star12, kappa):
    """The transposed operator through the pairwise sweep (stream of l1, l2,
    the pair constant with eps -> 1/eps, rows swapped and area-scaled)."""
    m, ctx = pb
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 32768)
    _say(f"fp32 pairwise transposed kappa={kappa}: {star12.n_tri} triangles")
    err, y = _err(m, ctx, star12, kappa=kappa, seed=8, transpose=True)
    _e, y2 = _err(m, ctx, star12, kappa=kappa, seed=8, transpose=True)
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 131072)
    _say(f"  max |dy|/S = {err:.3e}")
    assert err <= 5e-5
    assert np.array_equal(y, y2)


@pytest.mark.parametrize("freq,r0", [(2, 3.0), (8, 2.0)])
def test_pairwise_small_meshes(pb, freq, r0):
    """80 triangles (one real tile, one tile of padding only) and 1,280."""
    m, ctx = pb
    w = synth.star_protein(freq=freq, r0=r0, n_charges=1, seed=7) if freq == 2 else \
        synth.kirkwood_sphere()
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 32768)
    _say(f"pairwise small mesh: {w.n_tri} triangles")
    err, _y = _err(m, ctx, w)
    err_t, _y = _err(m, ctx, w, transpose=True)
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 131072)
    assert err <= 5e-5 and err_t <= 5e-5


@pytest.mark.parametrize("waves", [256, 8192, 131072])
def test_pairwise_plan_sizes_and_repeat(pb, star12, waves):
    """Items of many tiles or of one tile give the same matvec up to rounding,
    and a repeated call is bitwise identical."""
    m, ctx = pb
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, waves)
    err, y = _err(m, ctx, star12, seed=4)
    _e2, y2 = _err(m, ctx, star12, seed=4)
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 131072)
    assert err <= 5e-5
    assert np.array_equal(y, y2)


@pytest.mark.parametrize("waves", [32768, 131072])
def test_pairwise_full_size_sampled_rows(pb, waves):
    """81,920 triangles, forward and transposed; 131072 target waves is the
    launch configuration the bench times."""
    m, ctx = pb
    w = synth.star_protein()
    rows = np.sort(np.random.default_rng(5).choice(w.n_tri, 160, replace=False))
    rows = np.concatenate([rows, [0, w.n_tri - 1]])
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, waves)
    try:
        for transpose in (False, True):
            _say(f"pairwise full size: {w.n_tri} triangles, {len(rows)} rows, waves {waves}, "
                 f"transpose {transpose}")
            err, _y = _err(m, ctx, w, rows=rows, seed=3, transpose=transpose)
            _say(f"  max |dy|/S = {err:.3e}")
            assert err <= 5e-5
    finally:
        ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 131072)


def test_pairwise_largest_size_sampled_rows(pb):
    """The 327,680-triangle surface of the largest workload in the bench's
    launch configuration: FP32 pairwise forward and transposed, FP64 pairwise
    forward, on sampled rows plus the first and the last."""
    import types
    m, ctx = pb
    verts, tris = synth.large_star_surface()
    w = types.SimpleNamespace(verts=verts, tris=tris)
    n = tris.shape[0]
    rows = np.sort(np.random.default_rng(8).choice(n, 40, replace=False))
    rows = np.concatenate([rows, [0, n - 1]])
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 131072)
    ctx.set_fp64_sweep(m.PB_SWEEP_PAIRWISE)
    for transpose in (False, True):
        _say(f"pairwise largest size: {n} triangles, {len(rows)} rows, transpose {transpose}")
        err, _y = _err(m, ctx, w, rows=rows, seed=9, transpose=transpose)
        _say(f"  FP32 max |dy|/S = {err:.3e}")
        assert err <= 5e-5
    err64, _y = _err64(m, ctx, w, False, rows=rows, seed=9)
    _say(f"  FP64 max |dy|/S = {err64:.3e}")
    assert err64 <= FP64_BAR


def test_pairwise_ir_solve_matches_fp64(pb, star12):
    m, ctx = pb
    w = star12
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 32768)
    i64, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-12))
    i32, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                               m.Params(tol=1e-8, precision=m.PB_FP32_IR))
    ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 131072)
    assert i32.status == m.PB_OK and i32.matvecs_fp32 > 0
    assert abs(i32.e_solv - i64.e_solv) <= 1e-6 * abs(i64.e_solv)


def _err64(m, ctx, w, transpose, kappa=KAPPA, rows=None, seed=0):
    g = dsbi.geometry(w.verts, w.tris)
    x = np.random.default_rng(seed).normal(size=2 * g.n)
    y = ctx.pb_matvec(w.verts, w.tris, x, m.Params(kappa=kappa), transpose=transpose,
                      precision=m.PB_FP64)
    if rows is None:
        rows = np.arange(g.n)
    y1, y2, s1, s2 = dsbi.matvec(g, 80.0, kappa, x, rows=rows, transpose=transpose,
                                 with_abs=True)
    return max((np.abs(y[rows] - y1) / s1).max(), (np.abs(y[g.n + rows] - y2) / s2).max()), y


@pytest.mark.parametrize("kind", ["pairwise", 1])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("kappa", [KAPPA, 0.0])
def test_fp64_sweep_kinds_all_rows(pb, star12, kind, transpose, kappa):
    m, ctx = pb
    ctx.set_fp64_sweep(m.PB_SWEEP_PAIRWISE if kind == "pairwise" else kind)
    _say(f"fp64 sweep kind={kind} transpose={transpose} kappa={kappa}")
    err, _y = _err64(m, ctx, star12, transpose, kappa=kappa)
    ctx.set_fp64_sweep(m.PB_SWEEP_PAIRWISE)
    _say(f"  max |dy|/S = {err:.3e}")
    assert err <= FP64_BAR


def test_fp64_pairwise_small_mesh_and_repeat(pb):
    m, ctx = pb
    w = synth.star_protein(freq=2, r0=3.0, n_charges=1, seed=7)
    ctx.set_fp64_sweep(m.PB_SWEEP_PAIRWISE)
    for transpose in (False, True):
        err, y = _err64(m, ctx, w, transpose)
        _e, y2 = _err64(m, ctx, w, transpose)
        assert err <= FP64_BAR and np.array_equal(y, y2)


def test_fp64_pairwise_full_size_sampled_rows(pb):
    m, ctx = pb
    w = synth.star_protein()
    rows = np.sort(np.random.default_rng(6).choice(w.n_tri, 96, replace=False))
    ctx.set_fp64_sweep(m.PB_SWEEP_PAIRWISE)
    for transpose in (False, True):
        err, _y = _err64(m, ctx, w, transpose, rows=rows, seed=2)
        _say(f"fp64 pairwise full size transpose={transpose}: {err:.3e}")
        assert err <= FP64_BAR


@pytest.mark.parametrize("waves", [256, 8192, 131072, 1048576])
@pytest.mark.parametrize("transpose", [False, True])
def test_banded_plan_shapes_both_directions_and_repeat(pb, star12, waves, transpose):
    """The banded sweep over plans from a few long items (runs of up to 24
    source tiles, bands of several macro tiles) to many short ones: the
    oracle's matvec in both directions, and a repeated call bitwise
    identical."""
    m, ctx = pb
    ctx.set_sweep_config(m.PB_SWEEP_BANDED, waves)
    try:
        err, y = _err(m, ctx, star12, seed=5, transpose=transpose)
        _e2, y2 = _err(m, ctx, star12, seed=5, transpose=transpose)
    finally:
        ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 131072)
    _say(f"banded waves={waves} transpose={transpose}: max |dy|/S = {err:.3e}")
    assert err <= 5e-5
    assert np.array_equal(y, y2)


@pytest.mark.parametrize("freq,r0", [(2, 3.0), (8, 2.0)])
def test_banded_small_meshes(pb, freq, r0):
    """80 triangles (one tile: a macro tile of one real tile) and 1,280."""
    m, ctx = pb
    w = synth.star_protein(freq=freq, r0=r0, n_charges=1, seed=7) if freq == 2 else \
        synth.kirkwood_sphere()
    ctx.set_sweep_config(m.PB_SWEEP_BANDED, 131072)
    try:
        err, _y = _err(m, ctx, w)
        err_t, _y = _err(m, ctx, w, transpose=True)
    finally:
        ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 131072)
    assert err <= 5e-5 and err_t <= 5e-5


def test_banded_full_sizes_sampled_rows_and_solve(pb):
    """81,920 and 327,680 triangles on sampled rows, both directions, and a
    refined solve with the banded sweep against the FP64 solve."""
    import types
    m, ctx = pb
    ctx.set_sweep_config(m.PB_SWEEP_BANDED, 131072)
    try:
        w = synth.star_protein()
        verts, tris = synth.large_star_surface()
        big = types.SimpleNamespace(verts=verts, tris=tris)
        for surf, n in ((w, w.n_tri), (big, tris.shape[0])):
            rows = np.sort(np.random.default_rng(n).choice(n, 40, replace=False))
            rows = np.concatenate([rows, [0, n - 1]])
            for transpose in (False, True):
                err, _y = _err(m, ctx, surf, rows=rows, seed=11, transpose=transpose)
                _say(f"banded {n} triangles transpose={transpose}: max |dy|/S = {err:.3e}")
                assert err <= 5e-5
        i32, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                                   m.Params(tol=1e-7, precision=m.PB_FP32_IR, precond_leaf=24))
    finally:
        ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 131072)
    i64, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-12, precond_leaf=24))
    assert i32.status == m.PB_OK
    assert abs(i32.e_solv - i64.e_solv) <= 1e-6 * abs(i64.e_solv)
