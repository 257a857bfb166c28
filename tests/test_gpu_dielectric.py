"""Parity away from the default dielectric setting, the kappa -> 0+ range of the
reduced FP32 form, and the input guards of the C ABI.

* eps_in = 2, eps_out = 78.5, kappa = 0.05: eps_in scales S1/S2 (eq.
  source_terms) and the force factor 1/(4 pi eps_in); eps = eps_out/eps_in
  enters every kernel (eqs. eqbim_5/eqbim_6).  Matvec in both precisions and
  directions, sources, energy, solve and forces against the oracle with the
  same constants.
* kappa in {1e-13, 1e-6, 1e-3}: the FP32 sweeps measure lengths in a unit
  bounded below by the mesh's own length scale, so (sigma r)^-3 stays finite
  however small kappa is; kappa in {30, 100}: the large end of the accepted
  range.
* Coincident centroids, far coordinates, kappa out of range and a device
  memory cap are rejected with their status codes and the context stays
  usable.
"""
import numpy as np
import pytest

import synth
from oracle import dsbi

pytestmark = pytest.mark.gpu

EPS_IN, EPS_OUT, KAPPA = 2.0, 78.5, 0.05
FP64_BAR = 1e-14   # |dy_i| / S_i, S_i = sum of |terms| of row i
FP32_BAR = 5e-5


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
    """2,880 triangles (11 full tiles and a ragged tail), 300 charges."""
    return synth.star_protein(freq=12, r0=10.0, n_charges=300, seed=41)


def _P(m, **kw):
    base = dict(eps_in=EPS_IN, eps_out=EPS_OUT, kappa=KAPPA)
    base.update(kw)
    return m.Params(**base)


def _matvec_err(m, ctx, w, precision, transpose, kappa, eps_in=EPS_IN, eps_out=EPS_OUT,
                seed=0):
    g = dsbi.geometry(w.verts, w.tris)
    x = np.random.default_rng(seed).normal(size=2 * g.n)
    y = ctx.pb_matvec(w.verts, w.tris, x, m.Params(eps_in=eps_in, eps_out=eps_out, kappa=kappa),
                      transpose=transpose, precision=precision)
    rows = np.arange(g.n)
    y1, y2, s1, s2 = dsbi.matvec(g, eps_out / eps_in, kappa, x, rows=rows, transpose=transpose,
                                 with_abs=True)
    return max((np.abs(y[:g.n] - y1) / s1).max(), (np.abs(y[g.n:] - y2) / s2).max())


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("precision,bar", [(0, FP64_BAR), (1, FP32_BAR)])
def test_matvec_other_dielectrics(pb, star12, precision, bar, transpose):
    m, ctx = pb
    _say(f"matvec eps {EPS_IN}/{EPS_OUT} kappa {KAPPA} precision={precision} "
         f"transpose={transpose}: {star12.n_tri} triangles")
    err = _matvec_err(m, ctx, star12, precision, transpose, KAPPA)
    _say(f"  max |dy|/S = {err:.3e}")
    assert err <= bar


def test_source_and_energy_other_dielectrics(pb, star12):
    m, ctx = pb
    w = star12
    g = dsbi.geometry(w.verts, w.tris)
    _say(f"source and energy, eps_in {EPS_IN}")
    b = ctx.pb_source(w.verts, w.tris, w.pos, w.q, _P(m))
    ref = dsbi.source(g, w.pos, w.q, EPS_IN)
    assert np.max(np.abs(b - ref)) <= 1e-13 * np.abs(ref).max()
    xi = np.random.default_rng(8).normal(size=2 * g.n) * 1e-2
    e = ctx.pb_energy(w.verts, w.tris, w.pos, w.q, xi[:g.n], xi[g.n:], _P(m))
    eref = dsbi.energy(g, EPS_OUT / EPS_IN, KAPPA, xi, w.pos, w.q)
    P = dsbi.energy_terms(g, EPS_OUT / EPS_IN, KAPPA, xi, w.pos)
    bound = 1e-12 * 0.5 * 332.0716 * 4 * np.pi * np.sum(np.abs(w.q * P)) + 1e-13 * abs(eref)
    assert abs(e - eref) <= bound


def test_solve_and_forces_other_dielectrics(pb, star12):
    m, ctx = pb
    w = star12
    _say(f"solve and forces, eps {EPS_IN}/{EPS_OUT}, kappa {KAPPA}: {w.n_tri} triangles")
    ref = dsbi.solve(w.verts, w.tris, w.pos, w.q, eps_in=EPS_IN, eps_out=EPS_OUT, kappa=KAPPA,
                     tol=1e-12)
    info, phi, dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, _P(m, tol=1e-12))
    assert info.status == m.PB_OK
    assert abs(info.e_solv - ref.e_solv) <= 1e-10 * abs(ref.e_solv)
    xi = np.concatenate([phi, dphi])
    assert np.linalg.norm(xi - ref.xi) <= 1e-9 * np.linalg.norm(ref.xi)
    # the same energy differs from the default dielectric pair's
    d_ref = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-8)
    assert abs(d_ref.e_solv - ref.e_solv) > 1e-3 * abs(ref.e_solv)
    i32, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                               _P(m, tol=1e-8, precision=m.PB_FP32_IR))
    assert i32.status == m.PB_OK
    assert abs(i32.e_solv - ref.e_solv) <= 1e-6 * abs(ref.e_solv)
    o_pos, o_q, _lam, _i = dsbi.forces(ref, w.pos, w.q, eps_in=EPS_IN, eps_out=EPS_OUT,
                                       kappa=KAPPA, tol=1e-12)
    finfo, dpos, dq = ctx.pb_forces(w.verts, w.tris, w.pos, w.q, _P(m, tol=1e-12))
    assert finfo.status == m.PB_OK
    _say(f"  forces max rel {np.abs(dpos - o_pos).max() / np.abs(o_pos).max():.2e}")
    assert np.abs(dpos - o_pos).max() <= 1e-8 * np.abs(o_pos).max()
    assert np.abs(dq - o_q).max() <= 1e-8 * np.abs(o_q).max()


@pytest.mark.parametrize("kappa", [30.0, 100.0])
def test_sweeps_at_large_kappa(pb, star12, kappa):
    """kappa up to the accepted maximum: kappa r between a real point and the
    sweeps' padding points (2e6 A out, weight 0) then passes the FP64
    exponential's exact range, where its conversion saturates to a zero
    result.  Both precisions, both directions, all rows against the oracle."""
    m, ctx = pb
    for precision, bar in ((0, FP64_BAR), (1, FP32_BAR)):
        for transpose in (False, True):
            err = _matvec_err(m, ctx, star12, precision, transpose, kappa, eps_in=1.0,
                              eps_out=80.0)
            _say(f"kappa={kappa:g} precision={precision} transpose={transpose}: "
                 f"max |dy|/S = {err:.3e}")
            assert err <= bar


@pytest.mark.parametrize("kappa", [1e-13, 1e-6, 1e-3])
def test_fp32_sweeps_near_zero_kappa(pb, star12, kappa):
    """Both FP32 sweep kinds and directions at kappa far below 1/(mesh size)."""
    m, ctx = pb
    for kind in (m.PB_SWEEP_PAIRWISE, 1):
        ctx.set_sweep_config(kind, 0)
        try:
            for transpose in (False, True):
                err = _matvec_err(m, ctx, star12, m.PB_FP32_IR, transpose, kappa, eps_in=1.0,
                                  eps_out=80.0)
                _say(f"fp32 kappa={kappa:g} kind={kind} transpose={transpose}: "
                     f"max |dy|/S = {err:.3e}")
                assert err <= FP32_BAR
        finally:
            ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 0)


def test_refined_solve_near_zero_kappa(pb, star12):
    m, ctx = pb
    w = star12
    kappa = 1e-13
    ref = dsbi.solve(w.verts, w.tris, w.pos, w.q, kappa=kappa, tol=1e-12)
    info, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                                m.Params(kappa=kappa, tol=1e-8, precision=m.PB_FP32_IR))
    _say(f"refined solve kappa {kappa:g}: E={info.e_solv:.10f} oracle {ref.e_solv:.10f}")
    assert info.status == m.PB_OK
    assert abs(info.e_solv - ref.e_solv) <= 1e-6 * abs(ref.e_solv)


def test_coincident_centroids_are_rejected_by_index(pb):
    """Two copies of one triangle share a centroid: the collocation system
    would evaluate a pair at r = 0."""
    m, ctx = pb
    w = synth.kirkwood_sphere(freq=4)
    # append an exact copy of triangle 17 (the enclosed volume stays positive)
    t = np.vstack([w.tris, w.tris[17][None, :]]).astype(np.int32)
    with pytest.raises(m.PbError) as e:
        ctx.pb_solve(w.verts, t, w.pos, w.q, m.Params())
    _say(f"coincident: {e.value.message}")
    assert e.value.status == m.PB_ERR_GEOMETRY
    assert "triangle 17 shares its centroid" in e.value.message
    # the batch names the system
    with pytest.raises(m.PbError) as e:
        ctx.pb_solve_batch([(w.verts, w.tris, w.pos, w.q), (w.verts, t, w.pos, w.q)],
                           m.Params())
    assert e.value.status == m.PB_ERR_GEOMETRY and "system 1" in e.value.message
    info, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params())
    assert info.status == m.PB_OK


def test_far_coordinates_and_kappa_range_are_rejected(pb):
    m, ctx = pb
    w = synth.kirkwood_sphere(freq=4)
    v = w.verts + np.array([2e5, 0.0, 0.0])
    with pytest.raises(m.PbError) as e:
        ctx.pb_solve(v, w.tris, w.pos + np.array([2e5, 0.0, 0.0]), w.q, m.Params())
    assert e.value.status == m.PB_ERR_GEOMETRY and "beyond" in e.value.message
    for kappa in (101.0, float("nan"), float("inf"), -1e-9):
        with pytest.raises(m.PbError) as e:
            ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(kappa=kappa))
        assert e.value.status == m.PB_ERR_ARG
    info, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(kappa=100.0))
    assert info.status == m.PB_OK and np.isfinite(info.e_solv)


def test_memory_cap_gives_oom_and_the_context_recovers(pb):
    import paper_2312_10044_amd as m
    ctx = m.Context(0)
    try:
        w = synth.kirkwood_sphere(freq=8)
        ctx.set_memory_limit(64 * 1024)
        with pytest.raises(m.PbError) as e:
            ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params())
        _say(f"memory cap: {e.value.message}")
        assert e.value.status == m.PB_ERR_OOM and "limit" in e.value.message
        held = ctx.memory_used()
        assert held <= 64 * 1024
        ctx.set_memory_limit(0)
        info, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-10))
        assert info.status == m.PB_OK
        assert ctx.memory_used() > held
        ref = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-10)
        assert abs(info.e_solv - ref.e_solv) <= 1e-8 * abs(ref.e_solv)
    finally:
        ctx.close()
