"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (derived in the design notes):
* geometry: same IEEE operations in the same order -> <= 1 ulp-level.
* FP64 pair sums: |dy_i| <= 1e-14 * S_i, S_i = sum of |terms| of row i (the
  oracle reports it): a few ulps per term (the exponential and 1/r are within
  2.3 and 1 ulp), summed in different orders; the K4 difference, which loses
  ~u/(kappa r)^2 of its own size on the nearest pairs, is a small part of S_i.
* FP32 pair sums: |dy_i| <= 5e-5 * S_i (FP32 coordinates after recentring:
  ~1e-6 A position error against 0.1 A neighbour spacing, tile-blocked
  compensated accumulation).
* FP64 solve energies: <= 1e-10 relative when both sides solve to 1e-12;
  refined-FP32 energies: <= 1e-6 relative.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import dsbi, kirkwood

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
KAPPA = 0.1257
FP64_BAR = 1e-14


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
    """Star surface, 2,880 triangles (11 full tiles + a ragged tail of 64)."""
    return synth.star_protein(freq=12, r0=10.0, n_charges=300, seed=41)


@pytest.fixture(scope="module")
def star64():
    return synth.star_protein()


def _params(m, **kw):
    return m.Params(**kw)


def test_geometry_matches_oracle(pb, star64):
    m, ctx = pb
    _say(f"geometry: star {star64.n_tri} triangles")
    cen, nrm, area = ctx.pb_geometry(star64.verts, star64.tris)
    g = dsbi.geometry(star64.verts, star64.tris)
    assert np.allclose(cen, g.cen, rtol=2e-16, atol=0)
    assert np.allclose(nrm, g.nrm, rtol=0, atol=4e-16)
    assert np.allclose(area, g.area, rtol=4e-16, atol=0)


def test_source_matches_oracle_all_rows(pb, star12):
    m, ctx = pb
    w = star12
    _say(f"source: star {w.n_tri} triangles, {w.n_charges} charges")
    b = ctx.pb_source(w.verts, w.tris, w.pos, w.q, _params(m))
    g = dsbi.geometry(w.verts, w.tris)
    ref = dsbi.source(g, w.pos, w.q, 1.0)
    scale = np.abs(ref).max()
    assert np.max(np.abs(b - ref)) <= 1e-13 * scale


def _matvec_case(m, ctx, w, transpose, precision, rows=None, seed=0):
    g = dsbi.geometry(w.verts, w.tris)
    rng = np.random.default_rng(seed)
    x = rng.normal(size=2 * g.n)
    y = ctx.pb_matvec(w.verts, w.tris, x, _params(m), transpose=transpose, precision=precision)
    if rows is None:
        rows = np.arange(g.n)
    y1, y2, s1, s2 = dsbi.matvec(g, 80.0, KAPPA, x, rows=rows, transpose=transpose,
                                 with_abs=True)
    e1 = np.abs(y[rows] - y1) / s1
    e2 = np.abs(y[g.n + rows] - y2) / s2
    return max(e1.max(), e2.max())


@pytest.mark.parametrize("transpose", [False, True])
def test_matvec_fp64_all_rows_ragged(pb, star12, transpose):
    m, ctx = pb
    _say(f"matvec fp64 transpose={transpose}: {star12.n_tri} triangles")
    err = _matvec_case(m, ctx, star12, transpose, m.PB_FP64)
    _say(f"  max |dy|/S = {err:.3e}")
    assert err <= FP64_BAR


@pytest.mark.parametrize("transpose", [False, True])
def test_matvec_fp32_all_rows_ragged(pb, star12, transpose):
    m, ctx = pb
    _say(f"matvec fp32 transpose={transpose}: {star12.n_tri} triangles")
    err = _matvec_case(m, ctx, star12, transpose, m.PB_FP32_IR)
    _say(f"  max |dy|/S = {err:.3e}")
    assert err <= 5e-5


@pytest.mark.parametrize("precision,tol", [(0, 1e-14), (1, 5e-5)])
def test_matvec_full_size_sampled_rows(pb, star64, precision, tol):
    m, ctx = pb
    rows = np.sort(np.random.default_rng(5).choice(star64.n_tri, 192, replace=False))
    rows = np.concatenate([rows, [0, star64.n_tri - 1]])
    _say(f"matvec full size precision={precision}: {star64.n_tri} triangles, {len(rows)} rows")
    for transpose in (False, True):
        err = _matvec_case(m, ctx, star64, transpose, precision, rows=rows, seed=3)
        _say(f"  transpose={transpose} max |dy|/S = {err:.3e}")
        assert err <= tol


def test_energy_matches_oracle(pb, star12):
    m, ctx = pb
    w = star12
    g = dsbi.geometry(w.verts, w.tris)
    xi = np.random.default_rng(8).normal(size=2 * g.n) * 1e-2
    _say(f"energy: {w.n_tri} triangles, {w.n_charges} charges")
    e = ctx.pb_energy(w.verts, w.tris, w.pos, w.q, xi[:g.n], xi[g.n:], _params(m))
    ref = dsbi.energy(g, 80.0, KAPPA, xi, w.pos, w.q)
    P = dsbi.energy_terms(g, 80.0, KAPPA, xi, w.pos)
    bound = 1e-12 * 0.5 * 332.0716 * 4 * np.pi * np.sum(np.abs(w.q * P)) + 1e-13 * abs(ref)
    assert abs(e - ref) <= bound


def test_solve_fp64_kirkwood_matches_oracle_and_golden(pb):
    m, ctx = pb
    w = synth.kirkwood_sphere()
    gold = json.load(open(os.path.join(HERE, "golden", "kirkwood_f8.json")))
    assert synth.input_digest(w) == gold["digest"]
    _say("solve fp64: kirkwood sphere 1,280 triangles, tol 1e-12")
    info, phi, dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, _params(m, tol=1e-12))
    assert info.status == m.PB_OK
    assert abs(info.e_solv - gold["e_solv"]) <= 1e-10 * abs(gold["e_solv"])
    idx = np.asarray(gold["sample_index"])
    assert np.allclose(phi[idx], gold["phi"], rtol=1e-9, atol=0)
    assert np.allclose(dphi[idx], gold["dphi"], rtol=1e-9, atol=0)
    # distance to the closed form matches the oracle's discretisation error
    born = kirkwood.born_energy(2.0, 1.0)
    assert abs(info.e_solv - born) / abs(born) < 0.02


def test_solve_fp64_tiny_mesh_against_dense_lu(pb):
    """20 triangles (one partial tile), off-centre charge."""
    m, ctx = pb
    v, t = synth.icosphere(1, 3.0)
    pos = np.array([[0.3, -0.2, 0.5]])
    q = np.array([1.0])
    _say("solve fp64: 20-triangle icosahedron vs dense LU")
    ref = dsbi.solve_dense(v, t, pos, q)
    info, phi, dphi = ctx.pb_solve(v, t, pos, q, _params(m, tol=1e-13))
    assert info.status == m.PB_OK
    xi = np.concatenate([phi, dphi])
    assert np.linalg.norm(xi - ref.xi) <= 1e-10 * np.linalg.norm(ref.xi)
    assert abs(info.e_solv - ref.e_solv) <= 1e-10 * abs(ref.e_solv)


def test_solve_fp64_ragged_star_matches_oracle(pb, star12):
    m, ctx = pb
    w = star12
    _say(f"solve fp64: star {w.n_tri} triangles, {w.n_charges} charges, tol 1e-12")
    ref = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-12)
    info, phi, dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, _params(m, tol=1e-12))
    assert info.status == m.PB_OK
    assert abs(info.e_solv - ref.e_solv) <= 1e-10 * abs(ref.e_solv)
    xi = np.concatenate([phi, dphi])
    assert np.linalg.norm(xi - ref.xi) <= 1e-9 * np.linalg.norm(ref.xi)


def test_solve_fp32_ir_ragged_star(pb, star12):
    m, ctx = pb
    w = star12
    _say(f"solve fp32-ir: star {w.n_tri} triangles")
    ref = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-12)
    info, phi, dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                                   _params(m, tol=1e-8, precision=m.PB_FP32_IR))
    assert info.status == m.PB_OK
    assert info.refinements >= 1 and info.matvecs_fp32 > 0
    assert abs(info.e_solv - ref.e_solv) <= 1e-6 * abs(ref.e_solv)


def test_solve_full_size_fp64_and_fp32_ir(pb, star64):
    m, ctx = pb
    w = star64
    _say(f"solve full size: star {w.n_tri} triangles, {w.n_charges} charges")
    info64, phi, dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, _params(m, tol=1e-12))
    _say(f"  fp64 E={info64.e_solv:.12f} iters={info64.iters} t={info64.seconds:.2f}s")
    assert info64.status == m.PB_OK
    path = os.path.join(HERE, "golden", "star_f64_s2.json")
    if os.path.exists(path):
        gold = json.load(open(path))
        assert synth.input_digest(w) == gold["digest"]
        assert abs(info64.e_solv - gold["e_solv"]) <= 1e-10 * abs(gold["e_solv"])
        idx = np.asarray(gold["sample_index"])
        assert np.allclose(phi[idx], gold["phi"], rtol=1e-8, atol=1e-12 * np.abs(phi).max())
    # property that holds at any size: the FP64 solution satisfies the
    # oracle's equations on sampled rows, and the oracle's energy of it agrees
    g = dsbi.geometry(w.verts, w.tris)
    rows = np.sort(np.random.default_rng(6).choice(w.n_tri, 64, replace=False))
    xi = np.concatenate([phi, dphi])
    y1, y2 = dsbi.matvec(g, 80.0, KAPPA, xi, rows=rows)
    b1, b2 = dsbi.source(g, w.pos, w.q, 1.0, rows=rows)
    bn = np.abs(np.concatenate([b1, b2])).max()
    assert np.abs(np.concatenate([y1 - b1, y2 - b2])).max() <= 1e-9 * bn
    e_orc = dsbi.energy(g, 80.0, KAPPA, xi, w.pos, w.q)
    assert abs(e_orc - info64.e_solv) <= 1e-11 * abs(e_orc)
    info32, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                                  _params(m, tol=1e-7, precision=m.PB_FP32_IR))
    _say(f"  fp32-ir E={info32.e_solv:.12f} refinements={info32.refinements} "
         f"mv32={info32.matvecs_fp32} mv64={info32.matvecs_fp64} t={info32.seconds:.2f}s")
    assert info32.status == m.PB_OK
    assert abs(info32.e_solv - info64.e_solv) <= 1e-6 * abs(info64.e_solv)


def test_not_converged_returns_last_iterate(pb):
    m, ctx = pb
    w = synth.kirkwood_sphere(freq=4)
    info, phi, dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, _params(m, tol=1e-12, max_iter=1))
    assert info.status == m.PB_NOT_CONVERGED
    assert info.iters == 1 and info.rel_residual > 1e-12
    assert np.all(np.isfinite(phi)) and np.all(np.isfinite(dphi))


def test_invalid_inputs_are_rejected(pb):
    m, ctx = pb
    w = synth.kirkwood_sphere(freq=4)
    P = _params(m)

    def code(verts, tris, pos, q, params=P):
        with pytest.raises(m.PbError) as e:
            ctx.pb_solve(verts, tris, pos, q, params)
        return e.value.status

    t = w.tris.copy()
    t[5, 1] = w.verts.shape[0]
    assert code(w.verts, t, w.pos, w.q) == m.PB_ERR_GEOMETRY
    v = w.verts.copy()
    v[3, 0] = np.nan
    assert code(v, w.tris, w.pos, w.q) == m.PB_ERR_GEOMETRY
    t = w.tris.copy()
    t[7, 2] = t[7, 1]
    assert code(w.verts, t, w.pos, w.q) == m.PB_ERR_GEOMETRY
    assert code(w.verts, w.tris[:, ::-1].copy(), w.pos, w.q) == m.PB_ERR_GEOMETRY
    assert code(w.verts, w.tris, np.array([[0.0, 0.0, 5.0]]), w.q) == m.PB_ERR_CHARGE
    assert code(w.verts, w.tris, w.pos, w.q, _params(m, eps_in=0.0)) == m.PB_ERR_ARG
    assert code(w.verts, w.tris, w.pos, w.q, _params(m, kappa=-1.0)) == m.PB_ERR_ARG
    assert code(w.verts, w.tris, w.pos, w.q, _params(m, restart=0)) == m.PB_ERR_ARG
    # the context still works afterwards
    info, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, P)
    assert info.status == m.PB_OK


def test_repeated_solves_are_bitwise_identical(pb, star12):
    m, ctx = pb
    w = star12
    a = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, _params(m, tol=1e-8))
    b = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, _params(m, tol=1e-8))
    assert a[0].e_solv == b[0].e_solv
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_device_entry_points_match_host_ones(pb, star12):
    import torch
    m, ctx = pb
    w = star12
    dev = torch.device("cuda:0")
    tv = torch.from_numpy(w.verts).to(dev)
    tt = torch.from_numpy(w.tris.astype(np.int32)).to(dev)
    tp = torch.from_numpy(w.pos).to(dev)
    tq = torch.from_numpy(w.q).to(dev)
    x = np.random.default_rng(2).normal(size=2 * w.n_tri)
    tx = torch.from_numpy(x).to(dev)
    ty = torch.empty_like(tx)
    torch.cuda.synchronize()
    ctx.pb_matvec_dev(tv, tt, tx, ty, _params(m))
    y = ctx.pb_matvec(w.verts, w.tris, x, _params(m))
    assert np.array_equal(ty.cpu().numpy(), y)
    phi = torch.empty(w.n_tri, dtype=torch.float64, device=dev)
    dphi = torch.empty_like(phi)
    info = ctx.pb_solve_dev(tv, tt, tp, tq, _params(m, tol=1e-8), phi, dphi)
    info_h, ph, dh = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, _params(m, tol=1e-8))
    assert info.e_solv == info_h.e_solv
    assert np.array_equal(phi.cpu().numpy(), ph)
    # sources and energy on device arrays: the host entry points' values
    tb = torch.empty(2 * w.n_tri, dtype=torch.float64, device=dev)
    ctx.pb_source_dev(tv, tt, tp, tq, _params(m), tb)
    assert np.array_equal(tb.cpu().numpy(), ctx.pb_source(w.verts, w.tris, w.pos, w.q, _params(m)))
    e_dev = ctx.pb_energy_dev(tv, tt, tp, tq, phi, dphi, _params(m))
    assert e_dev == ctx.pb_energy(w.verts, w.tris, w.pos, w.q, ph, dh, _params(m))
    assert e_dev == info.e_solv


def test_interior_potential_and_coulomb_energy(pb, star12):
    """Eq. eq_inside at interior points and E_free - E_sol against the oracle."""
    m, ctx = pb
    w = star12
    info, phi, dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, _params(m, tol=1e-12))
    g = dsbi.geometry(w.verts, w.tris)
    pts = w.pos[:40] + 0.25   # points near the charges, inside the surface
    xi = np.concatenate([phi, dphi])
    ref_r, ref_t = dsbi.potential(g, 80.0, KAPPA, xi, w.pos, w.q, 1.0, pts)
    reac, tot = ctx.pb_potential(w.verts, w.tris, w.pos, w.q, phi, dphi, pts, _params(m))
    assert np.abs(reac - ref_r).max() <= 1e-12 * np.abs(ref_r).max()
    assert np.abs(tot - ref_t).max() <= 1e-12 * np.abs(ref_t).max()
    ec = ctx.pb_coulomb_energy(w.pos, w.q, _params(m))
    ref_c = dsbi.coulomb_energy(w.pos, w.q, 1.0)
    assert abs(ec - ref_c) <= 1e-12 * abs(ref_c)
    # at the charges themselves (self term excluded) the reaction part of
    # (1/2) sum q phi_1 is E_sol
    reac_k, _t = ctx.pb_potential(w.verts, w.tris, w.pos, w.q, phi, dphi, w.pos, _params(m))
    e_sol = 332.0716 * 4 * np.pi * 0.5 * np.sum(w.q * reac_k)
    assert abs(e_sol - info.e_solv) <= 1e-11 * abs(info.e_solv)
