"""Batched solves (pb_solve_batch) against one-at-a-time solves and the oracle."""
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
    ctx = m.Context(0)
    yield m, ctx
    ctx.close()


@pytest.fixture(scope="module")
def small_batch():
    """Six systems of uneven size: 320 to 3,920 triangles, 7 to 300 charges."""
    specs = [(4, 6.0, 7, 51), (14, 12.0, 300, 52), (6, 8.0, 40, 53), (9, 9.0, 120, 54),
             (5, 7.0, 20, 55), (12, 10.0, 257, 56)]
    out = []
    for f, r0, nc, seed in specs:
        w = synth.star_protein(freq=f, r0=r0, n_charges=nc, seed=seed)
        out.append((w.verts, w.tris, w.pos, w.q))
    return out


def test_batch_fp64_matches_single_solves_and_oracle(pb, small_batch):
    m, ctx = pb
    _say(f"batch fp64: {len(small_batch)} systems")
    P = m.Params(tol=1e-12)
    e, infos, _g, _q = ctx.pb_solve_batch(small_batch, P)
    for b, (v, t, pos, q) in enumerate(small_batch):
        info, _p, _d = ctx.pb_solve(v, t, pos, q, P)
        assert infos[b].status == m.PB_OK
        assert abs(e[b] - info.e_solv) <= 1e-10 * abs(info.e_solv), b
    for b, (v, t, pos, q) in enumerate(small_batch):
        ref = dsbi.solve(v, t, pos, q, tol=1e-12)
        _say(f"  system {b}: {t.shape[0]} triangles, E={e[b]:.12f} oracle {ref.e_solv:.12f}")
        assert abs(e[b] - ref.e_solv) <= 1e-10 * abs(ref.e_solv), b


def test_batch_forces_match_single_forces(pb, small_batch):
    m, ctx = pb
    P = m.Params(tol=1e-12)
    e, infos, gpos, gq = ctx.pb_solve_batch(small_batch, P, forces=True)
    off = 0
    for b, (v, t, pos, q) in enumerate(small_batch):
        info, dpos, dq = ctx.pb_forces(v, t, pos, q, P)
        n = q.shape[0]
        assert infos[b].adjoint_iters > 0
        assert abs(e[b] - info.e_solv) <= 1e-10 * abs(info.e_solv)
        assert np.abs(gpos[off:off + n] - dpos).max() <= 1e-8 * np.abs(dpos).max()
        assert np.abs(gq[off:off + n] - dq).max() <= 1e-8 * np.abs(dq).max()
        off += n


def test_batch_forces_match_oracle_adjoint(pb, small_batch):
    """Batch gradients of two systems (the largest and a small one) against
    the oracle's adjoint method (its own transpose GMRES and gradient sums)."""
    m, ctx = pb
    P = m.Params(tol=1e-12)
    e, infos, gpos, gq = ctx.pb_solve_batch(small_batch, P, forces=True)
    offs = np.cumsum([0] + [s[3].shape[0] for s in small_batch])
    for b in (1, 4):
        v, t, pos, q = small_batch[b]
        sol = dsbi.solve(v, t, pos, q, tol=1e-12)
        o_pos, o_q, _lam, _i = dsbi.forces(sol, pos, q, tol=1e-12)
        a, z = offs[b], offs[b + 1]
        err = np.abs(gpos[a:z] - o_pos).max() / np.abs(o_pos).max()
        _say(f"  system {b}: forces max rel err vs oracle adjoint {err:.2e}")
        assert err <= 1e-8
        assert np.abs(gq[a:z] - o_q).max() <= 1e-8 * np.abs(o_q).max()
        assert abs(e[b] - sol.e_solv) <= 1e-10 * abs(sol.e_solv)


def test_batch_eight_systems_spanning_the_batch_workload_sizes(pb):
    """Eight star systems of 5,120 to 81,920 triangles (the size range of the
    64-system batch workload), E_sol and forces in one call: FP64 batch against
    one-at-a-time FP64 solves, the refined-FP32 preconditioned batch (the
    benchmarked configuration) within 1e-6, and the smallest system's energy
    against the oracle."""
    m, ctx = pb
    specs = [(16, 10.0, 100), (23, 12.0, 300), (30, 14.0, 500), (37, 16.0, 800),
             (44, 18.0, 1100), (51, 20.0, 1400), (58, 22.0, 1700), (64, 25.0, 2000)]
    systems = []
    for k, (f, r0, nc) in enumerate(specs):
        w = synth.star_protein(freq=f, r0=r0, n_charges=nc, seed=70 + k)
        systems.append((w.verts, w.tris, w.pos, w.q))
    sizes = [s[1].shape[0] for s in systems]
    _say(f"batch of 8: {sizes} triangles")
    assert min(sizes) == 5120 and max(sizes) == 81920
    P64 = m.Params(tol=1e-12, precond_leaf=24, max_iter=2000)
    e, infos, gpos, gq = ctx.pb_solve_batch(systems, P64, forces=True)
    off = 0
    for b, (v, t, pos, q) in enumerate(systems):
        info, dpos, dq = ctx.pb_forces(v, t, pos, q, P64)
        n = q.shape[0]
        _say(f"  system {b}: E batch {e[b]:.12f} single {info.e_solv:.12f}")
        assert infos[b].status == m.PB_OK and info.status == m.PB_OK
        assert abs(e[b] - info.e_solv) <= 1e-10 * abs(info.e_solv), b
        assert np.abs(gpos[off:off + n] - dpos).max() <= 1e-8 * np.abs(dpos).max()
        assert np.abs(gq[off:off + n] - dq).max() <= 1e-8 * np.abs(dq).max()
        off += n
    P32 = m.Params(tol=1e-6, precision=m.PB_FP32_IR, inner_tol=1e-7, precond_leaf=24,
                   max_iter=2000)
    e32, i32, g32, _q = ctx.pb_solve_batch(systems, P32, forces=True)
    rel = np.abs(e32 - e) / np.abs(e)
    _say(f"  refined FP32 batch: worst E rel err {rel.max():.2e}")
    assert all(i.status == m.PB_OK for i in i32)
    assert rel.max() <= 1e-6
    v, t, pos, q = systems[0]
    ref = dsbi.solve(v, t, pos, q, tol=1e-12)
    assert abs(e[0] - ref.e_solv) <= 1e-10 * abs(ref.e_solv)


def test_batch_device_entry_point_matches_host_one(pb, small_batch):
    """pb_solve_batch_dev on device tensors gives the host entry point's
    energies and gradients bit for bit (same kernels, same order)."""
    import torch
    m, ctx = pb
    dev = torch.device("cuda:0")
    P = m.Params(tol=1e-10, precond_leaf=16)
    e_h, i_h, g_h, q_h = ctx.pb_solve_batch(small_batch, P, forces=True)
    sys_d = [(torch.from_numpy(v).to(dev), torch.from_numpy(t.astype(np.int32)).to(dev),
              torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev))
             for v, t, pos, q in small_batch]
    nct = sum(s[3].shape[0] for s in small_batch)
    gpos = torch.empty((nct, 3), dtype=torch.float64, device=dev)
    gq = torch.empty(nct, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    e_d, i_d = ctx.pb_solve_batch_dev(sys_d, P, gpos, gq)
    _say(f"batch dev: E {e_d}")
    assert np.array_equal(e_d, e_h)
    assert [i.iters for i in i_d] == [i.iters for i in i_h]
    assert np.array_equal(gpos.cpu().numpy(), g_h) and np.array_equal(gq.cpu().numpy(), q_h)
    e_e, _i = ctx.pb_solve_batch_dev(sys_d, P)   # energies only (their own charge sweep)
    e_e2, _i, _g, _q = ctx.pb_solve_batch(small_batch, P)
    assert np.array_equal(e_e, e_e2)
    assert np.max(np.abs(e_e - e_h) / np.abs(e_h)) <= 1e-13


def test_batch_fp32_refined_energies(pb, small_batch):
    m, ctx = pb
    e64, _i, _g, _q = ctx.pb_solve_batch(small_batch, m.Params(tol=1e-12))
    e32, infos, _g, _q = ctx.pb_solve_batch(small_batch,
                                            m.Params(tol=1e-8, precision=m.PB_FP32_IR))
    for b in range(len(small_batch)):
        assert infos[b].status == m.PB_OK and infos[b].matvecs_fp32 > 0
        assert abs(e32[b] - e64[b]) <= 1e-6 * abs(e64[b])


def test_batch_rejects_a_bad_system_by_name(pb, small_batch):
    m, ctx = pb
    bad = list(small_batch)
    v, t, pos, q = bad[3]
    t = t.copy()
    t[0, 0] = v.shape[0] + 5
    bad[3] = (v, t, pos, q)
    with pytest.raises(m.PbError) as e:
        ctx.pb_solve_batch(bad, m.Params())
    assert e.value.status == m.PB_ERR_GEOMETRY and "system 3" in e.value.message
    e2, infos, _g, _q = ctx.pb_solve_batch(small_batch[:2], m.Params(tol=1e-8))
    assert all(i.status == m.PB_OK for i in infos)


def test_batch_single_system_and_repeat_determinism(pb, small_batch):
    m, ctx = pb
    one = small_batch[1:2]
    a, _i, _g, _q = ctx.pb_solve_batch(one, m.Params(tol=1e-10))
    b, _i, _g, _q = ctx.pb_solve_batch(one, m.Params(tol=1e-10))
    assert a[0] == b[0]


@pytest.mark.parametrize("leaf", [1, 16])
def test_batch_preconditioned_matches_single_preconditioned(pb, small_batch, leaf):
    """Per-system leaf blocks in the concatenated layout give the single-system
    preconditioned energies and forces; leaf 1 (2x2 blocks) included."""
    m, ctx = pb
    _say(f"batch precond leaf {leaf}")
    P = m.Params(tol=1e-12, precond_leaf=leaf)
    e, infos, gpos, gq = ctx.pb_solve_batch(small_batch, P, forces=True)
    e0, infos0, _g, _q = ctx.pb_solve_batch(small_batch, m.Params(tol=1e-12))
    off = 0
    for b, (v, t, pos, q) in enumerate(small_batch):
        info, dpos, dq = ctx.pb_forces(v, t, pos, q, P)
        n = q.shape[0]
        assert infos[b].status == m.PB_OK
        assert abs(e[b] - info.e_solv) <= 1e-10 * abs(info.e_solv), b
        assert abs(e[b] - e0[b]) <= 1e-10 * abs(e0[b]), b
        assert np.abs(gpos[off:off + n] - dpos).max() <= 1e-8 * np.abs(dpos).max()
        assert np.abs(gq[off:off + n] - dq).max() <= 1e-8 * np.abs(dq).max()
        off += n
    if leaf == 16:
        assert sum(i.iters for i in infos) < sum(i.iters for i in infos0)


def test_batch_preconditioned_fp32_refined(pb, small_batch):
    m, ctx = pb
    e64, _i, _g, _q = ctx.pb_solve_batch(small_batch, m.Params(tol=1e-12))
    e32, infos, _g, _q = ctx.pb_solve_batch(
        small_batch, m.Params(tol=1e-8, precision=m.PB_FP32_IR, precond_leaf=16))
    for b in range(len(small_batch)):
        assert infos[b].status == m.PB_OK and infos[b].matvecs_fp32 > 0
        assert abs(e32[b] - e64[b]) <= 1e-6 * abs(e64[b])


def test_batch_sweep_kinds_agree(pb, small_batch):
    """The batch with per-target sweeps (FP32 and FP64) against the default
    pairwise sweeps: same energies and forces up to rounding."""
    m, ctx = pb
    P = m.Params(tol=1e-12, precond_leaf=16)
    e_pw, _i, g_pw, q_pw = ctx.pb_solve_batch(small_batch, P, forces=True)
    ctx.set_sweep_config(1, 0)
    ctx.set_fp64_sweep(1)
    try:
        e_pt, _i, g_pt, q_pt = ctx.pb_solve_batch(small_batch, P, forces=True)
        e32_pt, _i, _g, _q = ctx.pb_solve_batch(
            small_batch, m.Params(tol=1e-8, precision=m.PB_FP32_IR, precond_leaf=16))
    finally:
        ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 0)
        ctx.set_fp64_sweep(m.PB_SWEEP_PAIRWISE)
    e32_pw, _i, _g, _q = ctx.pb_solve_batch(
        small_batch, m.Params(tol=1e-8, precision=m.PB_FP32_IR, precond_leaf=16))
    assert np.max(np.abs(e_pw - e_pt) / np.abs(e_pt)) <= 1e-10
    assert np.abs(g_pw - g_pt).max() <= 1e-8 * np.abs(g_pt).max()
    assert np.abs(q_pw - q_pt).max() <= 1e-8 * np.abs(q_pt).max()
    assert np.max(np.abs(e32_pw - e_pt) / np.abs(e_pt)) <= 1e-6
    assert np.max(np.abs(e32_pt - e_pt) / np.abs(e_pt)) <= 1e-6


def test_batch_autotune_and_item_lengths(pb, small_batch):
    """The batch autotuner keeps one of its candidates in the context; batched
    solves agree across pairwise item lengths (FP64 to rounding) and after
    tuning (refined FP32 within 1e-6 of FP64)."""
    m, ctx = pb
    P64 = m.Params(tol=1e-12, precond_leaf=16)
    P32 = m.Params(tol=1e-8, precision=m.PB_FP32_IR, precond_leaf=16)
    try:
        e_ref = None
        for tiles in (1, 4, 32):
            ctx.set_batch_tiles(tiles)
            assert ctx.get_batch_tiles() == tiles
            e, _i, _g, _q = ctx.pb_solve_batch(small_batch, P64)
            _say(f"batch tiles={tiles}: E[0]={e[0]:.12f}")
            if e_ref is None:
                e_ref = e
            assert np.max(np.abs(e - e_ref) / np.abs(e_ref)) <= 1e-10
        kind, tiles = ctx.pb_autotune_batch(small_batch, P32)
        _say(f"batch autotune: kind={kind} tiles={tiles}")
        assert (kind, tiles) in {(m.PB_SWEEP_PAIRWISE, t) for t in (2, 4, 8, 16, 32)} or kind == 1
        assert ctx.get_sweep_config()[0] == kind
        if kind == m.PB_SWEEP_PAIRWISE:
            assert ctx.get_batch_tiles() == tiles
        e32, _i, _g, _q = ctx.pb_solve_batch(small_batch, P32)
        assert np.max(np.abs(e32 - e_ref) / np.abs(e_ref)) <= 1e-6
    finally:
        ctx.set_batch_tiles(4)
        ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 0)
