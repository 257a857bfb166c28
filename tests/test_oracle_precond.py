"""Pins of the preconditioner oracle (Sec. 2.2.4) against properties the
section fixes: the leaves partition the elements, hold at most N0 each and
only split clusters above N0; with one leaf M = A, so left-preconditioned
GMRES converges in one step; the preconditioned solve reaches the dense-LU
solution."""
import numpy as np
import pytest

import synth
from oracle import dsbi, precond


def _star(freq=8, r0=8.0, nc=6, seed=61):
    w = synth.star_protein(freq=freq, r0=r0, n_charges=nc, seed=seed)
    return w, dsbi.geometry(w.verts, w.tris)


@pytest.mark.parametrize("n0", [1, 7, 32, 100])
def test_leaves_partition_and_respect_leaf_size(n0):
    w, g = _star(freq=10)
    L = precond.leaves(g.cen, n0)
    allidx = np.concatenate(L)
    assert np.array_equal(np.sort(allidx), np.arange(g.n))
    assert max(len(x) for x in L) <= n0
    for x in L:
        assert np.all(np.diff(x) > 0)


def test_leaves_are_octree_cells():
    """Every leaf's points fit in one cube of the recursive subdivision: the
    bounding box of a leaf never straddles a parent split plane, so leaves of
    the same parent are separated along some axis."""
    w, g = _star(freq=10)
    L = precond.leaves(g.cen, 16)
    lo = g.cen.min(0)
    hi = g.cen.max(0)
    c0 = 0.5 * (lo + hi)
    # first split: each leaf lies entirely on one side of the root centre
    for x in L:
        p = g.cen[x]
        for k in range(3):
            side = p[:, k] >= c0[k]
            assert side.all() or (~side).all()


def test_single_leaf_preconditioner_is_exact_inverse():
    w, g = _star(freq=4, r0=6.0)
    b = dsbi.source(g, w.pos, w.q, 1.0)
    x, info, M = precond.solve_preconditioned(g, 80.0, 0.1257, b, n0=10 ** 6, tol=1e-12)
    assert len(M.leaves) == 1
    assert info.iters == 1
    ref = np.linalg.solve(dsbi.dense_matrix(g, 80.0, 0.1257), b)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_preconditioned_solve_reaches_dense_solution_faster():
    w, g = _star(freq=6, r0=8.0)
    b = dsbi.source(g, w.pos, w.q, 1.0)
    ref = np.linalg.solve(dsbi.dense_matrix(g, 80.0, 0.1257), b)
    x, info, M = precond.solve_preconditioned(g, 80.0, 0.1257, b, n0=16, tol=1e-12)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    _x0, plain = dsbi.gmres(lambda v: dsbi.matvec(g, 80.0, 0.1257, v), b, tol=1e-12)
    assert info.iters < plain.iters


def test_block_apply_is_the_inverse_of_the_leaf_blocks():
    w, g = _star(freq=5, r0=7.0)
    M = precond.BlockDiagonal(g, 80.0, 0.1257, 16)
    A = dsbi.dense_matrix(g, 80.0, 0.1257)
    n = g.n
    rng = np.random.default_rng(1)
    z = rng.normal(size=2 * n)
    y = M.apply(z)
    for idx in M.leaves:
        rows = np.concatenate([idx, n + idx])
        B = A[np.ix_(rows, rows)]
        assert np.allclose(B @ y[rows], z[rows], rtol=0, atol=1e-11 * np.abs(z).max())
