"""Block-diagonal leaf preconditioner of Sec. 2.2.4 (FP64 CPU oracle).

TEST INFRASTRUCTURE ONLY (part of the oracle).

The tree is the one Sec. 2.2.3 describes for the treecode: the root cluster
is a cube containing all collocation points, and a cluster holding more than
N0 points is divided into its eight child cubes until every leaf holds at
most N0.  The preconditioner M keeps, for each leaf, the interactions of the
leaf's elements with each other (the 2n x 2n block of A on the leaf's
indices) and drops everything else; M y = z is solved leaf by leaf with LU
factorization.  GMRES is applied to the left-preconditioned system
M^-1 A x = M^-1 b, as the section prescribes.

Reading of the tree rule (the paper gives no formula): root centre = the
midpoint of the bounding box of the centroids, root half-width = half of the
largest box extent; a point goes to child octant (x >= cx) + 2 (y >= cy) +
4 (z >= cz); child centres are c +- h/2 and child half-widths h/2; empty
children are dropped; leaves are listed depth first, children in octant
order, points within a leaf in increasing index order.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import lu_factor, lu_solve

from ._clib import lib, ptr, f64
from .dsbi import Geometry, gmres, matvec

MAX_DEPTH = 40


def leaves(cen: np.ndarray, n0: int):
    """Index arrays of the octree leaves, depth first."""
    cen = f64(cen)
    lo = cen.min(axis=0)
    hi = cen.max(axis=0)
    c0 = 0.5 * (lo + hi)
    h0 = float(np.max(0.5 * (hi - lo)))
    out = []

    def split(idx, c, h, depth):
        if idx.shape[0] <= n0 or depth >= MAX_DEPTH:
            # at the depth limit (coincident points) the leaf is cut into
            # consecutive runs of at most n0 points
            for a in range(0, idx.shape[0], n0):
                out.append(idx[a:a + n0])
            return
        p = cen[idx]
        octant = ((p[:, 0] >= c[0]).astype(np.int64) + 2 * (p[:, 1] >= c[1]).astype(np.int64)
                  + 4 * (p[:, 2] >= c[2]).astype(np.int64))
        for o in range(8):
            sub = idx[octant == o]
            if sub.shape[0] == 0:
                continue
            sgn = np.array([1.0 if o & 1 else -1.0, 1.0 if o & 2 else -1.0,
                            1.0 if o & 4 else -1.0])
            split(sub, c + sgn * (0.5 * h), 0.5 * h, depth + 1)

    split(np.arange(cen.shape[0], dtype=np.int64), c0, h0, 0)
    return out


class BlockDiagonal:
    """M = diag(M_1..M_L) on the leaves; apply() returns M^-1 z."""

    def __init__(self, g: Geometry, eps: float, kappa: float, n0: int):
        self.n = g.n
        self.leaves = leaves(g.cen, n0)
        self.lu = []
        for idx in self.leaves:
            m = idx.shape[0]
            B = np.empty((2 * m, 2 * m))
            ii = np.ascontiguousarray(idx, dtype=np.int64)
            lib().orc_assemble_subset(g.n, ptr(g.cen), ptr(g.nrm), ptr(g.area), float(eps),
                                      float(kappa), m, ptr(ii), ptr(B))
            self.lu.append(lu_factor(B))

    def block(self, k: int) -> np.ndarray:
        lu, piv = self.lu[k]
        m2 = lu.shape[0]
        return lu_solve((lu, piv), np.eye(m2))

    def apply(self, z: np.ndarray) -> np.ndarray:
        z = f64(z)
        n = self.n
        y = np.empty_like(z)
        for idx, f in zip(self.leaves, self.lu):
            rhs = np.concatenate([z[idx], z[n + idx]])
            sol = lu_solve(f, rhs)
            m = idx.shape[0]
            y[idx] = sol[:m]
            y[n + idx] = sol[m:]
        return y


def solve_preconditioned(g: Geometry, eps: float, kappa: float, b: np.ndarray, n0: int,
                         tol: float = 1e-6, restart: int = 10, max_iter: int = 1000):
    """GMRES on M^-1 A x = M^-1 b (left preconditioning, Sec. 2.2.4)."""
    M = BlockDiagonal(g, eps, kappa, n0)
    x, info = gmres(lambda v: M.apply(matvec(g, eps, kappa, v)), M.apply(b), restart=restart,
                    tol=tol, max_iter=max_iter)
    return x, info, M
