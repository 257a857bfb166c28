"""Treecode matvec of Sec. 2.2.3 (FP64 CPU oracle).

TEST INFRASTRUCTURE ONLY (part of the oracle).

The matvec sums of eqs. eqbim_5/6 are n-body potentials whose kernels K1..K4
are built from G0 = 1/r and G_kappa = exp(-kappa r)/r (4 pi scaled, as in the
rest of the oracle) and their normal derivatives.  The treecode of the paper
(particle-cluster form, eq. particle_cluster_form):

* the collocation points are clustered by the octree of Sec. 2.2.3 (reading
  R14 of the design notes: the same subdivision the preconditioner uses, all
  levels kept);
* for each target x_i the tree is walked from the root; a cluster c that
  satisfies the multipole acceptance criterion r_c / R <= theta, with
  R = |x_i - x_c|, contributes a p-th order Cartesian Taylor approximation
  about its centre x_c; a cluster that fails it is opened, and a leaf that
  fails it is summed directly (j != i).

Readings where the paper is silent (listed in the design notes):

* cluster centre x_c = midpoint of the tight bounding box of the cluster's
  points, r_c = half of that box's diagonal;
* each of the four kernel sums is replaced by the p-th order Taylor
  polynomial, in the source position y about x_c, of that kernel: with
  T^k(F; x, x_c) the coefficients of F(x - x_c - h) in the source offset h,
  a cluster's sum_j w_j F(x - x_j) becomes sum_{|k| <= p} T^k M^k,
  M^k = sum_j w_j h_j^k; a source normal derivative is part of the kernel
  being expanded, n_j . grad_y F = sum_d n_jd (k_d + 1) T^(k + e_d) h^k, so
  its moments carry the normal, D_d^k = sum_j v_j n_jd h_j^k; a target normal
  derivative acts on the coefficients, grad_x T^m = -(m_d + 1) T^(m + e_d).
  Coefficients up to order p + 2 are used (K4 has both derivatives).

The Taylor coefficients are obtained here by truncated power-series
arithmetic in the three components of h (composition of s = |R - h|^2 with
s^(-1/2), s^(1/2) and exp), not by a recurrence.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from ._clib import f64
from .dsbi import Geometry

MAX_DEPTH = 40


# ---- multi-indices and truncated series ------------------------------------

def multi_indices(order: int):
    """All k = (k1, k2, k3) with |k| <= order, graded by |k|."""
    out = []
    for n in range(order + 1):
        for k1 in range(n, -1, -1):
            for k2 in range(n - k1, -1, -1):
                out.append((k1, k2, n - k1 - k2))
    return out


class SeriesAlgebra:
    """Truncated power series in h = (h1, h2, h3) up to total degree P whose
    coefficients are arrays over a batch of targets: shape [n_terms, batch]."""

    def __init__(self, P: int):
        self.P = P
        self.ks = multi_indices(P)
        self.index = {k: i for i, k in enumerate(self.ks)}
        self.pairs = []   # (i_a, i_b, i_c) with k_a + k_b = k_c
        for ia, ka in enumerate(self.ks):
            for ib, kb in enumerate(self.ks):
                kc = (ka[0] + kb[0], ka[1] + kb[1], ka[2] + kb[2])
                if sum(kc) <= P:
                    self.pairs.append((ia, ib, self.index[kc]))

    def mul(self, a, b):
        c = np.zeros_like(a)
        for ia, ib, ic in self.pairs:
            c[ic] += a[ia] * b[ib]
        return c

    def compose(self, coef, t):
        """sum_n coef[n] t^n for a series t with zero constant term."""
        out = np.zeros_like(t)
        out[0] = coef[0]
        power = np.zeros_like(t)
        power[0] = 1.0
        for n in range(1, self.P + 1):
            power = self.mul(power, t)
            out += coef[n] * power
        return out


def taylor_coefficients(R: np.ndarray, kappa: float, P: int):
    """Coefficients T^k(F; R) of F(R - h) = sum_k T^k h^k for F = G0 and
    F = G_kappa, |k| <= P, for a batch of separations R [batch, 3].
    Returns (alg, T0 [n_terms, batch], Tk [n_terms, batch])."""
    alg = SeriesAlgebra(P)
    R = f64(R)
    nb = R.shape[0]
    s = np.zeros((len(alg.ks), nb))
    rho2 = np.sum(R * R, axis=1)
    s[0] = rho2
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        s[alg.index[tuple(e)]] = -2.0 * R[:, d]
        e[d] = 2
        if P >= 2:
            s[alg.index[tuple(e)]] = 1.0
    t = s.copy()
    t[0] = 0.0
    # s^(-1/2) and s^(1/2) about s0 = rho^2: binomial series
    inv = np.empty((P + 1, nb))
    sq = np.empty((P + 1, nb))
    for n in range(P + 1):
        inv[n] = _binom(-0.5, n) * rho2 ** (-0.5 - n)
        sq[n] = _binom(0.5, n) * rho2 ** (0.5 - n)
    g0 = alg.compose(inv, t)
    if kappa == 0.0:
        return alg, g0, g0.copy()
    r = alg.compose(sq, t)
    # exp(-kappa r) = exp(-kappa rho) exp(-kappa (r - rho))
    u = -kappa * r
    u[0] = 0.0
    fact = np.empty((P + 1, nb))
    e0 = np.exp(-kappa * np.sqrt(rho2))
    for n in range(P + 1):
        fact[n] = e0 / math.factorial(n)
    ex = alg.compose(fact, u)
    return alg, g0, alg.mul(ex, g0)


def _binom(a: float, n: int) -> float:
    out = 1.0
    for m in range(n):
        out *= (a - m) / (m + 1)
    return out


# ---- tree ------------------------------------------------------------------

@dataclass
class Node:
    idx: np.ndarray          # point indices of the cluster
    center: np.ndarray       # x_c
    radius: float            # r_c
    children: list


def build_tree(cen: np.ndarray, n0: int) -> Node:
    """Octree of Sec. 2.2.3 with the subdivision rule of reading R14; every
    node carries its tight-box centre and half-diagonal."""
    cen = f64(cen)
    lo = cen.min(axis=0)
    hi = cen.max(axis=0)

    def make(idx, c, h, depth):
        p = cen[idx]
        blo = p.min(axis=0)
        bhi = p.max(axis=0)
        node = Node(idx, 0.5 * (blo + bhi), 0.5 * float(np.linalg.norm(bhi - blo)), [])
        if idx.shape[0] <= n0 or depth >= MAX_DEPTH:
            return node
        octant = ((p[:, 0] >= c[0]).astype(np.int64) + 2 * (p[:, 1] >= c[1]).astype(np.int64)
                  + 4 * (p[:, 2] >= c[2]).astype(np.int64))
        for o in range(8):
            sub = idx[octant == o]
            if sub.shape[0] == 0:
                continue
            sgn = np.array([1.0 if o & 1 else -1.0, 1.0 if o & 2 else -1.0,
                            1.0 if o & 4 else -1.0])
            node.children.append(make(sub, c + sgn * (0.5 * h), 0.5 * h, depth + 1))
        return node

    return make(np.arange(cen.shape[0], dtype=np.int64), 0.5 * (lo + hi),
                float(np.max(0.5 * (hi - lo))), 0)


def interaction_lists(tree: Node, cen: np.ndarray, theta: float, rows=None):
    """For every target (or those in `rows`): the clusters accepted by the MAC
    (far) and the leaves summed directly (near), from a walk that starts at
    the root."""
    cen = f64(cen)
    n = cen.shape[0]
    far = [[] for _ in range(n)]
    near = [[] for _ in range(n)]
    for i in (range(n) if rows is None else rows):
        x = cen[i]
        stack = [tree]
        while stack:
            c = stack.pop()
            R = float(np.linalg.norm(x - c.center))
            if R > 0.0 and c.radius <= theta * R:
                far[i].append(c)
            elif not c.children:
                near[i].append(c)
            else:
                stack.extend(reversed(c.children))
    return far, near


# ---- matvec ----------------------------------------------------------------

def _direct_rows(g: Geometry, eps: float, kappa: float, phi, psi, i: int, j: np.ndarray):
    """Row i of both blocks summed over sources j (j != i), kernels of C3."""
    j = j[j != i]
    d = g.cen[i] - g.cen[j]
    rho = np.sqrt(np.sum(d * d, axis=1))
    ir = 1.0 / rho
    e = np.exp(-kappa * rho)
    tp2 = (1.0 + kappa * rho) * e
    cx = d @ g.nrm[i]
    cy = np.sum(g.nrm[j] * d, axis=1)
    nn = g.nrm[j] @ g.nrm[i]
    k1 = ir - e * ir
    k2 = (eps * tp2 - 1.0) * cy * ir ** 3
    k3 = (tp2 / eps - 1.0) * cx * ir ** 3
    h0 = (nn - 3.0 * cx * cy * ir * ir) * ir ** 3
    k4 = (tp2 - 1.0) * h0 - kappa * kappa * cx * cy * ir * ir * e * ir
    a = g.area[j]
    return (np.sum(a * (k1 * psi[j] + k2 * phi[j])), np.sum(a * (k3 * psi[j] + k4 * phi[j])))


def moments(g: Geometry, phi, psi, c: Node, p: int):
    """M^k = sum_j a_j psi_j h_j^k and D_d^k = sum_j a_j phi_j n_jd h_j^k at
    h_j = x_j - x_c, |k| <= p.  Returns M [n_terms], D [3, n_terms]."""
    ks = multi_indices(p)
    h = g.cen[c.idx] - c.center
    w = g.area[c.idx] * psi[c.idx]
    v = g.area[c.idx] * phi[c.idx]
    nr = g.nrm[c.idx]
    M = np.empty(len(ks))
    D = np.empty((3, len(ks)))
    for t, k in enumerate(ks):
        hk = h[:, 0] ** k[0] * h[:, 1] ** k[1] * h[:, 2] ** k[2]
        M[t] = np.sum(w * hk)
        for d in range(3):
            D[d, t] = np.sum(v * nr[:, d] * hk)
    return M, D


def _shift(k, d, by=1):
    kp = list(k)
    kp[d] += by
    return tuple(kp)


def far_rows(T0, Tk, alg: SeriesAlgebra, M, D, nrm_t, eps: float, p: int):
    """Far-field rows 1 and 2 for a batch of targets (normals nrm_t [batch, 3])
    from one cluster's moments; T0, Tk hold the coefficients to order p + 2."""
    ks = multi_indices(p)
    r1 = np.zeros(T0.shape[1])
    r2 = np.zeros(T0.shape[1])
    for t, k in enumerate(ks):
        i = alg.index[k]
        # K1: G0 - Gk on psi moments
        r1 += (T0[i] - Tk[i]) * M[t]
        for e in range(3):
            je = alg.index[_shift(k, e)]
            # K3: n_x . grad_x (G0 - Gk / eps) on psi moments
            r2 += -(k[e] + 1.0) * nrm_t[:, e] * (T0[je] - Tk[je] / eps) * M[t]
        for d in range(3):
            kd = _shift(k, d)
            jd = alg.index[kd]
            # K2: n_y . grad_y (eps Gk - G0) on phi moments
            r1 += (k[d] + 1.0) * (eps * Tk[jd] - T0[jd]) * D[d, t]
            for e in range(3):
                jde = alg.index[_shift(kd, e)]
                # K4: n_x . grad_x n_y . grad_y (Gk - G0)
                r2 += (-(kd[e] + 1.0) * (k[d] + 1.0) * nrm_t[:, e]
                       * (Tk[jde] - T0[jde]) * D[d, t])
    return r1, r2


class TreeOperator:
    """The treecode matvec for one geometry: the tree, every target's
    interaction lists and the Taylor coefficients of each accepted
    (target, cluster) pair are formed once; apply() then needs only the
    moments of the current vector.  With `rows`, only those rows are formed
    and apply() returns (y1, y2) for them."""

    def __init__(self, g: Geometry, eps: float, kappa: float, theta: float, p: int, n0: int,
                 rows=None):
        self.g, self.eps, self.kappa, self.p = g, eps, kappa, p
        self.rows = None if rows is None else np.asarray(rows)
        self.tree = build_tree(g.cen, n0)
        far, near = interaction_lists(self.tree, g.cen, theta, rows)
        targets = range(g.n) if rows is None else rows
        self.near = [(i, np.concatenate([c.idx for c in near[i]])) for i in targets if near[i]]
        users = {}
        for i in targets:
            for c in far[i]:
                users.setdefault(id(c), (c, []))[1].append(i)
        self.far = []
        for c, tl in users.values():
            tl = np.asarray(tl, dtype=np.int64)
            alg, T0, Tk = taylor_coefficients(g.cen[tl] - c.center, kappa, p + 2)
            self.far.append((c, tl, alg, T0, Tk))

    def apply(self, xi: np.ndarray):
        g, eps, kappa, p = self.g, self.eps, self.kappa, self.p
        n = g.n
        xi = f64(xi)
        phi, psi = xi[:n], xi[n:]
        s1 = np.zeros(n)
        s2 = np.zeros(n)
        for i, j in self.near:
            a1, a2 = _direct_rows(g, eps, kappa, phi, psi, i, j)
            s1[i] += a1
            s2[i] += a2
        for c, tl, alg, T0, Tk in self.far:
            M, D = moments(g, phi, psi, c, p)
            r1, r2 = far_rows(T0, Tk, alg, M, D, g.nrm[tl], eps, p)
            np.add.at(s1, tl, r1)
            np.add.at(s2, tl, r2)
        inv4pi = 1.0 / (4.0 * np.pi)
        if self.rows is not None:
            r = self.rows
            return (0.5 * (1.0 + eps) * phi[r] - inv4pi * s1[r],
                    0.5 * (1.0 + 1.0 / eps) * psi[r] - inv4pi * s2[r])
        y = np.empty(2 * n)
        y[:n] = 0.5 * (1.0 + eps) * phi - inv4pi * s1
        y[n:] = 0.5 * (1.0 + 1.0 / eps) * psi - inv4pi * s2
        return y


def matvec(g: Geometry, eps: float, kappa: float, xi: np.ndarray, theta: float, p: int,
           n0: int, rows=None):
    """y = A xi with the pair sums replaced by the treecode approximation.
    With `rows`, only those rows of both blocks are formed and (y1, y2) for
    them is returned."""
    return TreeOperator(g, eps, kappa, theta, p, n0, rows).apply(xi)


def solve(verts, tris, pos, q, theta: float, p: int, n0: int, eps_in=1.0, eps_out=80.0,
          kappa=0.1257, tol=1e-6, restart=10, max_iter=1000):
    """The FP64 DSBI solve of the oracle with the treecode matvec in GMRES."""
    from .dsbi import _ratios, energy, geometry, gmres, source
    g = geometry(f64(verts), np.asarray(tris))
    eps = _ratios(eps_in, eps_out)
    b = source(g, pos, q, eps_in)
    op = TreeOperator(g, eps, kappa, theta, p, n0)
    xi, info = gmres(op.apply, b, restart=restart, tol=tol, max_iter=max_iter)
    return energy(g, eps, kappa, xi, pos, q), xi, info


def counts(g: Geometry, theta: float, n0: int):
    """(particle-particle pairs, particle-cluster interactions) of one matvec."""
    tree = build_tree(g.cen, n0)
    far, near = interaction_lists(tree, g.cen, theta)
    pp = sum(sum(c.idx.shape[0] for c in near[i]) - 1 for i in range(g.n))
    pc = sum(len(f) for f in far)
    return pp, pc
