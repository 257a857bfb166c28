"""FP64 CPU oracle of the DSBI Poisson-Boltzmann path (plain and slow).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does, and this package imports nothing from the HIP library.

Each function follows one passage of the paper:

* :func:`geometry`      centroids x_i, unit normals, areas Delta s_i of the
                        flat triangles (Sec. 2.2.2, collocation points).
* :func:`source`        S1, S2 of eq. source_terms.
* :func:`matvec`        left-hand sides of eqs. eqbim_5/eqbim_6 (j = i omitted).
* :func:`gmres`         restarted GMRES (Saad & Schultz, cited in Sec. 2.2.2).
* :func:`energy`        E_sol of eq. solvation_energy, in kcal/mol.
* :func:`dense_matrix`  the same linear system assembled densely.
* :func:`forces`        dE_sol/d(charge positions, charges) by the adjoint
                        method (not in the paper; a plain Lagrangian derivation).

Units: lengths in Angstrom, charges in e_c.  G0 = 1/(4 pi r) and S1 carries
1/eps_in, so the unknowns are the physical potential (e_c/A, Gaussian-type,
phi = q/(eps r)) divided by 4 pi; E_sol in kcal/mol is therefore
332.0716 * 4 pi * (1/2) sum_k q_k phi_reac(y_k) (Sec. 2.1 units paragraph).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from ._clib import lib, ptr, f64

C_UNITS = 332.0716          # e_c^2/A -> kcal/mol (Sec. 2.1)


@dataclass
class Geometry:
    cen: np.ndarray     # [N, 3] centroids
    nrm: np.ndarray     # [N, 3] unit outward normals
    area: np.ndarray    # [N] triangle areas

    @property
    def n(self) -> int:
        return int(self.area.shape[0])


def geometry(verts: np.ndarray, tris: np.ndarray) -> Geometry:
    """Centroid, unit normal and area of each flat triangle (v0, v1, v2):
    x = (v0+v1+v2)/3, m = (v1-v0) x (v2-v0), area = |m|/2, n = m/|m|."""
    v0 = verts[tris[:, 0]]
    v1 = verts[tris[:, 1]]
    v2 = verts[tris[:, 2]]
    cen = (v0 + v1 + v2) / 3.0
    m = np.cross(v1 - v0, v2 - v0)
    mn = np.sqrt(np.sum(m * m, axis=1))
    return Geometry(f64(cen), f64(m / mn[:, None]), f64(0.5 * mn))


def _ratios(eps_in: float, eps_out: float) -> float:
    return eps_out / eps_in


def source(g: Geometry, pos: np.ndarray, q: np.ndarray, eps_in: float, rows=None):
    """b = [S1; S2] at the centroids (eq. source_terms)."""
    pos = f64(pos)
    q = f64(q)
    rr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = g.n if rr is None else rr.shape[0]
    s1 = np.empty(m)
    s2 = np.empty(m)
    lib().orc_source(g.n, ptr(g.cen), ptr(g.nrm), q.shape[0], ptr(pos), ptr(q), float(eps_in),
                     m, ptr(rr), ptr(s1), ptr(s2))
    return np.concatenate([s1, s2]) if rr is None else (s1, s2)


def matvec(g: Geometry, eps: float, kappa: float, xi: np.ndarray, rows=None,
           transpose: bool = False, with_abs: bool = False):
    """y = A xi for xi = [phi; psi] (eqs. eqbim_5/eqbim_6).  With ``rows``
    only those rows of each block are evaluated and ``(y1, y2)`` (and the
    absolute term sums when ``with_abs``) are returned."""
    n = g.n
    xi = f64(xi)
    a, b = xi[:n].copy(), xi[n:].copy()
    rr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = n if rr is None else rr.shape[0]
    y1, y2 = np.empty(m), np.empty(m)
    ab1 = np.empty(m) if with_abs else None
    ab2 = np.empty(m) if with_abs else None
    fn = lib().orc_matvec_t if transpose else lib().orc_matvec
    fn(n, ptr(g.cen), ptr(g.nrm), ptr(g.area), float(eps), float(kappa), ptr(a), ptr(b),
       m, ptr(rr), ptr(y1), ptr(y2), ptr(ab1), ptr(ab2))
    if rr is None and not with_abs:
        return np.concatenate([y1, y2])
    if with_abs:
        return y1, y2, ab1, ab2
    return y1, y2


def dense_matrix(g: Geometry, eps: float, kappa: float) -> np.ndarray:
    """The 2N x 2N matrix of :func:`matvec` (tiny meshes only)."""
    A = np.empty((2 * g.n, 2 * g.n))
    lib().orc_assemble(g.n, ptr(g.cen), ptr(g.nrm), ptr(g.area), float(eps), float(kappa), ptr(A))
    return A


@dataclass
class GmresInfo:
    converged: bool
    iters: int          # Arnoldi steps (one matvec each)
    matvecs: int        # all matvecs, including true-residual checks
    rel_residual: float
    restarts: int


def gmres(apply_A, b: np.ndarray, restart: int = 10, tol: float = 1e-6,
          max_iter: int = 1000, x0=None):
    """Restarted GMRES(m) of Saad & Schultz: Arnoldi with modified Gram-
    Schmidt, Givens rotations on the Hessenberg matrix, least-squares update
    at the end of each cycle.  A cycle ends early when the Arnoldi residual
    estimate |g_{j+1}| / |b| reaches ``tol``; the solve stops only when the
    true residual |b - A x| / |b| does."""
    b = f64(b)
    nb = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else f64(x0).copy()
    if nb == 0.0:
        return x, GmresInfo(True, 0, 0, 0.0, 0)
    iters = matvecs = restarts = 0
    m = int(restart)
    while True:
        if x0 is None and iters == 0:
            r = b.copy()
        else:
            r = b - apply_A(x)
            matvecs += 1
        beta = float(np.linalg.norm(r))
        rel = beta / nb
        if rel <= tol:
            return x, GmresInfo(True, iters, matvecs, rel, restarts)
        if iters >= max_iter:
            return x, GmresInfo(False, iters, matvecs, rel, restarts)
        V = np.zeros((m + 1, b.shape[0]))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = apply_A(V[j])
            iters += 1
            matvecs += 1
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            k = j + 1
            happy = hn == 0.0
            if not happy:
                V[j + 1] = w / hn
            if abs(gvec[j + 1]) / nb <= tol or iters >= max_iter or happy:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (gvec[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + V[:k].T @ y
        restarts += 1
        x0 = x  # later cycles start from the current iterate


def energy_terms(g: Geometry, eps: float, kappa: float, xi: np.ndarray,
                 pos: np.ndarray, with_grad: bool = False):
    """Per-charge reaction potential P_k = sum_j [K1(y_k,x_j) psi_j +
    K2(y_k,x_j) phi_j] a_j (the integral of eq. solvation_energy), and its
    gradient in y_k when asked."""
    n = g.n
    xi = f64(xi)
    phi, psi = xi[:n].copy(), xi[n:].copy()
    pos = f64(pos)
    nc = pos.shape[0]
    P = np.empty(nc)
    G = np.empty((nc, 3)) if with_grad else None
    lib().orc_reaction(n, ptr(g.cen), ptr(g.nrm), ptr(g.area), float(eps), float(kappa),
                       ptr(phi), ptr(psi), nc, ptr(pos), ptr(P), ptr(G))
    return (P, G) if with_grad else P


def energy(g: Geometry, eps: float, kappa: float, xi: np.ndarray, pos: np.ndarray,
           q: np.ndarray) -> float:
    """E_sol in kcal/mol: (1/2) sum_k q_k phi_reac(y_k), times 4 pi (BIE
    units) and 332.0716."""
    P = energy_terms(g, eps, kappa, xi, pos)
    return float(C_UNITS * 4.0 * math.pi * 0.5 * np.sum(f64(q) * P))


@dataclass
class Solution:
    geom: Geometry
    b: np.ndarray
    xi: np.ndarray
    e_solv: float
    info: GmresInfo


def solve(verts, tris, pos, q, eps_in=1.0, eps_out=80.0, kappa=0.1257, tol=1e-6,
          restart=10, max_iter=1000) -> Solution:
    """Full FP64 DSBI solve: geometry, sources, GMRES on eqs. eqbim_5/6, E_sol."""
    g = geometry(f64(verts), np.asarray(tris))
    eps = _ratios(eps_in, eps_out)
    b = source(g, pos, q, eps_in)
    xi, info = gmres(lambda v: matvec(g, eps, kappa, v), b, restart=restart, tol=tol,
                     max_iter=max_iter)
    e = energy(g, eps, kappa, xi, pos, q)
    return Solution(g, b, xi, e, info)


def solve_dense(verts, tris, pos, q, eps_in=1.0, eps_out=80.0, kappa=0.1257) -> Solution:
    """Same system solved by LU (numpy/LAPACK) -- tiny meshes only."""
    g = geometry(f64(verts), np.asarray(tris))
    eps = _ratios(eps_in, eps_out)
    b = source(g, pos, q, eps_in)
    xi = np.linalg.solve(dense_matrix(g, eps, kappa), b)
    e = energy(g, eps, kappa, xi, pos, q)
    return Solution(g, b, xi, e, GmresInfo(True, 0, 0, 0.0, 0))


def adjoint_rhs(g: Geometry, eps: float, kappa: float, pos, q) -> np.ndarray:
    """w = B^T q, with E = 2 pi c_u q^T B xi."""
    pos = f64(pos)
    q = f64(q)
    w1 = np.empty(g.n)
    w2 = np.empty(g.n)
    lib().orc_adjoint_rhs(g.n, ptr(g.cen), ptr(g.nrm), ptr(g.area), float(eps), float(kappa),
                          pos.shape[0], ptr(pos), ptr(q), ptr(w1), ptr(w2))
    return np.concatenate([w1, w2])


def forces(sol: Solution, pos, q, eps_in=1.0, eps_out=80.0, kappa=0.1257, tol=1e-10,
           restart=10, max_iter=2000, lam=None):
    """dE_sol/dy_k [Nc,3] (kcal/mol/A) and dE_sol/dq_k [Nc] (kcal/mol/e_c)
    for a fixed surface, by the adjoint method:
        E = 2 pi c_u q^T B xi,  A xi = C(y) q,  A^T lam = B^T q,
        dE/dq = 2 pi c_u (B xi + C^T lam),
        dE/dy_k = 2 pi c_u q_k (grad_y (B xi)_k + sum_i lam_i grad_y C_ik).
    Returns (dE_dpos, dE_dq, lam, info)."""
    g = sol.geom
    eps = _ratios(eps_in, eps_out)
    pos = f64(pos)
    q = f64(q)
    w = adjoint_rhs(g, eps, kappa, pos, q)
    info = None
    if lam is None:
        lam, info = gmres(lambda v: matvec(g, eps, kappa, v, transpose=True), w,
                          restart=restart, tol=tol, max_iter=max_iter)
    n = g.n
    P, gP = energy_terms(g, eps, kappa, sol.xi, pos, with_grad=True)
    nc = pos.shape[0]
    c = np.empty(nc)
    gc = np.empty((nc, 3))
    l1, l2 = f64(lam[:n]).copy(), f64(lam[n:]).copy()
    lib().orc_source_adjoint(n, ptr(g.cen), ptr(g.nrm), float(eps_in), ptr(l1), ptr(l2),
                             nc, ptr(pos), ptr(c), ptr(gc))
    k = 2.0 * math.pi * C_UNITS
    dE_dq = k * (P + c)
    dE_dpos = k * q[:, None] * (gP + gc)
    return dE_dpos, dE_dq, lam, info


def potential(g: Geometry, eps: float, kappa: float, xi: np.ndarray, pos, q, eps_in: float,
              points):
    """Potential inside the molecule (eq. eq_inside) at points [M, 3]:
    reaction part sum_j [K1(x, x_j) psi_j + K2(x, x_j) phi_j] a_j and total
    = reaction + S1(x).  BIE units (physical e_c/A divided by 4 pi)."""
    pts = f64(points)
    reac = energy_terms(g, eps, kappa, xi, pts)
    coul = np.empty(pts.shape[0])
    pos = f64(pos)
    q = f64(q)
    lib().orc_coulomb(pts.shape[0], ptr(pts), q.shape[0], ptr(pos), ptr(q), float(eps_in), 0,
                      ptr(coul))
    return reac, reac + coul


def coulomb_energy(pos, q, eps_in: float) -> float:
    """(1/2) sum_k q_k S1(y_k) without the self terms, in kcal/mol: the
    difference between E_free (eq. free_energy) and E_sol."""
    pos = f64(pos)
    q = f64(q)
    out = np.empty(q.shape[0])
    lib().orc_coulomb(q.shape[0], ptr(pos), q.shape[0], ptr(pos), ptr(q), float(eps_in), 1,
                      ptr(out))
    return float(C_UNITS * 4.0 * math.pi * 0.5 * np.sum(q * out))

