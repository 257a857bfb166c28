"""Point charges strictly inside a star-shaped surface, kept away from it."""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree


def point_triangle_distance(p: np.ndarray, a: np.ndarray, b: np.ndarray,
                            c: np.ndarray) -> np.ndarray:
    """Exact Euclidean distance from points p [M,3] to triangles (a,b,c) [M,3]
    (row-wise pairs), by locating the closest point in the Voronoi regions of
    the triangle's vertices, edges and face (Ericson, Real-Time Collision
    Detection, 2005, sec. 5.1.5)."""
    ab = b - a
    ac = c - a
    ap = p - a
    d1 = np.einsum("ij,ij->i", ab, ap)
    d2 = np.einsum("ij,ij->i", ac, ap)
    bp = p - b
    d3 = np.einsum("ij,ij->i", ab, bp)
    d4 = np.einsum("ij,ij->i", ac, bp)
    cp = p - c
    d5 = np.einsum("ij,ij->i", ab, cp)
    d6 = np.einsum("ij,ij->i", ac, cp)
    va = d3 * d6 - d5 * d4
    vb = d5 * d2 - d1 * d6
    vc = d1 * d4 - d3 * d2
    M = p.shape[0]
    q = np.empty((M, 3))
    done = np.zeros(M, dtype=bool)

    def put(mask, val):
        nonlocal done
        m = mask & ~done
        if np.any(m):
            q[m] = val[m] if val.ndim == 2 else val
        done |= m

    put((d1 <= 0) & (d2 <= 0), a)
    put((d3 >= 0) & (d4 <= d3), b)
    with np.errstate(divide="ignore", invalid="ignore"):
        v = d1 / (d1 - d3)
        put((vc <= 0) & (d1 >= 0) & (d3 <= 0), a + v[:, None] * ab)
        put((d6 >= 0) & (d5 <= d6), c)
        w = d2 / (d2 - d6)
        put((vb <= 0) & (d2 >= 0) & (d6 <= 0), a + w[:, None] * ac)
        w2 = (d4 - d3) / ((d4 - d3) + (d5 - d6))
        put((va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0), b + w2[:, None] * (c - b))
        denom = 1.0 / (va + vb + vc)
        v3 = vb * denom
        w3 = vc * denom
        put(np.ones(M, dtype=bool), a + v3[:, None] * ab + w3[:, None] * ac)
    return np.sqrt(np.sum((p - q) ** 2, axis=1))


def interior_charges(rng: np.random.Generator, verts: np.ndarray, tris: np.ndarray,
                     inside, n_charges: int, min_dist: float = 1.5,
                     q_var: float = 0.5, batch: int = 4096):
    """Draw ``n_charges`` points uniformly in the ball of radius max|v|, keep
    those with ``inside(p)`` true and at least ``min_dist`` from every
    triangle; then charges q ~ N(0, q_var) (variance), shifted by a common
    amount so that sum(q) is an integer.

    Returns ``(pos [n,3] float64, q [n] float64)``.
    """
    rmax = float(np.max(np.sqrt(np.sum(verts ** 2, axis=1))))
    A = verts[tris[:, 0]]
    B = verts[tris[:, 1]]
    C = verts[tris[:, 2]]
    cen = (A + B + C) / 3.0
    circ = np.max(np.stack([np.sqrt(np.sum((X - cen) ** 2, axis=1)) for X in (A, B, C)]))
    tree = cKDTree(cen)
    accepted = []
    n_acc = 0
    while n_acc < n_charges:
        p = rng.uniform(-rmax, rmax, size=(batch, 3))
        p = p[np.sum(p * p, axis=1) < rmax * rmax]
        p = p[inside(p)]
        if p.shape[0] == 0:
            continue
        near = tree.query_ball_point(p, r=min_dist + circ)
        ok = np.ones(p.shape[0], dtype=bool)
        for k, cand in enumerate(near):
            if not cand:
                continue
            cand = np.asarray(cand)
            d = point_triangle_distance(np.repeat(p[k:k + 1], len(cand), axis=0),
                                        A[cand], B[cand], C[cand])
            if np.min(d) < min_dist:
                ok[k] = False
        p = p[ok]
        take = min(p.shape[0], n_charges - n_acc)
        accepted.append(p[:take])
        n_acc += take
    pos = np.concatenate(accepted, axis=0)
    q = rng.normal(0.0, math.sqrt(q_var), size=n_charges)
    s = float(np.sum(q))
    q = q - (s - round(s)) / n_charges
    return pos, q
