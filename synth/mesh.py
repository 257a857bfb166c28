"""Closed triangulated surfaces: Class-I geodesic icospheres and star shapes.

The frequency-``n`` Class-I subdivision splits each of the 20 icosahedron
faces into an ``n x n`` triangular lattice and projects every lattice point
once onto the unit sphere, giving ``20 n**2`` triangles and ``10 n**2 + 2``
vertices for any ``n >= 1``.  Triangles are listed counter-clockwise as seen
from outside, so ``(v1 - v0) x (v2 - v0)`` points away from the enclosed
volume.

Everything here uses only +, -, *, / and sqrt, each of which IEEE-754 rounds
correctly, so the same seed gives bit-identical arrays on any x86-64 host.
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0


def _icosahedron():
    """Unit icosahedron: 12 vertices (cyclic permutations of (0, +-1, +-g))
    and its 20 faces, oriented outward, listed in lexicographic order."""
    g = _GOLDEN
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts.append((0.0, s1, s2 * g))
            pts.append((s1, s2 * g, 0.0))
            pts.append((s2 * g, 0.0, s1))
    v = np.array(pts, dtype=np.float64)
    faces = []
    for a in range(12):
        for b in range(a + 1, 12):
            if abs(np.sum((v[a] - v[b]) ** 2) - 4.0) > 1e-9:
                continue
            for c in range(b + 1, 12):
                if (abs(np.sum((v[a] - v[c]) ** 2) - 4.0) < 1e-9
                        and abs(np.sum((v[b] - v[c]) ** 2) - 4.0) < 1e-9):
                    nrm = np.cross(v[b] - v[a], v[c] - v[a])
                    if np.dot(nrm, v[a] + v[b] + v[c]) > 0:
                        faces.append((a, b, c))
                    else:
                        faces.append((a, c, b))
    assert len(faces) == 20
    return v, faces


def icosphere(freq: int, radius: float = 1.0):
    """Class-I geodesic icosphere of frequency ``freq``.

    Returns ``(verts [10 f^2 + 2, 3] float64, tris [20 f^2, 3] int32)``.
    """
    n = int(freq)
    if n < 1:
        raise ValueError("freq must be >= 1")
    iv, faces = _icosahedron()
    # edges of the icosahedron, sorted, with a stable index
    edges = {}
    for (a, b, c) in faces:
        for (u, w) in ((a, b), (b, c), (a, c)):
            key = (min(u, w), max(u, w))
            if key not in edges:
                edges[key] = len(edges)
    edge_keys = sorted(edges)
    edges = {k: i for i, k in enumerate(edge_keys)}
    n_edge_pts = n - 1
    n_int = (n - 1) * (n - 2) // 2
    nv = 12 + 30 * n_edge_pts + 20 * n_int
    P = np.empty((nv, 3), dtype=np.float64)
    P[:12] = iv
    # edge points: k-th point from the lower to the higher vertex id
    for (u, w), e in edges.items():
        if n_edge_pts == 0:
            break
        k = np.arange(1, n, dtype=np.float64)[:, None]
        P[12 + e * n_edge_pts: 12 + (e + 1) * n_edge_pts] = (
            (n - k) * iv[u] + k * iv[w]) / n
    tris = []
    next_id = 12 + 30 * n_edge_pts
    for (a, b, c) in faces:
        vid = np.full((n + 1, n + 1), -1, dtype=np.int64)
        # lattice point (i, j) has weights (n-i-j, i, j) on (a, b, c)
        for i in range(n + 1):
            for j in range(n + 1 - i):
                wa, wb, wc = n - i - j, i, j
                nz = [(vtx, wt) for vtx, wt in ((a, wa), (b, wb), (c, wc)) if wt > 0]
                if len(nz) == 1:
                    vid[i, j] = nz[0][0]
                elif len(nz) == 2:
                    (u, wu), (w, ww) = sorted(nz)
                    vid[i, j] = 12 + edges[(u, w)] * n_edge_pts + (ww - 1)
                else:
                    vid[i, j] = next_id
                    P[next_id] = (wa * iv[a] + wb * iv[b] + wc * iv[c]) / n
                    next_id += 1
        # up triangles (i,j),(i+1,j),(i,j+1); down (i+1,j),(i+1,j+1),(i,j+1)
        for i in range(n):
            for j in range(n - i):
                tris.append((vid[i, j], vid[i + 1, j], vid[i, j + 1]))
                if i + j <= n - 2:
                    tris.append((vid[i + 1, j], vid[i + 1, j + 1], vid[i, j + 1]))
    assert next_id == nv
    T = np.asarray(tris, dtype=np.int32)
    nrm = np.sqrt(np.sum(P * P, axis=1))
    U = P / nrm[:, None]
    return U * float(radius), T


def real_sph_harm(lmax: int, u: np.ndarray) -> dict:
    """Real orthonormal spherical harmonics Y_lm(u), 0 <= l <= lmax, at unit
    vectors ``u [M, 3]``, evaluated as polynomials in (x, y, z).

    Y_l0 = c_l0 Q_l^0(z); for m > 0, Y_lm = sqrt(2) c_lm Q_l^m(z) Re((x+iy)^m)
    and Y_l,-m = sqrt(2) c_lm Q_l^m(z) Im((x+iy)^m), where Q_l^m is the m-th
    derivative of the Legendre polynomial P_l and
    c_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
    """
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    C = [np.ones_like(x)]
    S = [np.zeros_like(x)]
    for m in range(1, lmax + 1):
        C.append(x * C[m - 1] - y * S[m - 1])
        S.append(x * S[m - 1] + y * C[m - 1])
    out = {}
    for m in range(0, lmax + 1):
        # Q_m^m = (2m-1)!!, Q_{m+1}^m = (2m+1) z Q_m^m,
        # (l-m) Q_l^m = (2l-1) z Q_{l-1}^m - (l+m-1) Q_{l-2}^m
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        Q = {m: np.full_like(z, dfact)}
        if m + 1 <= lmax:
            Q[m + 1] = (2 * m + 1) * z * Q[m]
        for l in range(m + 2, lmax + 1):
            Q[l] = ((2 * l - 1) * z * Q[l - 1] - (l + m - 1) * Q[l - 2]) / (l - m)
        for l in range(m, lmax + 1):
            c = math.sqrt((2 * l + 1) / (4 * math.pi)
                          * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                out[(l, 0)] = c * Q[l]
            else:
                out[(l, m)] = math.sqrt(2.0) * c * Q[l] * C[m]
                out[(l, -m)] = math.sqrt(2.0) * c * Q[l] * S[m]
    return out


def draw_shape_coeffs(rng: np.random.Generator, lmax: int = 6) -> dict:
    """a_lm ~ N(0, 1/(l+1)^2) (variance), drawn in (l, m) order, m = -l..l."""
    coef = {}
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            coef[(l, m)] = float(rng.normal(0.0, 1.0 / (l + 1)))
    return coef


def star_radius(u: np.ndarray, r0: float, coef: dict, amp: float = 0.15) -> np.ndarray:
    """r(u) = r0 (1 + amp sum_lm a_lm Y_lm(u)) for unit vectors u [M, 3]."""
    lmax = max(l for (l, _m) in coef)
    Y = real_sph_harm(lmax, u)
    s = np.zeros(u.shape[0])
    for (l, m) in sorted(coef):
        s = s + coef[(l, m)] * Y[(l, m)]
    return r0 * (1.0 + amp * s)


def star_surface(freq: int, r0: float, coef: dict, amp: float = 0.15):
    """Icosphere of frequency ``freq`` with each unit vertex u moved to
    r(u) u.  Star-shaped, hence never self-intersecting."""
    U, T = icosphere(freq, 1.0)
    r = star_radius(U, r0, coef, amp)
    if np.any(r <= 0):
        raise ValueError("star radius must stay positive")
    return U * r[:, None], T
