"""Pins of the treecode oracle (Sec. 2.2.3) against the direct sum, closed-form
derivatives and the convergence the Taylor approximation must show."""
import numpy as np
import pytest

import synth
from oracle import dsbi, treecode as tc

EPS, KAPPA = 80.0, 0.1257


@pytest.fixture(scope="module")
def star8():
    w = synth.star_protein(freq=8, r0=8.0, n_charges=1, seed=7)
    return dsbi.geometry(w.verts, w.tris)


def _g(R, kappa):
    r = np.linalg.norm(R)
    return np.exp(-kappa * r) / r


@pytest.mark.parametrize("kappa", [0.0, KAPPA])
def test_taylor_coefficients_match_closed_form_derivatives(kappa):
    """T^k is the coefficient of h^k in F(R - h): T^0 = F, T^{e_d} = -dF/dR_d,
    T^{2 e_d} = (1/2) d2F/dR_d^2 and T^{e_d + e_e} = d2F/dR_d dR_e, from the
    radial derivatives of exp(-kappa r)/r written out by hand."""
    R = np.array([1.3, -0.7, 2.1])
    alg, T0, Tk = tc.taylor_coefficients(R[None, :], kappa, 3)
    r = np.linalg.norm(R)
    e = np.exp(-kappa * r)
    f1 = -(1.0 + kappa * r) * e / r ** 3                     # F'(r)/r
    f2 = (3.0 + 3.0 * kappa * r + (kappa * r) ** 2) * e / r ** 5
    T = Tk[:, 0]
    assert T[alg.index[(0, 0, 0)]] == pytest.approx(e / r, rel=1e-15)
    for d in range(3):
        k = [0, 0, 0]
        k[d] = 1
        assert T[alg.index[tuple(k)]] == pytest.approx(-f1 * R[d], rel=1e-14)
        for q in range(3):
            k2 = [0, 0, 0]
            k2[d] += 1
            k2[q] += 1
            hess = f2 * R[d] * R[q] + (f1 if d == q else 0.0)
            want = 0.5 * hess if d == q else hess
            assert T[alg.index[tuple(k2)]] == pytest.approx(want, rel=1e-13)
    if kappa == 0.0:
        assert np.array_equal(T0, Tk)


@pytest.mark.parametrize("P", [2, 4, 5])
def test_taylor_remainder_has_the_right_order(P):
    """F(R - h) - sum_{|k|<=P} T^k h^k must shrink like |h|^(P+1): a wrong
    coefficient of any order <= P breaks the ratio under halving h."""
    R = np.array([2.0, -1.5, 1.0])
    alg, T0, Tk = tc.taylor_coefficients(R[None, :], KAPPA, P)
    u = np.array([0.36, -0.48, 0.8])
    errs = []
    for s in (0.2, 0.1):
        h = s * u
        hk = np.array([h[0] ** k[0] * h[1] ** k[1] * h[2] ** k[2] for k in alg.ks])
        errs.append((abs(_g(R - h, KAPPA) - hk @ Tk[:, 0]), abs(1.0 / np.linalg.norm(R - h)
                                                                 - hk @ T0[:, 0])))
    for a in range(2):
        assert errs[0][a] / errs[1][a] > 0.75 * 2.0 ** (P + 1)


def test_tree_lists_partition_every_target_row(star8):
    tree = tc.build_tree(star8.cen, 20)
    far, near = tc.interaction_lists(tree, star8.cen, 0.6)
    for i in range(0, star8.n, 37):
        pts = np.concatenate([c.idx for c in far[i] + near[i]])
        assert np.array_equal(np.sort(pts), np.arange(star8.n))
        for c in far[i]:
            assert i not in set(c.idx.tolist())
            assert c.radius <= 0.6 * np.linalg.norm(star8.cen[i] - c.center)
    # every cluster's radius covers its points
    stack = [tree]
    while stack:
        c = stack.pop()
        assert np.all(np.linalg.norm(star8.cen[c.idx] - c.center, axis=1) <= c.radius * (1 + 1e-14))
        assert c.children or c.idx.shape[0] <= 20
        stack.extend(c.children)


def test_theta_zero_is_the_direct_sum(star8):
    """With theta = 0 only one-point clusters pass the MAC, and their Taylor
    polynomial is exact: the treecode must equal the direct matvec."""
    x = np.random.default_rng(0).normal(size=2 * star8.n)
    ref = dsbi.matvec(star8, EPS, KAPPA, x)
    y = tc.matvec(star8, EPS, KAPPA, x, theta=0.0, p=2, n0=20)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_single_cluster_far_field_converges_in_p(star8):
    """Each kernel's far field at R = 10 r_c approaches the exact cluster sum
    geometrically in p."""
    x = np.random.default_rng(1).normal(size=2 * star8.n)
    phi, psi = x[:star8.n], x[star8.n:]
    idx = np.where(np.linalg.norm(star8.cen - star8.cen[0], axis=1) < 1.5)[0]
    p_ = star8.cen[idx]
    c = tc.Node(idx, 0.5 * (p_.min(0) + p_.max(0)), 0.5 * np.linalg.norm(p_.max(0) - p_.min(0)),
                [])
    u = np.array([0.6, -0.48, 0.64])
    xt = c.center + 10.0 * c.radius * u
    nt = np.array([0.0, 0.6, 0.8])
    # exact cluster sums through the direct-sum helper on a one-target geometry
    g1 = dsbi.Geometry(np.vstack([star8.cen[idx], xt]), np.vstack([star8.nrm[idx], nt]),
                       np.concatenate([star8.area[idx], [0.0]]))
    ph = np.concatenate([phi[idx], [0.0]])
    ps = np.concatenate([psi[idx], [0.0]])
    ex1, ex2 = tc._direct_rows(g1, EPS, KAPPA, ph, ps, len(idx), np.arange(len(idx) + 1))
    errs = []
    for p in range(0, 7):
        alg, T0, Tk = tc.taylor_coefficients((xt - c.center)[None, :], KAPPA, p + 2)
        M, D = tc.moments(star8, phi, psi, c, p)
        r1, r2 = tc.far_rows(T0, Tk, alg, M, D, nt[None, :], EPS, p)
        errs.append(max(abs(r1[0] - ex1) / abs(ex1), abs(r2[0] - ex2) / abs(ex2)))
    assert errs[6] < 1e-5
    assert errs[6] < errs[4] < errs[2] < errs[0]


def test_matvec_error_falls_with_order(star8):
    x = np.random.default_rng(2).normal(size=2 * star8.n)
    ref = dsbi.matvec(star8, EPS, KAPPA, x)
    s = np.abs(ref).max()
    e = [np.abs(tc.matvec(star8, EPS, KAPPA, x, theta=0.5, p=p, n0=20) - ref).max() / s
         for p in (0, 2, 4)]
    assert e[2] < e[1] < e[0] and e[2] < 5e-3
