"""Pins of the FP64 oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: each test checks it against a
closed form (Kirkwood/Born, image charge, Gauss law, solid-angle identity), a
library routine (scipy spherical Bessel functions, LAPACK LU), finite
differences of the Green's functions written from their definition, or an
invariant of the continuous problem.
"""
import ctypes
import math

import numpy as np
import pytest
from scipy.special import spherical_kn

import synth
from oracle import dsbi, kirkwood
from oracle._clib import lib

EPS_IN, EPS_OUT, KAPPA = 1.0, 80.0, 0.1257


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, ctypes.c_void_p(a.ctypes.data)


def green(x, nx, y, ny, kappa):
    out, po = _c(np.zeros(4))
    xs = [_c(v) for v in (x, nx, y, ny)]
    lib().orc_green(xs[0][1], xs[1][1], xs[2][1], xs[3][1], float(kappa), po)
    return out


def kernels(x, nx, y, ny, eps, kappa):
    out, po = _c(np.zeros(4))
    xs = [_c(v) for v in (x, nx, y, ny)]
    lib().orc_kernels(xs[0][1], xs[1][1], xs[2][1], xs[3][1], float(eps), float(kappa), po)
    return out


def G_def(x, y, kappa):
    """Eq. eq_potential written from its definition."""
    r = math.sqrt(sum((a - b) ** 2 for a, b in zip(x, y)))
    return math.exp(-kappa * r) / (4.0 * math.pi * r)


def _unit(v):
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("kappa", [0.0, 0.1257, 0.9])
def test_green_normal_derivatives_match_finite_differences(kappa):
    rng = np.random.default_rng(11)
    h = 1e-4
    for _ in range(20):
        x = rng.normal(size=3)
        y = x + _unit(rng.normal(size=3)) * rng.uniform(0.3, 3.0)
        nx = _unit(rng.normal(size=3))
        ny = _unit(rng.normal(size=3))
        g, dny, dnx, dxy = green(x, nx, y, ny, kappa)
        assert g == pytest.approx(G_def(x, y, kappa), rel=1e-14)
        fd_ny = (G_def(x, y + h * ny, kappa) - G_def(x, y - h * ny, kappa)) / (2 * h)
        fd_nx = (G_def(x + h * nx, y, kappa) - G_def(x - h * nx, y, kappa)) / (2 * h)

        def dGdny(xx):
            return (G_def(xx, y + h * ny, kappa) - G_def(xx, y - h * ny, kappa)) / (2 * h)

        fd_xy = (dGdny(x + h * nx) - dGdny(x - h * nx)) / (2 * h)
        scale = abs(g) / np.linalg.norm(x - y)
        assert abs(dny - fd_ny) <= 1e-7 * scale
        assert abs(dnx - fd_nx) <= 1e-7 * scale
        assert abs(dxy - fd_xy) <= 1e-5 * scale / np.linalg.norm(x - y)


def test_kernels_are_the_paper_combinations_of_green_derivatives():
    """K1..K4 (eqs. Eq_K1/Eq_K2) from finite differences of G0 and Gk."""
    rng = np.random.default_rng(12)
    h = 1e-4
    eps = EPS_OUT / EPS_IN
    for _ in range(20):
        x = rng.normal(size=3)
        y = x + _unit(rng.normal(size=3)) * rng.uniform(0.3, 3.0)
        nx = _unit(rng.normal(size=3))
        ny = _unit(rng.normal(size=3))

        def dny(k, xx=x):
            return (G_def(xx, y + h * ny, k) - G_def(xx, y - h * ny, k)) / (2 * h)

        def dnx(k):
            return (G_def(x + h * nx, y, k) - G_def(x - h * nx, y, k)) / (2 * h)

        def dxy(k):
            return (dny(k, x + h * nx) - dny(k, x - h * nx)) / (2 * h)

        K = kernels(x, nx, y, ny, eps, KAPPA)
        ref = [G_def(x, y, 0.0) - G_def(x, y, KAPPA),
               eps * dny(KAPPA) - dny(0.0),
               dnx(0.0) - dnx(KAPPA) / eps,
               dxy(KAPPA) - dxy(0.0)]
        r = np.linalg.norm(x - y)
        tol = [1e-12, 1e-6 * eps / r ** 2, 1e-6 / r ** 2, 1e-4 / r ** 3]
        for k in range(4):
            assert abs(K[k] - ref[k]) <= tol[k], (k, K[k], ref[k])


def test_kernel_symmetries():
    """K1 and K4 are symmetric under swapping (x, nu_x) and (y, nu_y)."""
    rng = np.random.default_rng(13)
    for _ in range(10):
        x, y = rng.normal(size=3), rng.normal(size=3)
        nx, ny = _unit(rng.normal(size=3)), _unit(rng.normal(size=3))
        a = kernels(x, nx, y, ny, 80.0, KAPPA)
        b = kernels(y, ny, x, nx, 80.0, KAPPA)
        assert a[0] == pytest.approx(b[0], rel=1e-13)
        assert a[3] == pytest.approx(b[3], rel=1e-10, abs=1e-15)


def test_kirkwood_g_matches_scipy_bessel():
    """g_n = x k_n'(x)/k_n(x) against scipy's modified spherical Bessel k_n."""
    for x in (0.05, 0.2514, 1.0, 3.0):
        g = kirkwood._g(12, x)
        for n in range(13):
            ref = x * spherical_kn(n, x, derivative=True) / spherical_kn(n, x)
            assert g[n] == pytest.approx(ref, rel=1e-12)


def test_kirkwood_conductor_limit_is_image_charge():
    """eps_out -> infinity, kappa = 0: grounded conducting sphere, image
    charge -q a/b at a^2/b gives phi_reac(b) = -q a/(a^2 - b^2)."""
    a, q = 2.0, 1.0
    for b in (0.0, 0.5, 1.0, 1.5):
        e = kirkwood.energy(a, q, b, eps_in=1.0, eps_out=1e14, kappa=0.0, n_max=2000)
        ref = 0.5 * kirkwood.C_UNITS * q * (-q * a / (a * a - b * b))
        assert e == pytest.approx(ref, rel=1e-9)


def test_kirkwood_central_is_born():
    for k in (0.0, KAPPA):
        assert kirkwood.energy(2.0, 1.0, 0.0, kappa=k) == pytest.approx(
            kirkwood.born_energy(2.0, 1.0, kappa=k), rel=1e-15)
    assert kirkwood.born_energy(2.0, 1.0, kappa=0.0) == pytest.approx(-81.98017625, abs=1e-8)
    assert kirkwood.born_energy(2.0, 1.0) == pytest.approx(-82.18864976, abs=1e-8)


def test_kirkwood_denergy_matches_fd_of_series():
    h = 1e-5
    for b in (0.5, 1.0, 1.5):
        fd = (kirkwood.energy(2, 1, b + h) - kirkwood.energy(2, 1, b - h)) / (2 * h)
        assert kirkwood.denergy_db(2, 1, b) == pytest.approx(fd, rel=1e-7)


def _small_star(freq=4, r0=6.0, nc=5, seed=21):
    rng = np.random.default_rng(seed)
    coef = synth.mesh.draw_shape_coeffs(rng, 6)
    v, t = synth.star_surface(freq, r0, coef)

    def inside(p):
        rr = np.linalg.norm(p, axis=1)
        return rr < synth.star_radius(p / rr[:, None], r0, coef)

    pos, q = synth.interior_charges(rng, v, t, inside, nc, min_dist=1.0)
    return v, t, pos, q


def test_gmres_matches_dense_lu():
    v, t, pos, q = _small_star(freq=4)
    lu = dsbi.solve_dense(v, t, pos, q)
    it = dsbi.solve(v, t, pos, q, tol=1e-13)
    assert it.info.converged
    err = np.linalg.norm(it.xi - lu.xi) / np.linalg.norm(lu.xi)
    assert err <= 1e-10
    assert it.e_solv == pytest.approx(lu.e_solv, rel=1e-10)


def test_matvec_matches_dense_assembly_and_transpose():
    v, t, pos, q = _small_star(freq=3)
    g = dsbi.geometry(v, t)
    A = dsbi.dense_matrix(g, 80.0, KAPPA)
    rng = np.random.default_rng(3)
    x = rng.normal(size=2 * g.n)
    y = rng.normal(size=2 * g.n)
    Ax = dsbi.matvec(g, 80.0, KAPPA, x)
    ATy = dsbi.matvec(g, 80.0, KAPPA, y, transpose=True)
    assert np.allclose(Ax, A @ x, rtol=0, atol=1e-12 * np.abs(A).sum(1).max() * np.abs(x).max())
    assert np.allclose(ATy, A.T @ y, rtol=0, atol=1e-12 * np.abs(A).sum(0).max() * np.abs(y).max())
    assert np.dot(Ax, y) == pytest.approx(np.dot(x, ATy), rel=1e-12)


def test_eps1_kappa0_is_identity_and_zero_energy():
    v, t, pos, q = _small_star(freq=3)
    g = dsbi.geometry(v, t)
    A = dsbi.dense_matrix(g, 1.0, 0.0)
    assert np.array_equal(A, np.eye(2 * g.n))
    s = dsbi.solve(v, t, pos, q, eps_in=2.0, eps_out=2.0, kappa=0.0, tol=1e-14)
    assert s.e_solv == 0.0
    assert np.allclose(s.xi, s.b, rtol=1e-15, atol=0)


def test_kappa0_decouples_potential_block():
    """kappa = 0: K1 = K4 = 0, so the phi rows do not see psi and vice versa."""
    v, t, _pos, _q = _small_star(freq=3)
    g = dsbi.geometry(v, t)
    A = dsbi.dense_matrix(g, 80.0, 0.0)
    n = g.n
    assert np.all(A[:n, n:] == 0.0)
    assert np.all(A[n:, :n] == 0.0)


def test_double_layer_solid_angle_identity_on_star_surface():
    """kappa = 0, phi = 1, psi = 0: sum_j a_j dG0/dnu_y -> -1/2 for every
    point of a closed smooth surface, so (A [1; 0])_i -> eps.  Collocation
    error falls with refinement on a non-uniform mesh."""
    rng = np.random.default_rng(2)
    coef = synth.mesh.draw_shape_coeffs(rng, 6)
    errs = []
    for f in (8, 16):
        v, t = synth.star_surface(f, 20.0, coef)
        g = dsbi.geometry(v, t)
        n = g.n
        y = dsbi.matvec(g, 80.0, 0.0, np.concatenate([np.ones(n), np.zeros(n)]))
        errs.append(np.median(np.abs(y[:n] - 80.0)) / 80.0)
        assert np.all(y[n:] == 0.0)
    assert errs[1] < errs[0] < 0.05


def test_gauss_law_source_and_solution():
    """sum_i S2_i a_i -> -Q/eps_in (flux of the charges' field through the
    surface) and the same holds for the solved psi, as the interior has no
    ions.  One charge set, two refinements of the same star shape."""
    w = synth.star_protein(freq=16, r0=10.0, n_charges=20, seed=7)
    Q = float(np.sum(w.q))
    err_src, err_sol = [], []
    for f in (8, 16):
        v, t = synth.star_surface(f, 10.0, w.meta["coef"])
        s = dsbi.solve(v, t, w.pos, w.q, tol=1e-8)
        n = s.geom.n
        a = s.geom.area
        err_src.append(abs(float(np.sum(s.b[n:] * a)) + Q / EPS_IN))
        err_sol.append(abs(float(np.sum(s.xi[n:] * a)) + Q / EPS_IN))
    assert err_src[1] < err_src[0] and err_src[1] < 5e-3 * abs(Q)
    assert err_sol[1] < err_sol[0] and err_sol[1] < 2e-2 * abs(Q)


def test_kirkwood_sphere_convergence_central():
    ref = kirkwood.born_energy(2.0, 1.0)
    errs = []
    for f in (4, 8, 16):
        w = synth.kirkwood_sphere(freq=f)
        s = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-10)
        errs.append(abs(s.e_solv - ref) / abs(ref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2


def test_kirkwood_sphere_off_centre():
    ref = kirkwood.energy(2.0, 1.0, 1.0)
    errs = []
    for f in (8, 16):
        w = synth.kirkwood_sphere(freq=f, offset=(0.0, 0.0, 1.0))
        s = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-8)
        errs.append(abs(s.e_solv - ref) / abs(ref))
    assert errs[1] < errs[0] < 0.05


def _icosa_rotations():
    iv, faces = synth.mesh._icosahedron()
    iv = iv / np.linalg.norm(iv, axis=1)[:, None]

    def rot(axis, ang):
        k = _unit(axis)
        K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K

    fa = faces[0]
    gens = [rot(iv[0], 2 * math.pi / 5), rot(iv[list(fa)].sum(0), 2 * math.pi / 3)]
    group = [np.eye(3)]
    frontier = [np.eye(3)]
    while frontier:
        new = []
        for g in frontier:
            for h in gens:
                m = h @ g
                if not any(np.allclose(m, x, atol=1e-9) for x in group):
                    group.append(m)
                    new.append(m)
        frontier = new
    return group


def test_icosahedral_symmetry_of_central_solution():
    """Central charge: phi and psi are invariant under the 60 rotations of
    the icosahedron, which map the geodesic mesh onto itself."""
    from scipy.spatial import cKDTree
    group = _icosa_rotations()
    assert len(group) == 60
    w = synth.kirkwood_sphere(freq=8)
    s = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-13)
    n = s.geom.n
    tree = cKDTree(s.geom.cen)
    for R in group:
        d, perm = tree.query(s.geom.cen @ R.T)
        assert d.max() < 1e-9
        assert np.allclose(s.xi[:n][perm], s.xi[:n], rtol=1e-10, atol=0)
        assert np.allclose(s.xi[n:][perm], s.xi[n:], rtol=1e-10, atol=0)


def test_rigid_motion_scaling_and_charge_invariants():
    v, t, pos, q = _small_star(freq=6, r0=8.0, nc=6, seed=5)
    base = dsbi.solve(v, t, pos, q, tol=1e-13).e_solv
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    sh = np.array([3.0, -7.0, 11.0])
    moved = dsbi.solve(v @ Q.T + sh, t, pos @ Q.T + sh, q, tol=1e-13).e_solv
    assert moved == pytest.approx(base, rel=1e-10)
    s = 2.0
    scaled = dsbi.solve(v * s, t, pos * s, q, kappa=KAPPA / s, tol=1e-13).e_solv
    assert scaled == pytest.approx(base / s, rel=1e-10)
    lam = -1.7
    q2 = dsbi.solve(v, t, pos, q * lam, tol=1e-13).e_solv
    assert q2 == pytest.approx(base * lam * lam, rel=1e-10)


def test_adjoint_forces_match_finite_differences_of_dense_solve():
    v, t, pos, q = _small_star(freq=3, r0=6.0, nc=4, seed=31)
    sol = dsbi.solve_dense(v, t, pos, q)
    dpos, dq, _lam, _ = dsbi.forces(sol, pos, q, tol=1e-14)
    h = 1e-4
    for k in range(pos.shape[0]):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[k, c] += h
            pm[k, c] -= h
            fd = (dsbi.solve_dense(v, t, pp, q).e_solv - dsbi.solve_dense(v, t, pm, q).e_solv) / (2 * h)
            assert dpos[k, c] == pytest.approx(fd, rel=1e-6, abs=1e-7 * np.abs(dpos).max())
        qp, qm = q.copy(), q.copy()
        qp[k] += h
        qm[k] -= h
        fdq = (dsbi.solve_dense(v, t, pos, qp).e_solv - dsbi.solve_dense(v, t, pos, qm).e_solv) / (2 * h)
        assert dq[k] == pytest.approx(fdq, rel=1e-6, abs=1e-7 * np.abs(dq).max())


def test_adjoint_force_on_off_centre_kirkwood_charge():
    """The radial force on an off-centre charge approaches dE/db of the
    closed form as the sphere is refined."""
    b = 1.0
    ref = kirkwood.denergy_db(2.0, 1.0, b)
    errs = []
    for f in (8, 16):
        w = synth.kirkwood_sphere(freq=f, offset=(0.0, 0.0, b))
        s = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-9)
        dpos, _dq, _l, _ = dsbi.forces(s, w.pos, w.q, tol=1e-9)
        errs.append(abs(dpos[0, 2] - ref) / abs(ref))
    assert errs[1] < errs[0] < 0.1


def test_interior_reaction_potential_is_kirkwood_constant_for_central_charge():
    """Central charge: the reaction potential inside the sphere is the
    constant (q/a)(1/(eps_out(1+kappa a)) - 1/eps_in) (Gaussian units), i.e.
    that divided by 4 pi in BIE units; the discrete value converges to it."""
    a, qv = 2.0, 1.0
    exact = qv / a * (1.0 / (80.0 * (1.0 + KAPPA * a)) - 1.0) / (4.0 * math.pi)
    pts = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.1], [0.0, 0.7, -0.4]])
    errs = []
    for f in (8, 16):
        w = synth.kirkwood_sphere(freq=f)
        s = dsbi.solve(w.verts, w.tris, w.pos, w.q, tol=1e-10)
        reac, total = dsbi.potential(s.geom, 80.0, KAPPA, s.xi, w.pos, w.q, 1.0, pts)
        errs.append(np.abs(reac - exact).max() / abs(exact))
        r = np.linalg.norm(pts[1:], axis=1)
        assert np.allclose(total[1:] - reac[1:], qv / (4 * math.pi * r), rtol=1e-14)
    assert errs[1] < errs[0] < 0.05


def test_coulomb_energy_of_two_charges():
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 3.0, 4.0]])
    q = np.array([1.5, -0.5])
    e = dsbi.coulomb_energy(pos, q, eps_in=2.0)
    assert e == pytest.approx(332.0716 * 1.5 * -0.5 / (2.0 * 5.0), rel=1e-14)
