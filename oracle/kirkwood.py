"""Kirkwood closed form for a point charge in a dielectric sphere.

Textbook solution (Kirkwood 1934; the sphere test the Juffer formulation
cited in Sec. 2.2.1 is usually checked on): a sphere of radius ``a`` with
permittivity eps_in and no ions, surrounded by a medium of permittivity
eps_out and inverse Debye length kappa that reaches the sphere surface, with a
charge q at distance b from the centre.  In Gaussian-type units
(phi = q/(eps r)) the reaction potential inside is
sum_n B_n r^n P_n(cos gamma) with

    B_n = q b^n / a^(2n+1) * ((n+1) + eps_out g_n / eps_in)
                           / (eps_in n - eps_out g_n),

g_n = x k_n'(x) / k_n(x) at x = kappa a (k_n the modified spherical Bessel
function of the second kind); g_n = -(n+1) when kappa = 0.  With
t_n = k_{n-1}(x)/k_n(x): t_0 = 1, 1/t_n = t_{n-1} + (2n-1)/x and
g_n = -x t_n - (n+1).

E_sol = (c_u / 2) q phi_reac(b) in kcal/mol (c_u = 332.0716).

TEST INFRASTRUCTURE ONLY (part of the oracle).
"""
from __future__ import annotations

C_UNITS = 332.0716


def _g(n_max: int, x: float):
    """g_0..g_n_max for the exterior solution k_n(kappa r)."""
    if x == 0.0:
        return [-(n + 1.0) for n in range(n_max + 1)]
    out = []
    t = 1.0
    for n in range(n_max + 1):
        if n > 0:
            t = 1.0 / (t + (2 * n - 1) / x)
        out.append(-x * t - (n + 1.0))
    return out


def coefficients(a: float, eps_in: float, eps_out: float, kappa: float, n_max: int):
    """c_n with B_n = q b^n c_n / a^(2n+1)."""
    g = _g(n_max, kappa * a)
    return [((n + 1.0) + eps_out * g[n] / eps_in) / (eps_in * n - eps_out * g[n])
            for n in range(n_max + 1)]


def energy(a: float, q: float, b: float, eps_in: float = 1.0, eps_out: float = 80.0,
           kappa: float = 0.1257, n_max: int = 400) -> float:
    """Solvation energy (kcal/mol) of charge q at distance b < a from the centre."""
    c = coefficients(a, eps_in, eps_out, kappa, n_max)
    s = 0.0
    rho = (b / a) ** 2
    p = 1.0
    for n in range(n_max + 1):
        s += c[n] * p
        p *= rho
    return 0.5 * C_UNITS * q * q * s / a


def denergy_db(a: float, q: float, b: float, eps_in: float = 1.0, eps_out: float = 80.0,
               kappa: float = 0.1257, n_max: int = 400) -> float:
    """dE/db (kcal/mol/A), b measured outward from the centre."""
    c = coefficients(a, eps_in, eps_out, kappa, n_max)
    s = 0.0
    for n in range(1, n_max + 1):
        s += c[n] * 2.0 * n * b ** (2 * n - 1) / a ** (2 * n)
    return 0.5 * C_UNITS * q * q * s / a


def born_energy(a: float, q: float, eps_in: float = 1.0, eps_out: float = 80.0,
                kappa: float = 0.1257) -> float:
    """Central charge: (c_u/2) (q^2/a) [1/(eps_out (1 + kappa a)) - 1/eps_in]."""
    return 0.5 * C_UNITS * q * q / a * (1.0 / (eps_out * (1.0 + kappa * a)) - 1.0 / eps_in)
