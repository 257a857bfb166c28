"""The five synthetic workloads (surface + charges + dielectric parameters).

* Kirkwood sphere: frequency-8 icosphere of radius 2 A (1,280 triangles),
  one +1 charge at the centre.
* Star protein: frequency-64 star surface (81,920 triangles), R0 = 20 A,
  2,000 interior charges, seed 2.
* Large star protein: frequency-128 (327,680 triangles), R0 = 40 A,
  10,000 charges, seed 3.
* Batch: 64 star surfaces, per-system seeds spawned from seed 5, frequency
  U{16..64}, R0 ~ U(10, 25) A, N_c ~ U{100..2000}.

Dielectric constants and screening follow the paper's runs: eps_in = 1,
eps_out = 80, ionic strength 0.15 M, i.e. kappa = 0.1257 1/A.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

from .mesh import icosphere, star_surface, star_radius, draw_shape_coeffs
from .charges import interior_charges

EPS_IN = 1.0
EPS_OUT = 80.0
KAPPA = 0.1257


@dataclass
class Workload:
    name: str
    verts: np.ndarray            # [Nv, 3] float64
    tris: np.ndarray             # [N, 3] int32, counter-clockwise from outside
    pos: np.ndarray              # [Nc, 3] float64
    q: np.ndarray                # [Nc] float64
    eps_in: float = EPS_IN
    eps_out: float = EPS_OUT
    kappa: float = KAPPA
    meta: dict = field(default_factory=dict)

    @property
    def n_tri(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_charges(self) -> int:
        return int(self.q.shape[0])


def _star_shape(freq, r0, rng, amp=0.15):
    """The star surface of a workload: its shape is drawn first from rng."""
    coef = draw_shape_coeffs(rng, 6)
    verts, tris = star_surface(freq, r0, coef, amp)
    return verts, tris, coef


def _star(name, freq, r0, n_charges, rng, amp=0.15, min_dist=1.5):
    verts, tris, coef = _star_shape(freq, r0, rng, amp)

    def inside(p):
        rr = np.sqrt(np.sum(p * p, axis=1))
        u = p / np.maximum(rr, 1e-300)[:, None]
        return rr < star_radius(u, r0, coef, amp)

    pos, q = interior_charges(rng, verts, tris, inside, n_charges, min_dist=min_dist)
    return Workload(name, verts, tris, pos, q,
                    meta={"freq": freq, "r0": r0, "amp": amp, "coef": coef})


def kirkwood_sphere(freq: int = 8, radius: float = 2.0, charge: float = 1.0,
                    offset=(0.0, 0.0, 0.0), kappa: float = KAPPA) -> Workload:
    verts, tris = icosphere(freq, radius)
    pos = np.asarray([offset], dtype=np.float64)
    q = np.asarray([charge], dtype=np.float64)
    return Workload(f"kirkwood_f{freq}", verts, tris, pos, q, kappa=kappa,
                    meta={"freq": freq, "radius": radius})


def star_protein(freq: int = 64, r0: float = 20.0, n_charges: int = 2000,
                 seed: int = 2) -> Workload:
    rng = np.random.default_rng(seed)
    return _star(f"star_f{freq}_s{seed}", freq, r0, n_charges, rng)


def large_star_protein(seed: int = 3) -> Workload:
    rng = np.random.default_rng(seed)
    return _star(f"star_f128_s{seed}", 128, 40.0, 10000, rng)


def large_star_surface(seed: int = 3):
    """(verts, tris) of large_star_protein(seed) without its 10,000 charges,
    which are drawn after the shape: the input of a matvec at that size."""
    verts, tris, _coef = _star_shape(128, 40.0, np.random.default_rng(seed))
    return verts, tris


def batch_conformations(n_sys: int = 64, seed: int = 5, freq_range=(16, 64),
                        r0_range=(10.0, 25.0), nc_range=(100, 2000)) -> list:
    out = []
    for k, child in enumerate(np.random.SeedSequence(seed).spawn(n_sys)):
        rng = np.random.default_rng(child)
        freq = int(rng.integers(freq_range[0], freq_range[1] + 1))
        r0 = float(rng.uniform(r0_range[0], r0_range[1]))
        nc = int(rng.integers(nc_range[0], nc_range[1] + 1))
        out.append(_star(f"batch{seed}_{k}", freq, r0, nc, rng))
    return out


def input_digest(w: Workload) -> str:
    """SHA-256 over the raw bytes of the arrays that define a workload."""
    h = hashlib.sha256()
    for a in (w.verts, w.tris, w.pos, w.q):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(np.asarray([w.eps_in, w.eps_out, w.kappa]).tobytes())
    return h.hexdigest()
