"""The seeded input generators: a workload's surface comes first from its
generator, so the surface-only helper gives the workload's exact surface."""
import numpy as np

import synth
from synth import workloads


def test_star_shape_is_drawn_before_the_charges():
    w = synth.star_protein(freq=12, r0=10.0, n_charges=300, seed=41)
    v, t, _coef = workloads._star_shape(12, 10.0, np.random.default_rng(41))
    assert np.array_equal(v, w.verts) and np.array_equal(t, w.tris)


def test_large_star_surface_shape_and_repeatability():
    v, t = synth.large_star_surface()
    assert t.shape == (327680, 3) and v.shape == (163842, 3)
    r = np.sqrt((v * v).sum(axis=1))
    # a star deformation of the radius-40 sphere (radial std about 7 %)
    assert 25.0 < r.min() and r.max() < 55.0
    v2, t2 = synth.large_star_surface()
    assert np.array_equal(v, v2) and np.array_equal(t, t2)
