"""FP64 CPU oracle of the DSBI Poisson-Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check
(``__graft_entry__.smoke``) and the benchmark's CPU-baseline leg may import,
call, link or execute anything in this package.  The HIP library and its
Python binding never do, and this package imports nothing from them: the two
share no kernels, headers, helpers or constants.  Only the seeded input
generators in ``synth`` serve both.

Contents: ``dsbi`` (geometry, source terms, K1..K4 matvec and its transpose,
restarted GMRES, solvation energy, adjoint forces, dense assembly) backed by
the plain C loops of ``dsbi_oracle.c``; ``kirkwood`` (closed-form sphere).
"""
from . import dsbi, kirkwood
from ._clib import build, lib

__all__ = ["dsbi", "kirkwood", "build", "lib"]
