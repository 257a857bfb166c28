"""Child process of the host-sanitizer tests: runs the library's entry points
from a build whose host code is compiled with sanitizers (the library that
PB_SANITIZED_LIBRARY names: libpbdsbi_hostsan.so, AddressSanitizer and
UndefinedBehaviorSanitizer with the ASan runtime preloaded by the parent, or
libpbdsbi_hostubsan.so, UndefinedBehaviorSanitizer alone).  Any sanitizer
report aborts this process; the parent checks the exit status and the
printed results.

usage: python hostsan_driver.py cpu        (no GPU: argument and error paths)
       python hostsan_driver.py gpu JSON   (every entry point on small inputs;
                                            JSON holds the oracle's energies)
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import numpy as np  # noqa: E402

from paper_2312_10044_amd import build, pbsolve  # noqa: E402


def say(*a):
    print(*a, flush=True)


def cpu_paths(L):
    import ctypes
    assert L.pb_abi_version() == 1
    h = ctypes.c_void_p()
    st = L.pb_create(0, None, ctypes.byref(h))
    say("pb_create without a GPU:", st)
    assert st < 0
    ints = (ctypes.c_int, ctypes.c_int32, ctypes.c_int64)
    for name in ("pb_solve", "pb_forces", "pb_matvec", "pb_source", "pb_energy"):
        f = getattr(L, name)
        st = f(*[0 if t in ints else None for t in f.argtypes])
        say(name, "with NULL arguments:", st)
        assert st == pbsolve.PB_ERR_ARG
    say("cpu ok")


def gpu_paths(L, expect):
    import synth
    m = pbsolve
    w = synth.kirkwood_sphere(freq=8)
    star = synth.star_protein(freq=10, r0=8.0, n_charges=60, seed=43)
    with m.Context(0) as ctx:
        info, phi, dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-12))
        say("kirkwood FP64", info.e_solv, info.status)
        assert info.status == m.PB_OK
        assert abs(info.e_solv - expect["kirkwood"]) <= 1e-10 * abs(expect["kirkwood"])
        info, _p, _d = ctx.pb_solve(star.verts, star.tris, star.pos, star.q,
                                    m.Params(tol=1e-9, precision=m.PB_FP32_IR, precond_leaf=16))
        say("star FP32-IR leaf 16", info.e_solv, info.status)
        assert abs(info.e_solv - expect["star"]) <= 1e-6 * abs(expect["star"])
        info, _p, _d = ctx.pb_solve(star.verts, star.tris, star.pos, star.q,
                                    m.Params(tol=1e-12, precond_leaf=100))
        say("star FP64 leaf 100", info.e_solv)
        assert abs(info.e_solv - expect["star"]) <= 1e-10 * abs(expect["star"])
        finfo, dpos, dq = ctx.pb_forces(star.verts, star.tris, star.pos, star.q,
                                        m.Params(tol=1e-10))
        say("forces", finfo.status, float(np.abs(dpos).max()))
        assert finfo.status == m.PB_OK and np.all(np.isfinite(dpos)) and np.all(np.isfinite(dq))
        e, infos, gpos, gq = ctx.pb_solve_batch(
            [(w.verts, w.tris, w.pos, w.q), (star.verts, star.tris, star.pos, star.q)],
            m.Params(tol=1e-12), forces=True)
        say("batch", list(e))
        assert abs(e[0] - expect["kirkwood"]) <= 1e-10 * abs(expect["kirkwood"])
        assert abs(e[1] - expect["star"]) <= 1e-10 * abs(expect["star"])
        for kind in (m.PB_SWEEP_PAIRWISE, m.PB_SWEEP_BANDED, 1):
            ctx.set_sweep_config(kind, 0)
            y = ctx.pb_matvec(star.verts, star.tris, np.ones(2 * star.n_tri), m.Params(),
                              precision=m.PB_FP32_IR)
            assert np.all(np.isfinite(y))
        ctx.set_sweep_config(m.PB_SWEEP_PAIRWISE, 0)
        yt = ctx.pb_matvec_tree(star.verts, star.tris, np.ones(2 * star.n_tri), m.Params())
        assert np.all(np.isfinite(yt))
        leaves = ctx.pb_precond_leaves(star.verts, star.tris, 100)
        assert sum(len(a) for a in leaves) == star.n_tri
        pts = np.array([[0.5, 0.0, 0.0], [0.0, 0.3, -0.2]])   # inside, off the charge
        reac, tot = ctx.pb_potential(w.verts, w.tris, w.pos, w.q, phi, dphi, pts, m.Params())
        say("potential", list(reac), list(tot))
        assert np.all(np.isfinite(reac)) and np.all(np.isfinite(tot))
        # error paths: the context stays usable after each
        bad = w.verts.copy()
        bad[3, 1] = np.nan
        for verts, tris, kw, status in (
                (bad, w.tris, {}, m.PB_ERR_GEOMETRY),
                (w.verts, np.vstack([w.tris, w.tris[17][None, :]]).astype(np.int32), {},
                 m.PB_ERR_GEOMETRY),
                (w.verts, w.tris, {"kappa": 101.0}, m.PB_ERR_ARG)):
            try:
                ctx.pb_solve(verts, tris, w.pos, w.q, m.Params(**kw))
                raise AssertionError("expected an error")
            except m.PbError as e:
                say("rejected:", e.status, e.message)
                assert e.status == status
        with m.Context(0) as fresh:   # a cap below what a first solve allocates
            fresh.set_memory_limit(64 * 1024)
            try:
                fresh.pb_solve(star.verts, star.tris, star.pos, star.q, m.Params())
                raise AssertionError("expected PB_ERR_OOM")
            except m.PbError as e:
                say("memory cap:", e.status)
                assert e.status == m.PB_ERR_OOM
            fresh.set_memory_limit(0)
            info, _p, _d = fresh.pb_solve(star.verts, star.tris, star.pos, star.q,
                                          m.Params(tol=1e-12))
            assert abs(info.e_solv - expect["star"]) <= 1e-10 * abs(expect["star"])
        info, _p, _d = ctx.pb_solve(w.verts, w.tris, w.pos, w.q,
                                    m.Params(tol=1e-6, max_iter=1))
        say("max_iter 1:", info.status)
        assert info.status == m.PB_NOT_CONVERGED
    say("gpu ok")


def main():
    L = pbsolve.load_library(os.environ.get("PB_SANITIZED_LIBRARY", build.SAN_LIB))
    if sys.argv[1] == "cpu":
        cpu_paths(L)
    else:
        gpu_paths(L, json.loads(sys.argv[2]))


if __name__ == "__main__":
    main()
