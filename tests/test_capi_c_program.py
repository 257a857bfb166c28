"""The C ABI from plain C: tests/c/pb_solve_demo.c is compiled by gcc against
include/pbsolve.h alone and linked to the built library.  On the CPU it must
compile and link cleanly; on a GPU its solves, energy and derivatives must
equal the Python binding's (same library, same inputs) and the FP64 energy
the oracle's."""
import os
import struct
import subprocess

import numpy as np
import pytest

import synth
from oracle import dsbi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2312_10044_amd")
SRC = os.path.join(ROOT, "tests", "c", "pb_solve_demo.c")


def _build(out_dir):
    exe = os.path.join(str(out_dir), "pb_solve_demo")
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-Werror", "-pedantic",
           "-I", os.path.join(ROOT, "include"), SRC, "-L", PKG, "-lpbdsbi",
           f"-Wl,-rpath,{PKG}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return exe


def _write_input(path, w):
    with open(path, "wb") as f:
        f.write(struct.pack("<3q", w.verts.shape[0], w.tris.shape[0], w.q.shape[0]))
        f.write(struct.pack("<3d", w.eps_in, w.eps_out, w.kappa))
        f.write(np.ascontiguousarray(w.verts, dtype="<f8").tobytes())
        f.write(np.ascontiguousarray(w.tris, dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(w.pos, dtype="<f8").tobytes())
        f.write(np.ascontiguousarray(w.q, dtype="<f8").tobytes())


def _parse(text):
    vals, dq, dpos = {}, {}, {}
    for line in text.splitlines():
        key, _, rest = line.partition(" ")
        if key == "de_dq":
            k, v = rest.split()
            dq[int(k)] = float(v)
        elif key == "de_dpos":
            k, *v = rest.split()
            dpos[int(k)] = [float(t) for t in v]
        else:
            vals[key] = rest
    return vals, dq, dpos


def test_c_program_compiles_against_the_header(tmp_path):
    assert os.path.exists(os.path.join(PKG, "libpbdsbi.so")), "build the library first"
    _build(tmp_path)


@pytest.mark.gpu
def test_c_program_matches_the_binding_and_the_oracle(tmp_path):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_10044_amd as m

    w = synth.star_protein(freq=8, r0=8.0, n_charges=6, seed=17)
    exe = _build(tmp_path)
    inp = os.path.join(str(tmp_path), "in.bin")
    _write_input(inp, w)
    print(f"C program on {w.n_tri} triangles, {w.n_charges} charges", flush=True)
    r = subprocess.run([exe, inp], capture_output=True, text=True, timeout=120)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    vals, dq, dpos = _parse(r.stdout)
    from paper_2312_10044_amd import pbsolve
    assert int(vals["abi"]) == pbsolve.load_library().pb_abi_version()

    ctx = m.Context(0)
    try:
        info64, _phi, _dphi = ctx.pb_solve(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-10))
        info_f, g_pos, g_q = ctx.pb_forces(w.verts, w.tris, w.pos, w.q, m.Params(tol=1e-10))
    finally:
        ctx.close()
    e64 = float(vals["e_fp64"])
    assert e64 == info64.e_solv                      # same library, same inputs, deterministic
    assert abs(float(vals["e_energy"]) - e64) <= 1e-12 * abs(e64)
    assert abs(float(vals["e_fp32ir"]) - e64) <= 1e-6 * abs(e64)
    assert int(vals["matvecs_fp32"]) > 0
    assert float(vals["e_forces"]) == info_f.e_solv
    assert np.array_equal(np.array([dq[k] for k in range(w.n_charges)]), g_q)
    assert np.array_equal(np.array([dpos[k] for k in range(w.n_charges)]), g_pos)
    assert int(vals["bad_tol_status"]) == m.PB_ERR_ARG
    assert vals["bad_tol_message"].strip()

    ref = dsbi.solve(w.verts, w.tris, w.pos, w.q, w.eps_in, w.eps_out, w.kappa, tol=1e-12)
    assert abs(e64 - ref.e_solv) <= 1e-9 * abs(ref.e_solv)
