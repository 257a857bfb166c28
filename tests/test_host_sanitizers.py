"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

* The oracle's C loops (oracle/dsbi_oracle.c), every entry point, on a
  320-triangle icosphere: no sanitizer report, and the matvec loops agree
  with the oracle's own dense matrix.
* The library's host-side octree (paper_2312_10044_amd/csrc/pb_host.cpp, the
  preconditioner's leaves): no sanitizer report, threaded and single-threaded
  builds identical, and the leaves identical to the oracle's (index work:
  bit-exact), including a cloud with coincident points that reaches the
  depth limit.

* The library's own host code (the C ABI, planning, context and buffer
  handling in the .hip sources), built with ASan and UBSan on the host side
  only (libpbdsbi_hostsan.so), and with UBSan alone (libpbdsbi_hostubsan.so):
  their argument and error paths without a GPU.  ROCm's ASan runtime
  intercepts HSA memory-pool allocations for device ASan, which this GPU
  pool does not run, so tests/test_gpu_host_sanitizers.py runs every entry
  point on the GPU with the UBSan build.

Any sanitizer report aborts the program (-fno-sanitize-recover=all).
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import synth
from oracle import dsbi, precond

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc/g++")


def _build(tmp_path, compiler, srcs, name, extra=()):
    exe = os.path.join(str(tmp_path), name)
    cmd = [compiler, *SAN, *extra, *srcs, "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return exe


def test_oracle_loops_under_sanitizers(tmp_path):
    exe = _build(tmp_path, "gcc", [os.path.join(ROOT, "tests", "c", "oracle_sanitize.c"),
                                   os.path.join(ROOT, "oracle", "dsbi_oracle.c")],
                 "oracle_sanitize", ["-std=c99", "-Wno-unknown-pragmas"])
    w = synth.star_protein(freq=4, r0=6.0, n_charges=7, seed=3)
    g = dsbi.geometry(w.verts, w.tris)
    path = os.path.join(str(tmp_path), "in.bin")
    with open(path, "wb") as f:
        f.write(struct.pack("<2q", g.n, w.n_charges))
        for a in (g.cen, g.nrm, g.area, w.pos, w.q):
            f.write(np.ascontiguousarray(a, dtype="<f8").tobytes())
    r = subprocess.run([exe, path], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    vals = dict(line.split() for line in r.stdout.splitlines())
    print(vals)
    assert float(vals["matvec_vs_dense"]) <= 1e-13
    assert float(vals["rows_subset"]) == 0.0
    assert float(vals["subset_block"]) == 0.0
    assert vals["finite"] == "1"


def _leaves_run(exe, tmp_path, pts, n0):
    inp = os.path.join(str(tmp_path), "pts.bin")
    out = os.path.join(str(tmp_path), "leaves.bin")
    with open(inp, "wb") as f:
        f.write(struct.pack("<2q", pts.shape[0], n0))
        f.write(np.ascontiguousarray(pts.T, dtype="<f8").tobytes())
    r = subprocess.run([exe, inp, out], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    data = np.fromfile(out, dtype="<i8")
    n = pts.shape[0]
    res, k = [], 0
    for _ in range(2):
        L = int(data[k])
        start = data[k + 1:k + 2 + L]
        perm = data[k + 2 + L:k + 2 + L + n]
        k += 2 + L + n
        res.append([perm[start[i]:start[i + 1]] for i in range(L)])
    return res


@pytest.mark.parametrize("n0", [1, 7, 24, 100])
def test_host_octree_under_sanitizers_matches_the_oracle(tmp_path, n0):
    exe = _build(tmp_path, "g++", [os.path.join(ROOT, "tests", "c", "host_leaves_check.cpp"),
                                   os.path.join(ROOT, "paper_2312_10044_amd", "csrc",
                                                "pb_host.cpp")],
                 "host_leaves_check",
                 ["-std=c++17", "-pthread", "-I",
                  os.path.join(ROOT, "paper_2312_10044_amd", "csrc")])
    w = synth.star_protein(freq=40, r0=12.0, n_charges=1, seed=9)   # 32,000 points: threaded
    cen = dsbi.geometry(w.verts, w.tris).cen
    rng = np.random.default_rng(n0)
    cloud = rng.normal(size=(3000, 3))
    cloud[100:160] = cloud[7]          # 61 coincident points: the depth limit cuts them
    for pts in (cen, cloud):
        threaded, single = _leaves_run(exe, tmp_path, pts, n0)
        ref = precond.leaves(pts, n0)
        assert len(threaded) == len(single) == len(ref)
        for a, b, c in zip(threaded, single, ref):
            assert np.array_equal(a, c) and np.array_equal(b, c)


def _plans(tmp_path, kind, cases):
    exe = os.path.join(str(tmp_path), "host_plan_check")
    if not os.path.exists(exe):
        _build(tmp_path, "g++", [os.path.join(ROOT, "tests", "c", "host_plan_check.cpp"),
                                 os.path.join(ROOT, "paper_2312_10044_amd", "csrc", "pb_host.cpp")],
               "host_plan_check",
               ["-std=c++17", "-pthread", "-I", os.path.join(ROOT, "paper_2312_10044_amd", "csrc")])
    args = [str(v) for c in cases for v in (kind, *c)]
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0, r.stderr
    blocks = r.stdout.split("case ")[1:]
    assert len(blocks) == len(cases)
    return blocks


def test_pairwise_sweep_plan_under_sanitizers(tmp_path):
    """Every tile pair (I <= J) belongs to exactly one item; row_start lists
    each target tile's items in ascending J0 with consecutive slots; no item
    crosses a strip of T/16 source tiles (from 512 tiles on; one strip
    below); launch position b holds an item of XCD b mod 8 (strips k and
    15 - k) in every round where all XCDs still have items, the items of an
    XCD come longest first, and the XCDs get equal shares of the tile pairs
    (within 10 %)."""
    cases = [(256, 1), (512, 64), (2560, 8), (3072, 100000), (130816, 2048), (131072, 2048),
             (81920, 16384), (81920, 1024), (327680, 32768), (327680, 4096)]
    blocks = _plans(tmp_path, "sym", cases)
    for blk in blocks:
        lines = blk.splitlines()
        npad, target, n_items, L, ns = (int(v) for v in lines[0].split()[1:])
        T = npad // 256
        assert ns == (16 if T >= 512 else 1)
        items = [tuple(int(v) for v in ln.split()[1:]) for ln in lines if ln.startswith("item")]
        rs = [int(v) for v in next(ln for ln in lines if ln.startswith("rowstart")).split()[1:]]
        assert len(items) == n_items and len(rs) == T + 1 and rs[0] == 0 and rs[T] == n_items
        edge = [k * T // ns for k in range(ns + 1)]
        strip = np.searchsorted(edge, np.arange(T), side="right") - 1
        xcd_of_strip = [k if k < 8 else 15 - k for k in range(16)] if ns == 16 else [0]
        cover = np.zeros((T, T), dtype=np.int32)
        by_slot = {}
        work = np.zeros(8)
        per_xcd = {x: [] for x in range(8)}
        for b, (I, j0, j1, slot) in enumerate(items):
            assert I <= j0 < j1 <= T and j1 - j0 <= L
            assert strip[j0] == strip[j1 - 1]
            cover[I, j0:j1] += 1
            assert slot not in by_slot
            by_slot[slot] = (I, j0)
            x = xcd_of_strip[strip[j0]]
            per_xcd[x].append((b, j1 - j0))
            work[x] += j1 - j0
        assert np.all(cover[np.triu_indices(T)] == 1) and np.all(cover[np.tril_indices(T, -1)] == 0)
        for I in range(T):
            got = [by_slot[s] for s in range(rs[I], rs[I + 1])]
            assert all(g[0] == I for g in got)
            assert [g[1] for g in got] == sorted(g[1] for g in got)
        for x, v in per_xcd.items():
            assert [n for _, n in v] == sorted((n for _, n in v), reverse=True)
        if ns == 16:
            rounds = min(len(v) for v in per_xcd.values())
            for x, v in per_xcd.items():
                assert all(b % 8 == x for b, _n in v[:rounds])
            assert work.max() <= 1.1 * work.min()
        else:
            assert [b for b, _n in per_xcd[0]] == list(range(n_items))
        print(f"T={T} target={target}: {n_items} items, L={L}, XCD work {work.min():.0f}-{work.max():.0f}")


def test_banded_sweep_plan_under_sanitizers(tmp_path):
    """Every unordered tile pair (I <= J) belongs to exactly one item; each
    tile's record list holds exactly the row records of the items that sweep
    it as a target (run reaching it) and the column records of the items whose
    run holds it and whose band starts below it; record slots are distinct and
    within n_records; run and band stay within their bounds."""
    cases = [(256, 2048), (512, 1), (2560, 2048), (3072, 4), (3072, 100000), (81920, 2048),
             (81920, 128), (327680, 2048), (327680, 64)]
    blocks = _plans(tmp_path, "band", cases)
    MT, RUN_MAX = 4, 24
    for blk in blocks:
        lines = blk.splitlines()
        npad, target, n_items, run, band, n_rec = (int(v) for v in lines[0].split()[1:])
        T = npad // 256
        assert 1 <= run <= RUN_MAX and band >= 1
        items = [tuple(int(v) for v in ln.split()[1:]) for ln in lines if ln.startswith("item")]
        lists = {int(ln.split()[1]): [int(v) for v in ln.split()[2:]]
                 for ln in lines if ln.startswith("list")}
        assert len(items) == n_items and len(lists) == T
        cover = np.zeros((T, T), dtype=np.int32)
        rows = {K: [] for K in range(T)}
        cols = {K: [] for K in range(T)}
        slots = []
        for m0, m1, j0, j1, rslot, cslot in items:
            i0, i1 = m0 * MT, min(T, m1 * MT)
            assert 0 < j1 - j0 <= run and i0 <= j0 and m1 - m0 <= band
            for I in range(i0, i1):
                for J in range(max(j0, I), j1):
                    cover[I, J] += 1
                if j1 > I:
                    rows[I].append(rslot + I - i0)
            for J in range(j0, j1):
                if J > i0:
                    cols[J].append(cslot + J - j0)
            slots += list(range(rslot, rslot + (i1 - i0))) + list(range(cslot, cslot + j1 - j0))
        assert len(set(slots)) == len(slots) and max(slots) < n_rec
        assert np.all(cover[np.triu_indices(T)] == 1) and np.all(cover[np.tril_indices(T, -1)] == 0)
        for K in range(T):
            assert sorted(lists[K]) == sorted(rows[K] + cols[K])
            assert len(set(lists[K])) == len(lists[K])
        # far fewer records than one per tile pair (the pairwise sweep's count)
        if target == 2048 and T >= 320:
            assert n_rec < T * (T + 1) // 2 * (0.5 if T < 1000 else 0.15)


def sanitized_library_env(kind: str = "asan"):
    """Environment for a child process that loads a host-sanitized library:
    kind "asan" (libpbdsbi_hostsan.so) with the ASan runtime preloaded ahead of
    whatever the environment preloads; kind "ubsan" (libpbdsbi_hostubsan.so)
    with the directory of the minimal UBSan runtime on the library path.
    PB_SANITIZED_LIBRARY names the library for the child."""
    from paper_2312_10044_amd import build
    rt = build.sanitizer_runtime("asan" if kind == "asan" else "ubsan_minimal")
    if rt is None:
        pytest.skip(f"ROCm's {kind} runtime not found")
    lib = build.SAN_LIB if kind == "asan" else build.UBSAN_LIB
    if not os.path.exists(lib):
        build.build_hostsan(kind)
    env = dict(os.environ)
    env["PB_SANITIZED_LIBRARY"] = lib
    if kind == "asan":
        env["LD_PRELOAD"] = rt + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:verify_asan_link_order=0"
        env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    else:
        d = os.path.dirname(rt)
        env["LD_LIBRARY_PATH"] = d + (":" + env["LD_LIBRARY_PATH"]
                                      if env.get("LD_LIBRARY_PATH") else "")
    return env


@pytest.mark.parametrize("kind", ["asan", "ubsan"])
def test_library_host_code_error_paths_under_sanitizers(kind):
    """Without a GPU: pb_create fails cleanly and every §8(b) call rejects
    NULL arguments, with no sanitizer report."""
    import sys
    env = sanitized_library_env(kind)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "hostsan_driver.py"), "cpu"],
                       capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:], r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "cpu ok" in r.stdout
