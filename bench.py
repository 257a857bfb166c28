#!/usr/bin/env python3
"""Benchmark of the DSBI Poisson-Boltzmann hot path on one MI355X.

One step = one whole solve of the large star-shaped synthetic protein surface
(327,680 triangles, 10,000 interior charges): collocation geometry, source
terms, restarted GMRES(10) with the refined-FP32 matvec (FP64 outer
residuals, FP64 Arnoldi) and the block-diagonal leaf preconditioner (the
paper's leaf size N0 = 100 by default here, 24 on the smaller surfaces),
solvation energy.  Inputs are device-resident before
the timed region starts.  The solve tolerance is the loosest of the decade
ladder 1e-4, 1e-5, ... whose energy is within 1e-6 (relative) of an FP64
solve at tol 1e-12; the ladder search runs before timing.

The same JSON line carries two more legs, each measured the same way:
`star81920` (81,920 triangles, 2,000 charges) and `batch64` (64 star
surfaces of 5,120-81,920 triangles solved for E_sol and forces in one
pb_solve_batch call, against the same 64 solves one at a time).

Prints one JSON line.  `value` = matvec pair interactions per second over
the whole step (all FP32 and FP64 matvecs, N(N-1) pairs each) in G/s;
`ms_per_step` = time to E_solv at 1e-6 relative error.
"""
from __future__ import annotations

import argparse
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 58.0          # algorithmic FLOP of one matvec pair (FMA = 2)
PEAK_FP32_VECTOR = 157.3e12   # MI355X published FP32 vector peak
PEAK_FP64_VECTOR = 78.6e12
TOL_LADDER = [1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10]
E_TARGET = 1e-6
PAIRWISE = 8   # pb_set_sweep_config kind of the pairwise sweep (PB_SWEEP_PAIRWISE)
BANDED = 16    # the banded pairwise FP32 sweep (PB_SWEEP_BANDED)

WORKLOADS = {"star327680": "large_star_protein", "star81920": "star_protein"}
# preconditioner leaf size per workload unless --precond-leaf is given: the
# paper's N0 = 100 on the large surface (7 iterations against 8 at leaf 24,
# 6 % less time); 24 on the 81,920-triangle surface and the batch, where the
# larger blocks' inversion costs more than the iteration they save
DEFAULT_LEAF = {"star327680": 100, "star81920": 24, "batch64": 24}


def leaf_for(key: str, args) -> int:
    return args.precond_leaf if args.precond_leaf is not None else DEFAULT_LEAF[key]


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def fp32_kernel_name(kind: int) -> str:
    return {PAIRWISE: "k_pairs_f32_sym", BANDED: "k_pairs_f32_band"}.get(kind, "k_pairs_f32_fwd")


def fp64_kernel_name(kind: int) -> str:
    return "k_pairs_f64_sym" if kind == PAIRWISE else "k_pairs<double>"


def sweep_label(kind: int) -> str:
    return {PAIRWISE: "pairwise", BANDED: "pairwise, banded"}.get(
        kind, f"per-target, {kind} targets per thread")


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace runs collapsed, so
    that the digest follows the code and not its commentary."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_digest(kind: int) -> str:
    """SHA-256 of the FP32 forward sweep's code (comments and layout
    stripped): the shared device headers, the kernel interface header (it
    fixes the FP32 length unit and the tile sizes), the host work plans (they
    set the order in which items reach the XCDs, hence the traffic) and the
    text of the sweep kernel that `kind` selects."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2312_10044_amd", "csrc")
    dev = "".join(open(os.path.join(csrc, f)).read()
                  for f in ("pb_fp64math.h", "pb_device.h", "pb_kernels.h", "pb_host.h",
                            "pb_host.cpp")
                  if os.path.exists(os.path.join(csrc, f)))
    ker = open(os.path.join(csrc, "pb_kernels.hip")).read()
    name = fp32_kernel_name(kind)
    b0 = ker.index(f" void {name}(")
    a = ker.rindex("template <", 0, b0)
    b = ker.index("\n}\n", b0) + 3
    return hashlib.sha256(_code_only(dev + ker[a:b]).encode()).hexdigest()


def counter_record(workload: str, sweep):
    """The committed rocprofv3 counter record of the FP32 sweep on this
    workload (calibrated FETCH_SIZE/WRITE_SIZE bytes, hardware-counted VALU
    FLOPs per launch), or None when the kernel source or its launch
    configuration changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{fp32_kernel_name(sweep[0])}_{workload}_counters.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if (rec.get("kernel_digest") != kernel_digest(sweep[0])
            or [rec.get("sweep_kind"), rec.get("target_waves")] != list(sweep)):
        return None
    return rec


def cpu_baseline(w, seconds=12.0):
    """The FP64 oracle's matvec on a bounded sample of target rows of the
    same workload, on the host's cores."""
    import numpy as np
    from oracle import dsbi
    g = dsbi.geometry(w.verts, w.tris)
    x = np.random.default_rng(0).normal(size=2 * g.n)
    rng = np.random.default_rng(1)
    probe = np.sort(rng.choice(g.n, 128, replace=False))
    t0 = time.perf_counter()
    dsbi.matvec(g, w.eps_out / w.eps_in, w.kappa, x, rows=probe)
    dt = time.perf_counter() - t0
    rows_n = int(min(g.n, max(128, 128 * seconds / max(dt, 1e-3))))
    rows = np.sort(rng.choice(g.n, rows_n, replace=False))
    t0 = time.perf_counter()
    dsbi.matvec(g, w.eps_out / w.eps_in, w.kappa, x, rows=rows)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": rows_n * (g.n - 1) / dt / 1e9,
        "unit": "G pair-interactions/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"FP64 oracle matvec, {rows_n} of {g.n} target rows of the same "
                  f"{g.n}-triangle surface ({rows_n * (g.n - 1):.3g} pairs, {dt:.1f} s)",
    }


def make_workload(name):
    import synth
    return getattr(synth, WORKLOADS[name])()


def solve_leg(ctx, w, key, args, steps, warmup, compare=True, host_arrays=True):
    """Time-to-solution and matvec pair rate of one workload: the reference
    FP64 energy, the tolerance pick, `warmup` untimed and `steps` timed
    device-resident solves, the dominant sweep's live timing, and optionally
    the host-array solve and the comparison variants."""
    import numpy as np
    import torch
    from paper_2312_10044_amd import Params, PB_FP64, PB_FP32_IR
    from paper_2312_10044_amd import pbsolve as pbs

    dev = torch.device("cuda:0")
    N = w.n_tri
    _log(f"bench: workload {w.name}: {N} triangles, {w.n_charges} charges")
    tv = torch.from_numpy(w.verts).to(dev)
    tt = torch.from_numpy(w.tris.astype(np.int32)).to(dev)
    tp = torch.from_numpy(w.pos).to(dev)
    tq = torch.from_numpy(w.q).to(dev)
    phi = torch.empty(N, dtype=torch.float64, device=dev)
    dphi = torch.empty_like(phi)
    torch.cuda.synchronize()

    def solve(params):
        info = ctx.pb_solve_dev(tv, tt, tp, tq, params, phi, dphi)
        if info.status != pbs.PB_OK:
            raise RuntimeError(f"solve did not converge: {info}")
        return info

    base = dict(eps_in=w.eps_in, eps_out=w.eps_out, kappa=w.kappa, restart=10, max_iter=2000)
    tuned = ctx.get_sweep_config()
    ref = solve(Params(tol=1e-12, precision=PB_FP64, precond_leaf=leaf_for(key, args), **base))
    e_ref = ref.e_solv
    _log(f"bench: FP64 reference E={e_ref:.10f} (tol 1e-12, {ref.iters} iterations)")

    def params_for(precision, leaf, tol):
        if precision == PB_FP32_IR:
            return Params(tol=tol, precision=PB_FP32_IR, inner_tol=0.1 * tol, max_refine=20,
                          precond_leaf=leaf, **base)
        return Params(tol=tol, precision=PB_FP64, precond_leaf=leaf, **base)

    def pick(precision, leaf):
        for tol in TOL_LADDER:
            p = params_for(precision, leaf, tol)
            info = solve(p)
            err = abs(info.e_solv - e_ref) / abs(e_ref)
            _log(f"bench: {w.name} precision={precision} leaf={leaf} tol={tol:g} E err={err:.2e} "
                 f"iters={info.iters} t={info.seconds:.3f}s")
            if err <= E_TARGET:
                return p, err
        raise RuntimeError("no tolerance on the ladder reached the energy target")

    def timed_once(p):
        solve(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = solve(p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return {"time_to_solution_s": dt, "tol": p.tol, "iters": info.iters,
                "matvecs_fp32": info.matvecs_fp32, "matvecs_fp64": info.matvecs_fp64,
                "e_rel_err": abs(info.e_solv - e_ref) / abs(e_ref),
                "gpairs_per_s": (info.matvecs_fp32 + info.matvecs_fp64) * float(N) * (N - 1)
                / dt / 1e9}

    prec = PB_FP32_IR if args.precision == "fp32-ir" else PB_FP64
    leaf = leaf_for(key, args)
    params, _err_pick = pick(prec, leaf)

    for _ in range(warmup):
        solve(params)
    ctx.profile_reset()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    step_s = []
    for k in range(steps):
        ts = time.perf_counter()
        infos.append(solve(params))   # returns once E_solv is on the host
        step_s.append(time.perf_counter() - ts)
        _log(f"bench: {w.name} step {k + 1}/{steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile_enable(False)
    ms_step = 1e3 * elapsed / steps
    pairs_per_mv = float(N) * float(N - 1)
    n_mv = sum(i.matvecs_fp32 + i.matvecs_fp64 for i in infos)
    value = n_mv * pairs_per_mv / elapsed / 1e9
    errs = [abs(i.e_solv - e_ref) / abs(e_ref) for i in infos]

    dom = pbs.PB_KERNEL_PAIRS_FP32 if prec == PB_FP32_IR else pbs.PB_KERNEL_PAIRS_FP64
    launches, kms, kpairs = ctx.profile_read(dom)
    avg_ms = kms / max(launches, 1)
    pairs_launch = kpairs / max(launches, 1)
    achieved = FLOP_PER_PAIR * pairs_launch / (avg_ms * 1e-3)
    peak = PEAK_FP32_VECTOR if prec == PB_FP32_IR else PEAK_FP64_VECTOR
    kernel_rows = {}
    for name, kid in (("pairs_fp32", pbs.PB_KERNEL_PAIRS_FP32),
                      ("pairs_fp64", pbs.PB_KERNEL_PAIRS_FP64),
                      ("source", pbs.PB_KERNEL_SOURCE), ("charge", pbs.PB_KERNEL_CHARGE)):
        n_l, ms_l, pr_l = ctx.profile_read(kid)
        if n_l:
            kernel_rows[name] = {"launches": n_l, "avg_ms": ms_l / n_l,
                                 "gpairs_per_s": pr_l / (ms_l * 1e-3) / 1e9}
    rec = counter_record(key, tuned) if prec == PB_FP32_IR else None
    counted = None
    if rec is not None:
        fl = float(rec["valu_flop_per_launch"])
        counted = {"flop_per_launch": fl, "achieved": fl / (avg_ms * 1e-3) / 1e12,
                   "frac": fl / (avg_ms * 1e-3) / peak,
                   "flop_per_ordered_pair": fl / pairs_launch}
    roofline = {
        "bound": "alu",
        "kernel": (fp32_kernel_name(tuned[0]) if prec == PB_FP32_IR
                   else fp64_kernel_name(ctx.get_fp64_sweep())),
        "achieved": achieved / 1e12,
        "peak": peak / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": float(rec["bytes_per_launch"]) if rec is not None else None,
        "basis": "algorithmic: 58 FLOP per ordered pair x N(N-1) pairs per launch, over the "
                 "launch's HIP-event duration (the pairwise sweep shares work between the two "
                 "directions of a pair, so it executes fewer FLOPs than this)",
        "counted": counted,
        "traffic_unit": "bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
        "flop_per_pair": FLOP_PER_PAIR,
        "pairs_per_launch": pairs_launch,
        "avg_launch_ms": avg_ms,
        "launches": launches,
    }

    host_med = None
    if host_arrays:
        # the same solve through the host-array entry point (surface and
        # charges copied in, phi/dphi copied out over PCIe): reported beside
        # `value`, which stays the device-resident rate
        ctx.pb_solve(w.verts, w.tris, w.pos, w.q, params)
        host_s = []
        for _ in range(min(steps, 5)):
            ts = time.perf_counter()
            ctx.pb_solve(w.verts, w.tris, w.pos, w.q, params)
            host_s.append(time.perf_counter() - ts)
        host_med = float(np.median(host_s))
        _log(f"bench: {w.name} host-array solves: median {1e3 * host_med:.2f} ms")

    cmp = {}
    if compare:
        variants = [("fp64_same_preconditioner", PB_FP64, leaf),
                    ("fp32_ir_no_preconditioner", PB_FP32_IR, 0),
                    ("fp64_no_preconditioner", PB_FP64, 0)]
        for name, pr, lf in variants:
            if pr == prec and lf == leaf:
                continue
            pv, _e = pick(pr, lf)
            cmp[name] = timed_once(pv)

    return {
        "n_tri": N,
        "n_charges": w.n_charges,
        "value": value,
        "ms_per_step": ms_step,
        "tol": params.tol,
        "inner_tol": params.inner_tol if prec == PB_FP32_IR else None,
        "e_ref_fp64_tol1e-12": e_ref,
        "e_solv": infos[-1].e_solv,
        "e_rel_err": max(errs),
        "iters": infos[-1].iters,
        "matvecs_fp32": infos[-1].matvecs_fp32,
        "matvecs_fp64": infos[-1].matvecs_fp64,
        "refinements": infos[-1].refinements,
        "time_to_solution_median_s": float(np.median(step_s)),
        "time_to_solution_host_arrays_median_s": host_med,
        "step_s": [round(t, 6) for t in step_s],
        "kernels": kernel_rows,
        "roofline": roofline,
        "compare": cmp,
        "fp32_sweep": {"kind": sweep_label(tuned[0]), "target_waves": tuned[1]},
    }


def batch_leg(ctx, args, steps):
    """64 star surfaces of uneven size (5,120-81,920 triangles, 100-2,000
    charges): E_sol plus forces of all of them in one pb_solve_batch call
    (shared launches, hipGraph-replayed restart cycles, autotuned tiles)
    against the same 64 solves one at a time.  Each variant's tolerance is the
    loosest on the decade ladder whose worst energy error over the 64 systems
    is within 1e-6 of an FP64 batch solve at tol 1e-12."""
    import numpy as np
    import torch

    import synth
    from paper_2312_10044_amd import Params, PB_FP64, PB_FP32_IR

    systems = synth.batch_conformations()
    sys_list = [(w.verts, w.tris, w.pos, w.q) for w in systems]
    n_tri = [w.n_tri for w in systems]
    pairs = float(sum(float(n) * (n - 1) for n in n_tri))
    _log(f"bench batch: {len(systems)} systems, {sum(n_tri)} triangles, "
         f"{pairs:.3g} pairs per batched matvec")
    leaf = leaf_for("batch64", args)
    prec = PB_FP32_IR if args.precision == "fp32-ir" else PB_FP64

    def prm(precision, tol):
        if precision == PB_FP32_IR:
            return Params(tol=tol, precision=PB_FP32_IR, inner_tol=0.1 * tol, restart=10,
                          max_iter=2000, precond_leaf=leaf)
        return Params(tol=tol, precision=PB_FP64, restart=10, max_iter=2000, precond_leaf=leaf)

    tuned_kind, tuned_tiles = ctx.pb_autotune_batch(sys_list, prm(prec, 1e-6))
    _log(f"bench batch: autotuned sweep kind={tuned_kind} tiles/item={tuned_tiles}")
    e_ref, _inf, g_ref, _q = ctx.pb_solve_batch(sys_list, prm(PB_FP64, 1e-12), forces=True)
    e_ref = np.asarray(e_ref)

    def energy_err(e):
        return float(np.max(np.abs(np.asarray(e) - e_ref) / np.abs(e_ref)))

    def force_err(g):
        out, k = 0.0, 0
        for w in systems:
            a, b = g[k:k + w.n_charges], g_ref[k:k + w.n_charges]
            out = max(out, float(np.abs(a - b).max() / np.abs(b).max()))
            k += w.n_charges
        return out

    def pick(run):
        for tol in TOL_LADDER:
            e = run(tol)
            err = energy_err(e)
            _log(f"bench batch: tol={tol:g} worst E err={err:.2e}")
            if err <= E_TARGET:
                return tol, err
        raise RuntimeError("no tolerance on the ladder reached the energy target")

    def batched(tol):
        e, infos, g, _gq = ctx.pb_solve_batch(sys_list, prm(prec, tol), forces=True)
        if any(i.status != 0 for i in infos):
            raise RuntimeError("a batched system did not converge")
        return e

    tol_b, err_b = pick(batched)
    e_b, inf_b, g_b, _q = ctx.pb_solve_batch(sys_list, prm(prec, tol_b), forces=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e_b, inf_b, g_b, _q = ctx.pb_solve_batch(sys_list, prm(prec, tol_b), forces=True)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    _log(f"bench batch: batched {t_batch:.3f} s at tol {tol_b:g}")

    def sequential(precision, tol):
        p1 = prm(precision, tol)
        t = time.perf_counter()
        es = []
        for sysd in sys_list:
            info, _gp, _gq = ctx.pb_forces(*sysd, p1)
            if info.status != 0:
                raise RuntimeError("a sequential solve did not converge")
            es.append(info.e_solv)
        torch.cuda.synchronize()
        return time.perf_counter() - t, es

    seq = {}
    for name, precision in (("sequential_fp64", PB_FP64), ("sequential_fp32_ir", PB_FP32_IR)):
        tol_s, err_s = pick(lambda t: sequential(precision, t)[1])
        t_s, _e = sequential(precision, tol_s)
        seq[name] = {"seconds": t_s, "solves_per_s": len(systems) / t_s, "tol": tol_s,
                     "worst_e_rel_err": err_s, "speedup_of_batch": t_s / t_batch}
        _log(f"bench batch: {name} {t_s:.3f} s at tol {tol_s:g}")
    return {
        "workload": "64 star surfaces, 5,120-81,920 triangles, 100-2,000 charges (seed 5); "
                    "E_sol + forces",
        "n_sys": len(systems),
        "total_triangles": int(sum(n_tri)),
        "pairs_per_batched_matvec": pairs,
        "precision": "FP32 matvec + FP64 restart residuals" if prec == PB_FP32_IR else "FP64",
        "precond_leaf": leaf,
        "tol": tol_b,
        "worst_e_rel_err": energy_err(e_b),
        "worst_force_rel_err_vs_fp64_tol1e-12": force_err(g_b),
        "autotuned": {"sweep_kind": sweep_label(tuned_kind), "tiles_per_item": tuned_tiles},
        "batched_s": t_batch,
        "solves_per_s": len(systems) / t_batch,
        "arnoldi_steps_forward_max": max(i.iters for i in inf_b),
        "arnoldi_steps_adjoint_max": max(i.adjoint_iters for i in inf_b),
        "matvec_gpairs_per_s": sum((i.matvecs_fp32 + i.matvecs_fp64) * float(n) * (n - 1)
                                   for i, n in zip(inf_b, n_tri)) / t_batch / 1e9,
        **seq,
    }


def _tree_record(ctx, w, args, pbs, Params, PB_FP64, PB_FP32_IR):
    import numpy as np
    import torch
    N = w.n_tri
    base = Params(eps_in=w.eps_in, eps_out=w.eps_out, kappa=w.kappa)
    x = np.random.default_rng(0).normal(size=2 * N)
    out = {"n_tri": N}
    y64 = ctx.pb_matvec(w.verts, w.tris, x, base, precision=PB_FP64)
    ctx.pb_matvec(w.verts, w.tris, x, base, precision=PB_FP32_IR)
    for kid, prec, label in ((pbs.PB_KERNEL_PAIRS_FP64, PB_FP64, "direct_fp64"),
                             (pbs.PB_KERNEL_PAIRS_FP32, PB_FP32_IR, "direct_fp32_pairwise")):
        ctx.profile_reset()
        ctx.profile_enable(True)
        for _ in range(max(1, args.steps)):
            y = ctx.pb_matvec(w.verts, w.tris, x, base, precision=prec)
        ctx.profile_enable(False)
        n_l, ms_l, _p = ctx.profile_read(kid)
        out[label] = {"ms": ms_l / n_l,
                      "rel_err_vs_fp64": float(np.abs(y - y64).max() / np.abs(y64).max())}
    y, cnt = ctx.pb_matvec_tree(w.verts, w.tris, x, base, theta=args.theta, order=args.order,
                                leaf_size=args.leaf, with_counts=True)
    ctx.profile_reset()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps)):
        y = ctx.pb_matvec_tree(w.verts, w.tris, x, base, theta=args.theta, order=args.order,
                               leaf_size=args.leaf)
    wall = (time.perf_counter() - t0) / max(1, args.steps)
    ctx.profile_enable(False)
    n_l, ms_l, _p = ctx.profile_read(pbs.PB_KERNEL_TREE)
    out["treecode"] = {"ms": ms_l / n_l, "call_wall_ms": wall * 1e3,
                       "rel_err_vs_fp64": float(np.abs(y - y64).max() / np.abs(y64).max()),
                       "particle_cluster": cnt[0], "particle_particle": cnt[1],
                       "nodes": cnt[2]}
    out["speedup_tree_vs_fp64_direct"] = out["direct_fp64"]["ms"] / out["treecode"]["ms"]
    out["speedup_tree_vs_fp32_pairwise"] = (out["direct_fp32_pairwise"]["ms"]
                                            / out["treecode"]["ms"])
    return out


def run_tree(args):
    """Treecode matvec (theta 0.8, p 3, N0 100 unless given) against the
    direct sums: kernel time per matvec (cluster moments plus tree walk; the
    host-side tree build is in the call's wall time) and the error against the
    FP64 direct matvec.  --tree-freqs lists star surfaces of 20 f^2 triangles
    (the break-even sweep); otherwise --workload is used."""
    import synth
    from paper_2312_10044_amd import Context, Params, PB_FP64, PB_FP32_IR, PB_SWEEP_PAIRWISE
    from paper_2312_10044_amd import pbsolve as pbs

    if args.tree_freqs:
        works = [synth.star_protein(freq=int(f), r0=20.0 * int(f) / 64.0, n_charges=1, seed=2)
                 for f in args.tree_freqs.split(",")]
    else:
        works = [make_workload(args.workload)]
    ctx = Context(0)
    ctx.set_sweep_config(PB_SWEEP_PAIRWISE, 0)
    recs = []
    for w in works:
        _log(f"bench tree: {w.n_tri} triangles")
        recs.append(_tree_record(ctx, w, args, pbs, Params, PB_FP64, PB_FP32_IR))
    solve_cmp = None
    if len(works) == 1:
        # whole solves: treecode GMRES against the direct solves, same preconditioner
        w = works[0]
        base = dict(eps_in=w.eps_in, eps_out=w.eps_out, kappa=w.kappa, restart=10,
                    max_iter=2000)
        args_s = (w.verts, w.tris, w.pos, w.q)
        ref, _p, _d = ctx.pb_solve(*args_s, Params(tol=1e-12, **base))
        solve_cmp = {}
        tleaf = args.precond_leaf if args.precond_leaf is not None else 24
        for label, fn, prm in (
                ("treecode_fp64", "tree", Params(tol=1e-6, precond_leaf=tleaf, **base)),
                ("direct_fp64", "direct", Params(tol=1e-6, precond_leaf=tleaf, **base)),
                ("direct_fp32_ir", "direct", Params(tol=1e-6, precision=PB_FP32_IR,
                                                    inner_tol=1e-7,
                                                    precond_leaf=tleaf, **base))):
            def run():
                if fn == "tree":
                    return ctx.pb_solve_tree(*args_s, prm, theta=args.theta, order=args.order,
                                             leaf_size=args.leaf)[0]
                return ctx.pb_solve(*args_s, prm)[0]
            run()
            t0 = time.perf_counter()
            info = run()
            dt = time.perf_counter() - t0
            solve_cmp[label] = {"seconds": dt, "iters": info.iters, "status": info.status,
                                "e_rel_err": abs(info.e_solv - ref.e_solv) / abs(ref.e_solv)}
        _log(f"bench tree: solves {solve_cmp}")
    ctx.close()
    out = {"mode": "tree", "theta": args.theta, "order": args.order, "leaf_size": args.leaf}
    if len(recs) == 1:
        out.update(recs[0])
        out["solve_tol_1e-6_host_arrays"] = solve_cmp
    else:
        out["sizes"] = recs
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32-ir", "fp64"], default="fp32-ir")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="star327680",
                    help="headline workload (default: 327,680 triangles, 10,000 charges)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 81,920-triangle leg of the solve benchmark")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-system batch leg of the solve benchmark")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--theta", type=float, default=0.8, help="treecode MAC parameter (mode tree)")
    ap.add_argument("--order", type=int, default=3, help="treecode Taylor order (mode tree)")
    ap.add_argument("--leaf", type=int, default=100, help="treecode leaf size N0 (mode tree)")
    ap.add_argument("--tree-freqs", default="",
                    help="mode tree: comma-separated star frequencies f (20 f^2 triangles, "
                         "radius scaled with f) for a break-even sweep")
    ap.add_argument("--mode", choices=["solve", "matvec", "copy", "batch", "tree", "probe"],
                    default="solve",
                    help="solve: the benchmark; matvec: only --steps matvecs of --precision "
                         "(for counter runs); copy: a device copy of --copy-mib MiB (the "
                         "reference kernel that calibrates FETCH_SIZE/WRITE_SIZE); batch: only "
                         "the 64-system leg; tree: treecode matvec vs the direct sums; probe: "
                         "the library's counter-calibration kernels (known VALU operation "
                         "counts), --steps launches of each kind")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--precond-leaf", type=int, default=None,
                    help="leaf size of the block-diagonal preconditioner (0 = none; default "
                         "100 on the 327,680-triangle surface, 24 on the 81,920-triangle "
                         "surface and the batch)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the FP32 sweep configurations first and use the fastest")
    ap.add_argument("--fp32-sweep", choices=["default", "pairwise", "banded", "1", "2"],
                    default="default", help="FP32 sweep kind (default: the library's)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2312_10044_amd import Context, Params, PB_FP64, PB_FP32_IR
    from paper_2312_10044_amd import pbsolve as pbs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    if args.mode == "copy":
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(max(1, args.steps)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read": n * 8, "bytes_written": n * 8,
                          "launches": max(1, args.steps)}), flush=True)
        return
    if args.mode == "tree":
        run_tree(args)
        return
    ctx = Context(0, torch.cuda.current_stream())
    if args.mode == "probe":
        rec = {}
        for name, kind in (("fma_f32", pbs.PB_PROBE_FMA_F32), ("fma_f64", pbs.PB_PROBE_FMA_F64),
                           ("exp_f32", pbs.PB_PROBE_EXP_F32)):
            ops = [ctx.probe_valu(kind) for _ in range(max(1, args.steps))]
            rec[name] = {"launches": len(ops), "lane_ops_per_launch": ops[0]}
        ctx.close()
        print(json.dumps({"mode": "probe", **rec}), flush=True)
        return
    if args.mode == "batch":
        out = {"mode": "batch", **batch_leg(ctx, args, max(1, args.steps))}
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    w = make_workload(args.workload)
    N = w.n_tri
    base = dict(eps_in=w.eps_in, eps_out=w.eps_out, kappa=w.kappa, restart=10, max_iter=2000)
    if args.fp32_sweep != "default":
        ctx.set_sweep_config({"pairwise": PAIRWISE, "banded": BANDED}.get(args.fp32_sweep)
                             or int(args.fp32_sweep), 0)
    if args.autotune:
        tuned = ctx.pb_autotune(w.verts, w.tris, Params(**base))
    else:
        tuned = ctx.get_sweep_config()
    _log(f"bench: FP32 sweep: targets/thread={tuned[0]} target_waves={tuned[1]} "
         f"({'autotuned' if args.autotune else 'library default'})")
    if args.mode == "matvec":
        prec = PB_FP32_IR if args.precision == "fp32-ir" else PB_FP64
        tv = torch.from_numpy(w.verts).to(dev)
        tt = torch.from_numpy(w.tris.astype(np.int32)).to(dev)
        x = torch.from_numpy(np.random.default_rng(0).normal(size=2 * N)).to(dev)
        y = torch.empty_like(x)
        ctx.profile_reset()
        ctx.profile_enable(True)
        for _ in range(args.steps):
            ctx.pb_matvec_dev(tv, tt, x, y, Params(**base), precision=prec)
        torch.cuda.synchronize()
        kid = pbs.PB_KERNEL_PAIRS_FP32 if prec == PB_FP32_IR else pbs.PB_KERNEL_PAIRS_FP64
        n_l, ms_l, pr_l = ctx.profile_read(kid)
        print(json.dumps({"mode": "matvec", "precision": args.precision, "n_tri": N,
                          "kernel": (fp32_kernel_name(tuned[0]) if prec == PB_FP32_IR
                                     else fp64_kernel_name(ctx.get_fp64_sweep())),
                          "kernel_digest": (kernel_digest(tuned[0]) if prec == PB_FP32_IR
                                            else None),
                          "launches": n_l, "avg_ms": ms_l / n_l,
                          "pairs_per_launch": pr_l / n_l,
                          "tflops_algorithmic": FLOP_PER_PAIR * pr_l / (ms_l * 1e-3) / 1e12,
                          "fp32_sweep": list(tuned)}), flush=True)
        ctx.close()
        return

    head = solve_leg(ctx, w, args.workload, args, args.steps, args.warmup,
                     compare=not args.no_fp64_compare, host_arrays=True)
    legs = {}
    if not args.no_secondary and args.workload != "star81920":
        w2 = make_workload("star81920")
        legs["star81920"] = solve_leg(ctx, w2, "star81920", args, max(args.steps, 5), max(args.warmup, 1),
                                      compare=False, host_arrays=False)
    if not args.no_batch:
        legs["batch64"] = batch_leg(ctx, args, max(1, min(args.steps, 3)))
    ctx.close()
    prec = PB_FP32_IR if args.precision == "fp32-ir" else PB_FP64
    out = {
        "metric": "BIE matvec G-pair-interactions/s; time to E_solv at 1e-6 rel. error",
        "value": head["value"],
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == PB_FP32_IR else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"star-shaped surface {N} triangles, {w.n_charges} charges, "
                        f"eps 1/80, kappa 0.1257; one full solve to E_solv within 1e-6",
            "n_tri": N,
            "n_charges": w.n_charges,
            "precision": "FP32 matvec + FP64 refinement" if prec == PB_FP32_IR else "FP64",
            "precond_leaf": leaf_for(args.workload, args),
            "tol": head["tol"],
            "tol_ladder": TOL_LADDER,
            "inner_tol": head["inner_tol"],
            "gmres_restart": 10,
            "fp32_sweep": head["fp32_sweep"],
        },
        "time_to_solution_s": head["ms_per_step"] / 1e3,
        "roofline": head.pop("roofline"),
        "cpu_baseline": None,
        **{k: v for k, v in head.items() if k not in ("value", "ms_per_step")},
        "legs": legs,
    }
    if not args.no_cpu_baseline:
        _log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
