#!/usr/bin/env python3
"""Benchmark of the DSBI Poisson-Boltzmann hot path on one MI355X.

One step = one whole solve of the star-shaped synthetic protein surface
(81,920 triangles, 2,000 interior charges): collocation geometry, source
terms, restarted GMRES(10) with the refined-FP32 matvec (FP64 outer
residuals, FP64 Arnoldi) and the block-diagonal leaf preconditioner (leaf
size 16 by default), solvation energy.  Inputs are device-resident
before the timed region starts.  The solve tolerance is the loosest of a
fixed ladder whose energy is within 1e-6 (relative) of an FP64 solve at
tol 1e-12; the ladder search runs before timing.

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
TOL_LADDER = [1e-3, 5e-4, 2e-4, 1e-4, 5e-5, 2e-5, 1e-5, 5e-6, 2e-6, 1e-6, 5e-7, 2e-7, 1e-7,
              1e-8]
E_TARGET = 1e-6


TRAFFIC_RECORDS = {   # FETCH_SIZE/WRITE_SIZE records per FP32 sweep kind
    8: os.path.join(ROOT, "profiles", "k_pairs_f32_sym_star81920_traffic.json"),
    1: os.path.join(ROOT, "profiles", "k_pairs_f32_star81920_traffic.json"),
}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


PAIRWISE = 8   # pb_set_sweep_config kind of the pairwise sweep (PB_SWEEP_PAIRWISE)


def fp32_kernel_name(kind: int) -> str:
    return "k_pairs_f32_sym" if kind == PAIRWISE else "k_pairs_f32_fwd"


def fp64_kernel_name(kind: int) -> str:
    return "k_pairs_f64_sym" if kind == PAIRWISE else "k_pairs<double>"


def sweep_label(kind: int) -> str:
    return "pairwise" if kind == PAIRWISE else f"per-target, {kind} targets per thread"


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace runs collapsed, so
    that the digest follows the code and not its commentary."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_digest(kind: int) -> str:
    """SHA-256 of the FP32 forward sweep's code (comments and layout
    stripped): the shared device header plus the text of the sweep kernel
    that `kind` selects."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2312_10044_amd", "csrc")
    dev = open(os.path.join(csrc, "pb_device.h")).read()
    ker = open(os.path.join(csrc, "pb_kernels.hip")).read()
    name = fp32_kernel_name(kind)
    b0 = ker.index(f" void {name}(")
    a = ker.rindex("template <", 0, b0)
    b = ker.index("\n}\n", b0) + 3
    return hashlib.sha256(_code_only(dev + ker[a:b]).encode()).hexdigest()


def measured_traffic(n_tri, sweep):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE record,
    or None when the kernel source or its configuration changed since."""
    try:
        rec = json.load(open(TRAFFIC_RECORDS[sweep[0]]))
    except (KeyError, OSError, ValueError):
        return None
    if (rec.get("kernel_digest") != kernel_digest(sweep[0]) or rec.get("n_tri") != n_tri
            or [rec.get("sweep_kind"), rec.get("target_waves")] != list(sweep)):
        return None
    return float(rec["bytes_per_launch"])


def cpu_baseline(w, seconds=12.0):
    """The FP64 oracle's matvec on a bounded sample of target rows of the
    same workload, on the host's cores."""
    import numpy as np
    from oracle import dsbi
    g = dsbi.geometry(w.verts, w.tris)
    x = np.random.default_rng(0).normal(size=2 * g.n)
    rng = np.random.default_rng(1)
    probe = np.sort(rng.choice(g.n, 256, replace=False))
    t0 = time.perf_counter()
    dsbi.matvec(g, w.eps_out / w.eps_in, w.kappa, x, rows=probe)
    dt = time.perf_counter() - t0
    rows_n = int(min(g.n, max(256, 256 * seconds / max(dt, 1e-3))))
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


def run_batch(args):
    """64 star surfaces of uneven size (5,120-81,920 triangles, 100-2,000
    charges): E_sol plus forces for all of them in one pb_solve_batch call
    (shared persistent launches, hipGraph-replayed restart cycles) against
    the same 64 solves one at a time with pb_forces in FP64."""
    import numpy as np
    import torch

    import synth
    from paper_2312_10044_amd import Context, Params, PB_FP64, PB_FP32_IR

    systems = synth.batch_conformations()
    sys_list = [(w.verts, w.tris, w.pos, w.q) for w in systems]
    n_tri = [w.n_tri for w in systems]
    pairs = float(sum(float(n) * (n - 1) for n in n_tri))
    _log(f"bench batch: {len(systems)} systems, {sum(n_tri)} triangles, "
         f"{pairs:.3g} pairs per batched matvec")
    ctx = Context(0)
    tol = 1e-6
    leaf = args.precond_leaf
    prec = PB_FP32_IR if args.precision == "fp32-ir" else PB_FP64
    pb = Params(tol=tol, precision=prec, restart=10, max_iter=2000, precond_leaf=leaf)
    # tile shapes of the batched sweeps picked on this batch, outside the timing
    tuned_kind, tuned_tiles = ctx.pb_autotune_batch(sys_list, pb)
    _log(f"bench batch: autotuned sweep kind={tuned_kind} tiles/item={tuned_tiles}")
    e_b, inf_b, g_b, q_b = ctx.pb_solve_batch(sys_list, pb, forces=True)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps)):
        e_b, inf_b, g_b, q_b = ctx.pb_solve_batch(sys_list, pb, forces=True)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / max(1, args.steps)
    _log(f"batched: {t_batch:.3f} s")

    def sequential(leaf_s, prec_s=PB_FP64):
        p1 = Params(tol=tol, precision=prec_s, restart=10, max_iter=2000, precond_leaf=leaf_s)
        ctx.pb_forces(*sys_list[0], p1)
        t = time.perf_counter()
        es = []
        for sysd in sys_list:
            info, _gp, _gq = ctx.pb_forces(*sysd, p1)
            es.append(info.e_solv)
        torch.cuda.synchronize()
        return time.perf_counter() - t, es

    t_seq, e_s = sequential(leaf)
    _log(f"sequential FP64 (leaf {leaf}): {t_seq:.3f} s")
    t_seq0, e_s0 = sequential(0) if leaf > 0 else (t_seq, e_s)
    _log(f"sequential FP64 (no preconditioner): {t_seq0:.3f} s")
    t_seq32, _e_s32 = sequential(leaf, PB_FP32_IR)
    _log(f"sequential refined FP32 (leaf {leaf}): {t_seq32:.3f} s")
    rel = float(np.max(np.abs(np.asarray(e_b) - np.asarray(e_s)) / np.abs(e_s)))
    rel0 = float(np.max(np.abs(np.asarray(e_b) - np.asarray(e_s0)) / np.abs(e_s0)))
    out = {
        "mode": "batch",
        "metric": "solves/s (E_sol + forces), batched vs one-at-a-time FP64",
        "n_sys": len(systems),
        "total_triangles": int(sum(n_tri)),
        "pairs_per_batched_matvec": pairs,
        "precision": "FP32 matvec + FP64 restart residuals" if prec == PB_FP32_IR else "FP64",
        "precond_leaf": leaf,
        "tol": tol,
        "autotuned": {"sweep_kind": sweep_label(tuned_kind), "tiles_per_item": tuned_tiles},
        "batched_s": t_batch,
        "batched_solves_per_s": len(systems) / t_batch,
        "sequential_fp64_same_preconditioner_s": t_seq,
        "sequential_solves_per_s": len(systems) / t_seq,
        "speedup": t_seq / t_batch,
        "sequential_fp64_no_preconditioner_s": t_seq0,
        "speedup_vs_unpreconditioned_fp64": t_seq0 / t_batch,
        "sequential_fp32ir_same_preconditioner_s": t_seq32,
        "speedup_vs_sequential_fp32ir": t_seq32 / t_batch,
        "max_rel_energy_diff_vs_sequential": rel,
        "max_rel_energy_diff_vs_unpreconditioned": rel0,
        "arnoldi_steps_forward_max": max(i.iters for i in inf_b),
        "arnoldi_steps_adjoint_max": max(i.adjoint_iters for i in inf_b),
        "matvec_gpairs_per_s_batched": sum(
            (i.matvecs_fp32 + i.matvecs_fp64) * float(n) * (n - 1)
            for i, n in zip(inf_b, n_tri)) / t_batch / 1e9,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def _tree_record(ctx, w, args, pbs, Params, PB_FP64, PB_FP32_IR, PB_SWEEP_PAIRWISE):
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
        works = [synth.star_protein() if args.workload == "star81920"
                 else synth.large_star_protein()]
    ctx = Context(0)
    ctx.set_sweep_config(PB_SWEEP_PAIRWISE, 0)
    recs = []
    for w in works:
        _log(f"bench tree: {w.n_tri} triangles")
        recs.append(_tree_record(ctx, w, args, pbs, Params, PB_FP64, PB_FP32_IR,
                                 PB_SWEEP_PAIRWISE))
    solve_cmp = None
    if len(works) == 1:
        # whole solves: treecode GMRES against the direct solves, same preconditioner
        w = works[0]
        base = dict(eps_in=w.eps_in, eps_out=w.eps_out, kappa=w.kappa, restart=10,
                    max_iter=2000)
        args_s = (w.verts, w.tris, w.pos, w.q)
        ref, _p, _d = ctx.pb_solve(*args_s, Params(tol=1e-12, **base))
        solve_cmp = {}
        for label, fn, prm in (
                ("treecode_fp64", "tree", Params(tol=1e-6, precond_leaf=args.precond_leaf,
                                                 **base)),
                ("direct_fp64", "direct", Params(tol=1e-6, precond_leaf=args.precond_leaf,
                                                 **base)),
                ("direct_fp32_ir", "direct", Params(tol=1e-6, precision=PB_FP32_IR,
                                                    inner_tol=1e-7,
                                                    precond_leaf=args.precond_leaf, **base))):
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
    ap.add_argument("--workload", choices=["star81920", "star327680"], default="star81920")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--theta", type=float, default=0.8, help="treecode MAC parameter (mode tree)")
    ap.add_argument("--order", type=int, default=3, help="treecode Taylor order (mode tree)")
    ap.add_argument("--leaf", type=int, default=100, help="treecode leaf size N0 (mode tree)")
    ap.add_argument("--tree-freqs", default="",
                    help="mode tree: comma-separated star frequencies f (20 f^2 triangles, "
                         "radius scaled with f) for a break-even sweep")
    ap.add_argument("--mode", choices=["solve", "matvec", "copy", "batch", "tree"],
                    default="solve",
                    help="solve: the benchmark; matvec: only --steps matvecs of --precision "
                         "(for counter runs); copy: a device copy of --copy-mib MiB (the "
                         "reference kernel that calibrates FETCH_SIZE/WRITE_SIZE); batch: 64 "
                         "uneven systems in one call; tree: treecode matvec vs the direct sums")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--precond-leaf", type=int, default=24,
                    help="leaf size of the block-diagonal preconditioner (0 = none)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the FP32 sweep configurations first and use the fastest")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
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
    if args.mode == "batch":
        run_batch(args)
        return
    if args.mode == "tree":
        run_tree(args)
        return
    if args.workload == "star81920":
        w = synth.star_protein()
    else:
        w = synth.large_star_protein()
    N = w.n_tri
    _log(f"bench: workload {w.name}: {N} triangles, {w.n_charges} charges")
    tv = torch.from_numpy(w.verts).to(dev)
    tt = torch.from_numpy(w.tris.astype(np.int32)).to(dev)
    tp = torch.from_numpy(w.pos).to(dev)
    tq = torch.from_numpy(w.q).to(dev)
    phi = torch.empty(N, dtype=torch.float64, device=dev)
    dphi = torch.empty_like(phi)
    stream = torch.cuda.current_stream()
    ctx = Context(0, stream)

    def solve(params):
        return ctx.pb_solve_dev(tv, tt, tp, tq, params, phi, dphi)

    base = dict(eps_in=w.eps_in, eps_out=w.eps_out, kappa=w.kappa, restart=10, max_iter=2000)
    if args.autotune:
        tuned = ctx.pb_autotune(w.verts, w.tris, Params(**base))
    else:
        tuned = ctx.get_sweep_config()
    _log(f"bench: FP32 sweep: targets/thread={tuned[0]} target_waves={tuned[1]} "
         f"({'autotuned' if args.autotune else 'library default'})")
    if args.mode == "matvec":
        prec = PB_FP32_IR if args.precision == "fp32-ir" else PB_FP64
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
    ref = solve(Params(tol=1e-12, precision=PB_FP64, **base))
    e_ref = ref.e_solv
    _log(f"bench: FP64 reference E={e_ref:.10f} (tol 1e-12, {ref.iters} iterations)")

    def pick(precision, leaf):
        for tol in TOL_LADDER:
            if precision == PB_FP32_IR:
                p = Params(tol=tol, precision=PB_FP32_IR, inner_tol=0.1 * tol,
                           max_refine=20, precond_leaf=leaf, **base)
            else:
                p = Params(tol=tol, precision=PB_FP64, precond_leaf=leaf, **base)
            info = solve(p)
            err = abs(info.e_solv - e_ref) / abs(e_ref)
            _log(f"bench: precision={precision} leaf={leaf} tol={tol:g} E err={err:.2e} "
                 f"iters={info.iters} t={info.seconds:.3f}s")
            if err <= E_TARGET and info.status == 0:
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
    leaf = args.precond_leaf
    params, err_pick = pick(prec, leaf)

    for _ in range(args.warmup):
        solve(params)
    ctx.profile_reset()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    step_s = []
    for k in range(args.steps):
        ts = time.perf_counter()
        infos.append(solve(params))   # returns once E_solv is on the host
        step_s.append(time.perf_counter() - ts)
        _log(f"bench: step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile_enable(False)
    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / args.steps
    pairs_per_mv = float(N) * float(N - 1)
    n_mv = sum(i.matvecs_fp32 + i.matvecs_fp64 for i in infos)
    value = n_mv * pairs_per_mv / elapsed / 1e9
    errs = [abs(i.e_solv - e_ref) / abs(e_ref) for i in infos]

    dom = pbs.PB_KERNEL_PAIRS_FP32 if prec == PB_FP32_IR else pbs.PB_KERNEL_PAIRS_FP64
    launches, kms, kpairs = ctx.profile_read(dom)
    avg_ms = kms / max(launches, 1)
    achieved = FLOP_PER_PAIR * (kpairs / max(launches, 1)) / (avg_ms * 1e-3)
    peak = PEAK_FP32_VECTOR if prec == PB_FP32_IR else PEAK_FP64_VECTOR
    kernel_rows = {}
    for name, kid in (("pairs_fp32", pbs.PB_KERNEL_PAIRS_FP32), ("pairs_fp64", pbs.PB_KERNEL_PAIRS_FP64),
                      ("source", pbs.PB_KERNEL_SOURCE), ("charge", pbs.PB_KERNEL_CHARGE)):
        n_l, ms_l, pr_l = ctx.profile_read(kid)
        if n_l:
            kernel_rows[name] = {"launches": n_l, "avg_ms": ms_l / n_l,
                                 "gpairs_per_s": pr_l / (ms_l * 1e-3) / 1e9}

    # the same solve through the host-array entry point (surface and charges
    # copied in, phi/dphi copied out over PCIe): reported beside `value`,
    # which stays the device-resident rate
    ctx.pb_solve(w.verts, w.tris, w.pos, w.q, params)
    host_s = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        ctx.pb_solve(w.verts, w.tris, w.pos, w.q, params)
        host_s.append(time.perf_counter() - ts)
    _log(f"bench: host-array solves: median {1e3 * float(np.median(host_s)):.2f} ms")

    compare = {}
    if not args.no_fp64_compare:
        variants = [("fp64_same_preconditioner", PB_FP64, leaf),
                    ("fp32_ir_no_preconditioner", PB_FP32_IR, 0),
                    ("fp64_no_preconditioner", PB_FP64, 0)]
        for name, pr, lf in variants:
            if pr == prec and lf == leaf:
                continue
            pv, _e = pick(pr, lf)
            compare[name] = timed_once(pv)

    out = {
        "metric": "BIE matvec G-pair-interactions/s; time to E_solv at 1e-6 rel. error",
        "value": value,
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
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
            "precond_leaf": leaf,
            "tol": params.tol,
            "inner_tol": params.inner_tol if prec == PB_FP32_IR else None,
            "gmres_restart": 10,
            "fp32_sweep": {"kind": sweep_label(tuned[0]), "target_waves": tuned[1]},
        },
        "time_to_solution_s": ms_step / 1e3,
        "time_to_solution_median_s": float(np.median(step_s)),
        "time_to_solution_host_arrays_median_s": float(np.median(host_s)),
        "step_s": [round(t, 6) for t in step_s],
        "e_solv": infos[-1].e_solv,
        "e_rel_err": max(errs),
        "iters": infos[-1].iters,
        "matvecs_fp32": infos[-1].matvecs_fp32,
        "matvecs_fp64": infos[-1].matvecs_fp64,
        "refinements": infos[-1].refinements,
        "kernels": kernel_rows,
        "compare": compare,
        "roofline": {
            "bound": "alu",
            "kernel": (fp32_kernel_name(tuned[0]) if prec == PB_FP32_IR
                       else fp64_kernel_name(ctx.get_fp64_sweep())),
            "achieved": achieved / 1e12,
            "peak": peak / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": (measured_traffic(N, tuned) if prec == PB_FP32_IR else None),
            "traffic_unit": "bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
            "flop_per_pair": FLOP_PER_PAIR,
            "pairs_per_launch": kpairs / max(launches, 1),
            "avg_launch_ms": avg_ms,
            "launches": launches,
        },
        "cpu_baseline": None,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        _log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
