"""Accuracy of the FP64 functions of the pair sweeps (exp(-kappa r) and the
refined 1/sqrt(r^2) of paper_2312_10044_amd/csrc/pb_fp64math.h), on the CPU.

The header uses only fused multiply-add, round-to-nearest-even and scaling by
a power of two, which round identically on the host and on gfx950, so a host
build measures exactly the values the FP64 sweeps compute.  References are
long-double expl and 1/sqrtl (64-bit significands).  The rsqrt refinement is
fed seeds perturbed by up to 2^-22 relative, twice the documented error bound
of the hardware estimate it refines on the GPU.
"""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "fp64math_check.cpp")
INC = os.path.join(ROOT, "paper_2312_10044_amd", "csrc")


def _run(tmp_path):
    exe = os.path.join(str(tmp_path), "fp64math_check")
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-Wall", "-Wextra", "-Werror",
           "-I", INC, SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, check=True).stdout
    vals = {}
    for line in out.splitlines():
        k, v = line.split()
        vals[k] = float(v)
    return vals


def test_exp_and_rsqrt_accuracy(tmp_path):
    v = _run(tmp_path)
    print(v)
    # exp(-x): 8 million arguments on [0, 708]
    assert v["exp_count"] >= 8e6
    assert v["exp_max_ulp"] <= 1.35
    assert v["exp_mean_ulp"] <= 0.35
    assert v["exp_at_zero"] == 1.0
    # the 256 table entries 2^(j/256) are correctly rounded
    assert v["table_max_ulp"] <= 0.5
    # beyond the normal range: subnormal or zero, never negative, NaN or inf
    assert v["exp_tail_bad"] == 0
    assert v["exp_tail_max_abs_in_min_subnormals"] <= 2.0
    assert v["exp_beyond_745"] == 0.0
    assert v["exp_at_max_arg"] == 0.0   # kappa r at its largest accepted value
    # 1/sqrt(x) from a seed with relative error up to 2^-22
    assert v["rsqrt_count"] >= 6e6
    assert v["rsqrt_max_ulp"] <= 1.0
