"""The FP64 pair functions on the device (pb_eval_pair_math): exp(-x) and
1/sqrt(y) as the FP64 pair sweeps evaluate them for the screened Coulomb
kernel (Sec. 2.2.1, eq. eq_potential).

* exp(-x) on the device equals, bit for bit, a host build of the same header
  (tests/c/fp64math_shim.cpp, g++ with contraction off): the header uses only
  operations that round identically on both, which is what lets the host test
  (test_fp64math_host.py) measure the device's accuracy.  It is also checked
  directly against long-double exp: within 1.35 ulp on [0, 708]; subnormal
  or 0 up to 745.2; exactly 0 from there to the accepted maximum, through the
  range of the sweeps' padding points (kappa r up to 3.5e8), where the
  reduction's integer conversion saturates.
* 1/sqrt(y) (the hardware estimate refined once) is within 1 ulp of
  long-double 1/sqrt over the whole accepted range, log-uniform.
* Arguments outside the documented ranges, and sizes above the limit, are
  rejected and nothing is written.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIM = os.path.join(ROOT, "tests", "c", "fp64math_shim.cpp")
INC = os.path.join(ROOT, "paper_2312_10044_amd", "csrc")


def _host_exp(tmp_path, x):
    so = os.path.join(str(tmp_path), "libfp64shim.so")
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC",
                        "-I", INC, SHIM, "-o", so], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lib = ctypes.CDLL(so)
    lib.host_exp_neg_pair.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    lib.host_exp_neg_pair.restype = None
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib.host_exp_neg_pair(x.size, x.ctypes.data, out.ctypes.data)
    return out


def _ulp_err(got, ref_ld):
    ref = ref_ld.astype(np.float64)
    return np.abs(got.astype(np.longdouble) - ref_ld) / np.spacing(np.abs(ref)).astype(np.longdouble)


def _args():
    rng = np.random.default_rng(20231215)
    x = np.concatenate([
        np.linspace(0.0, 708.0, 1_000_001),
        rng.uniform(0.0, 0.5, 500_000),           # near pairs
        rng.uniform(0.0, 708.0, 500_000),
        np.linspace(708.0, 746.0, 20_001),        # subnormal tail and the underflow to 0
        np.exp(rng.uniform(np.log(746.0), np.log(1e12), 20_000)),
        [0.0, 5e-324, 1e-300, 1e-17, 745.13, 745.2, 1e3, 5.79e6, 5.8e6, 1e7, 3.5e8, 1e12],
    ])
    y = np.exp(rng.uniform(np.log(1e-30), np.log(1e30), x.size))
    y[:8] = [1e-30, 1e-10, 0.25, 1.0, 2.0, 4.0, 1e13, 1e30]
    return x, y


def test_device_exp_matches_host_build_and_bounds(tmp_path):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_10044_amd as m
    x, y = _args()
    print(f"pb_eval_pair_math on {x.size} arguments", flush=True)
    with m.Context(0) as ctx:
        ex, rq = ctx.eval_pair_math(x, y)
    assert np.all(np.isfinite(ex)) and np.all(ex >= 0.0)

    # bit-identical to the host build wherever the reduction's integer is exact
    host = _host_exp(tmp_path, x)
    exact = x < 5.8e6
    diff = np.flatnonzero(ex[exact].view(np.int64) != host[exact].view(np.int64))
    print(f"exp: {diff.size} of {int(exact.sum())} differ from the host build", flush=True)
    assert diff.size == 0, (x[exact][diff[:5]], ex[exact][diff[:5]], host[exact][diff[:5]])

    # against long-double exp
    xl = x.astype(np.longdouble)
    ref = np.exp(-xl)
    normal = x <= 708.0
    err = _ulp_err(ex[normal], ref[normal])
    print(f"exp: max {float(err.max()):.4f} ulp, mean {float(err.mean()):.4f} ulp on [0, 708]",
          flush=True)
    assert float(err.max()) <= 1.35
    tail = (x > 708.0) & (x <= 745.2)
    tiny = np.float64(5e-324)
    assert np.all(np.abs(ex[tail].astype(np.longdouble) - ref[tail]) <= 2 * tiny)
    assert np.all(ex[x > 745.2] == 0.0)
    assert ex[x == 0.0][0] == 1.0

    # 1/sqrt(y) against long double
    rref = 1.0 / np.sqrt(y.astype(np.longdouble))
    rerr = _ulp_err(rq, rref)
    print(f"rsqrt: max {float(rerr.max()):.4f} ulp over [1e-30, 1e30]", flush=True)
    assert float(rerr.max()) <= 1.0


def test_arguments_outside_the_ranges_are_rejected():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_10044_amd as m
    from paper_2312_10044_amd import pbsolve as pbs
    with m.Context(0) as ctx:
        e0, r0 = ctx.eval_pair_math(np.array([]), np.array([]))
        assert e0.size == 0 and r0.size == 0
        for xb, yb in ((-1e-300, 1.0), (np.nan, 1.0), (2 * pbs.PB_PAIR_MATH_XMAX, 1.0),
                       (1.0, 0.0), (1.0, np.inf), (1.0, 1e-31), (1.0, 1e31)):
            with pytest.raises(m.PbError) as e:
                ctx.eval_pair_math(np.array([0.5, xb]), np.array([1.0, yb]))
            assert e.value.status == m.PB_ERR_ARG
        # one more than the size limit: rejected before anything is copied
        big = pbs.PB_PAIR_MATH_MAX + 1
        with pytest.raises(m.PbError) as e:
            ctx.eval_pair_math(np.zeros(big), np.ones(big))
        assert e.value.status == m.PB_ERR_ARG
        # the context stays usable
        ex, rq = ctx.eval_pair_math(np.array([0.0, 1.0]), np.array([1.0, 4.0]))
        assert ex[0] == 1.0
        assert np.all(np.abs(rq - [1.0, 0.5]) <= np.spacing([1.0, 0.5]))
