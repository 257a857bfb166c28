"""The committed rocprofv3 counter record that bench.py's roofline reads
(profiles/<kernel>_<workload>_counters.json), on the CPU.

* Its derived fields follow from its raw counters: the byte factors are the
  1 GiB device copy's bytes over what FETCH_SIZE and WRITE_SIZE read for it,
  the bytes per launch are the calibrated sum of the sweep's two counters, and
  the FLOPs per launch are SQ_INSTS_VALU_FLOPS_FP32 (FLOPs per wave
  instruction) times the 64 lanes of a wave.
* bench.counter_record hands the record out only for the kernel source and
  launch shape it was taken on (digest, sweep kind, target waves), so a stale
  record can never reach the bench line.
* The digest follows the code, not its comments or layout.
"""
import glob
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORDS = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_counters.json")))


def _fp32_records():
    out = []
    for path in RECORDS:
        rec = json.load(open(path))
        if "sweep_kind" in rec and "fetch_size_kib" in rec:
            out.append((path, rec))
    return out


def test_there_is_a_record_for_the_headline_workload():
    names = [os.path.basename(p) for p, _ in _fp32_records()]
    assert "k_pairs_f32_sym_star327680_counters.json" in names


@pytest.mark.parametrize("path,rec", _fp32_records(), ids=lambda v: os.path.basename(v)
                         if isinstance(v, str) else "")
def test_record_arithmetic(path, rec):
    KiB = 1024.0
    ff = rec["copy_bytes_each_way"] / (rec["copy_fetch_size_kib"] * KiB)
    wf = rec["copy_bytes_each_way"] / (rec["copy_write_size_kib"] * KiB)
    assert rec["fetch_factor"] == pytest.approx(ff, rel=1e-12)
    assert rec["write_factor"] == pytest.approx(wf, rel=1e-12)
    # a device copy reads each byte once through the counted path: the factors
    # are near 2 (FETCH_SIZE counts half) and 1 on this hardware
    assert 1.5 < ff < 2.5 and 0.8 < wf < 1.2
    b = (rec["fetch_size_kib"] * ff + rec["write_size_kib"] * wf) * KiB
    assert rec["bytes_per_launch"] == pytest.approx(b, rel=1e-12)
    assert rec["valu_flop_per_launch"] == pytest.approx(64.0 * rec["sq_insts_valu_flops_fp32"],
                                                        rel=1e-12)
    # the counted FLOPs per ordered pair lie below the algorithmic 58 (pairs
    # share work between their two directions) and above a third of it
    n = rec["n_tri"]
    per_pair = rec["valu_flop_per_launch"] / (float(n) * (n - 1))
    assert 58.0 / 3 < per_pair < 58.0
    assert len(rec["kernel_digest"]) == 64
    assert all("rocprofv3" in c and "--pmc" in c for c in rec["commands"])


def test_counter_record_only_for_its_own_kernel_and_launch_shape():
    import bench
    for path, rec in _fp32_records():
        workload = os.path.basename(path)[len(bench.fp32_kernel_name(rec["sweep_kind"])) + 1:
                                          -len("_counters.json")]
        shape = (rec["sweep_kind"], rec["target_waves"])
        got = bench.counter_record(workload, shape)
        if bench.kernel_digest(rec["sweep_kind"]) == rec["kernel_digest"]:
            assert got == rec
        else:
            assert got is None
        assert bench.counter_record(workload, (rec["sweep_kind"], rec["target_waves"] * 2)) is None
        assert bench.counter_record("no_such_workload", shape) is None


def test_digest_ignores_comments_and_layout():
    import bench
    a = "int f(int x)\n{\n    return x + 1;   // one more\n}\n"
    b = "int f(int x) { /* the successor */\n  return x + 1; }"
    c = "int f(int x) { return x + 2; }"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)
