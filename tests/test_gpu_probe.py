"""The counter-calibration probe (pb_probe_valu): every kind runs and reports
its exact operation count; an unknown kind is rejected and the context stays
usable.  The counts are what rocprofv3's VALU counters are checked against."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_kinds_and_counts():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_10044_amd as m
    from paper_2312_10044_amd import pbsolve as pbs
    with m.Context(0) as ctx:
        for kind in (pbs.PB_PROBE_FMA_F32, pbs.PB_PROBE_FMA_F64, pbs.PB_PROBE_EXP_F32):
            n = ctx.probe_valu(kind)
            print(f"probe kind {kind}: {n} lane operations", flush=True)
            assert n == 1024 * 256 * 8 * 1024
        with pytest.raises(m.PbError) as e:
            ctx.probe_valu(3)
        assert e.value.status == m.PB_ERR_ARG
        assert ctx.probe_valu(pbs.PB_PROBE_FMA_F32) == 2 ** 31
