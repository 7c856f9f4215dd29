"""Per-phase event timing through the C ABI: only the selected phases are
timed, and a bad mask is rejected."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1412_1087_amd import workloads as W  # noqa: E402
from paper_1412_1087_amd.mhdpic import MhdpicError  # noqa: E402

from gpu_helpers import DeviceRun  # noqa: E402


def test_timing_selects_phases():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_1087_amd import mhdpic as M
    g = DeviceRun(W.gyro2d(nx=16, ny=16, ppc=4, seed=40))
    ctx = g.ctx
    ctx.timing(True, phases=("push",))
    g.step(3)
    torch.cuda.synchronize()
    ctx.timing(False)
    t = ctx.timing_read()
    assert t["push"][1] == 3 and t["push"][0] > 0.0
    assert t["bin"][1] == 0 and t["fieldprep"][1] == 0 and t["clear"][1] == 0
    ctx.timing(True)
    g.step(2)
    torch.cuda.synchronize()
    ctx.timing(False)
    t = ctx.timing_read()
    assert t["push"][1] == 2 and t["fieldprep"][1] == 2
    assert t["clear"][1] == 0  # the field preparation clears the next n, J buffer
    assert t["bin"][1] == 2  # the call's re-binning and one between its two steps
    g.step(1)
    assert ctx.timing_read()["push"][1] == 0  # off again
    for bad in (-1, 16):
        with pytest.raises(MhdpicError):
            M._check(M.lib().mhdpic_timing_enable(ctx._h, bad))
    g.ctx.check()
