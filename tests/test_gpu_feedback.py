"""GPU parity of the cell-centred predictor feedback (mhdpic_feedback): the
ten channels from the current n_CR, J_CR against the oracle's, bit for bit
(the same IEEE operations in the same order on both sides)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from paper_1412_1087_amd import workloads as W  # noqa: E402

from gpu_helpers import DeviceRun, oracle_box, oracle_run  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("which", ["bell3d_hall", "gyro2d"])
def test_feedback_matches_oracle_bitwise(which):
    _need_gpu()
    if which == "bell3d_hall":
        wl = W.bell3d(n=(12, 10, 9), ppc=4, seed=1300, hall=1)
    else:
        wl = W.gyro2d(nx=24, ny=20, ppc=5, seed=1301)
    g = DeviceRun(wl)
    o = oracle_run(wl)
    for k in range(2):
        out_g = g.ctx.feedback(g.B, g.vg, g.rho).cpu().numpy()
        out_o = o.feedback(wl.B, wl.vg, wl.rho)
        for ch in range(10):
            bad = np.nonzero(out_g[ch].view(np.int64) != out_o[ch].view(np.int64))[0]
            assert len(bad) == 0, f"step {k}: channel {ch} differs in {len(bad)} cells"
        g.step(1)
        o.step(wl.B, wl.vg, wl.rho, wl.dt, 1)


def test_feedback_of_boxes_with_and_without_hall():
    _need_gpu()
    wa = W.gyro2d(nx=16, ny=18, ppc=3, seed=1310)
    wb = W.gyro2d(nx=20, ny=16, ppc=4, seed=1311)
    wb.box.hall = 1
    g = DeviceRun([wa, wb])
    out = g.ctx.feedback(g.B, g.vg, g.rho).cpu().numpy()
    for b, w in enumerate([wa, wb]):
        sl = slice(g.cell_off[b], g.cell_off[b + 1])
        o = oracle_run(w)                      # the oracle's own initial n_CR, J_CR
        want = O.feedback(oracle_box(w.box), w.B, w.vg, w.rho, o.D)
        assert (out[:, sl] == want).all(), b
    sla = slice(g.cell_off[0], g.cell_off[1])
    assert (out[4:7, sla] == 0).all()
