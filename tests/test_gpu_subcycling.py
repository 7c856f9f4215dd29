"""GPU parity of particle sub-cycling (mhdpic_step_sub) against the oracle.

Each step forms E once and moves the particles n_sub times by dt/n_sub;
-dM, -dE_k accumulate every sub-step and n_CR, J_CR are deposited after the
last.  Deposits must be bit-identical to the oracle's; particle states are
identical too, like the plain step's.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1412_1087_amd import workloads as W  # noqa: E402

from gpu_helpers import DeviceRun, assert_states_exact, oracle_run  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _compare(wl, g, o, tag):
    (D,) = g.deposits()
    for ch in range(8):
        bad = np.nonzero(D[ch] != o.D[ch])[0]
        assert len(bad) == 0, f"{tag}: channel {ch} differs in {len(bad)} cells"
    ((x, v),) = g.particles()
    assert_states_exact(x, v, o.positions(), o.v, tag)


@pytest.mark.parametrize("n_sub", [2, 5])
def test_subcycled_2d_matches_oracle(n_sub):
    _need_gpu()
    wl = W.gyro2d(nx=40, ny=36, ppc=6, seed=1200 + n_sub)   # tiles of 32x16 plus ragged edges
    g = DeviceRun(wl)
    o = oracle_run(wl)
    for rep in range(2):
        g.step(2, n_sub=n_sub)
        o.step(wl.B, wl.vg, wl.rho, wl.dt, 2, n_sub=n_sub)
        _compare(wl, g, o, f"call {rep}")
    g.ctx.check()


@pytest.mark.parametrize("hall", [0, 1])
def test_subcycled_3d_matches_oracle(hall):
    _need_gpu()
    wl = W.bell3d(n=(17, 9, 13), ppc=5, seed=1210 + hall, hall=hall)
    g = DeviceRun(wl)
    o = oracle_run(wl)
    g.step(2, n_sub=3)
    o.step(wl.B, wl.vg, wl.rho, wl.dt, 2, n_sub=3)
    _compare(wl, g, o, "n_sub 3")
    # switching back to single steps re-bins for the new particle step
    g.step(1)
    o.step(wl.B, wl.vg, wl.rho, wl.dt, 1)
    _compare(wl, g, o, "n_sub 1 after 3")
    g.ctx.check()


def test_subcycled_step_checks_its_arguments():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    wl = W.gyro2d(nx=16, ny=16, ppc=2, seed=1220)
    g = DeviceRun(wl)
    with pytest.raises(M.MhdpicError):
        g.step(1, n_sub=0)
    big = 2.5 * 0.98 * wl.box.max_move_cells * wl.box.dx[0] / wl.box.C
    with pytest.raises(M.MhdpicError):
        g.step(1, dts=[big])
    o = oracle_run(wl)
    g.step(1, dts=[big], n_sub=3)      # over the limit as one step, within it as three
    o.step(wl.B, wl.vg, wl.rho, big, 1, n_sub=3)
    _compare(wl, g, o, "large dt in 3 sub-steps")


def test_subcycled_precision_form_equals_its_plain_substeps():
    """Without the Hall term the field does not depend on n_CR, J_CR, so a
    sub-cycled step of the precision form equals its own plain steps of
    dt/n_sub bit for bit (the same kernels on the same binary32 states)."""
    _need_gpu()
    wl = W.gyro2d(nx=36, ny=20, ppc=6, seed=1230)
    a = DeviceRun(wl, precision=1)
    b = DeviceRun(wl, precision=1)
    a.step(2, n_sub=3)
    for _ in range(6):
        b.step(1, dts=[wl.dt / 3])
    (Da,) = a.deposits()
    (Db,) = b.deposits()
    assert (Da == Db).all()
    ((xa, va),) = a.particles()
    ((xb, vb),) = b.particles()
    assert (va == vb).all() and (xa == xb).all()


def test_subcycled_multi_box_context_equals_single_boxes():
    _need_gpu()
    wls = [W.gyro2d(nx=20 + 6 * k, ny=18, ppc=3 + k, seed=1240 + k) for k in range(3)]
    wls[1].box.hall = 1
    many = DeviceRun(wls)
    many.step(2, n_sub=4)
    Dm = many.deposits()
    Pm = many.particles()
    for k, w in enumerate(wls):
        one = DeviceRun(w)
        one.step(2, n_sub=4)
        (D1,) = one.deposits()
        ((x1, v1),) = one.particles()
        assert (Dm[k] == D1).all(), k
        assert (Pm[k][1] == v1).all(), k
