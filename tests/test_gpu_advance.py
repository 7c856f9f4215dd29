"""mhdpic_advance (one call without a context) against the oracle, bit for
bit, and against the context path on the same workspace layout."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1412_1087_amd import workloads as W  # noqa: E402

from gpu_helpers import DeviceRun, assert_states_exact, gpu_box, oracle_run, to_dev  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cat(wls, f):
    return np.concatenate([f(w) for w in wls], axis=-1)


def _advance(wls, n_steps, n_sub=1, precision=0):
    from paper_1412_1087_amd import mhdpic as M
    boxes = [gpu_box(w.box) for w in wls]
    out = M.advance(boxes, [w.N for w in wls], to_dev(_cat(wls, lambda w: w.x)),
                    to_dev(_cat(wls, lambda w: w.v)), to_dev(_cat(wls, lambda w: w.m)),
                    to_dev(_cat(wls, lambda w: w.qm)), to_dev(_cat(wls, lambda w: w.B)),
                    to_dev(_cat(wls, lambda w: w.vg)), to_dev(_cat(wls, lambda w: w.rho)),
                    [w.dt for w in wls], n_steps, n_sub=n_sub, precision=precision)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


@pytest.mark.parametrize("make,n_steps,n_sub", [
    (lambda: W.gyro2d(nx=37, ny=23, ppc=5, seed=60, dx=(0.5, 2.0, 1.0), x0=(-3.7, 11.2, 0.0)), 3, 1),
    (lambda: W.bell3d(n=(13, 9, 7), ppc=3, seed=61, dx=(0.5, 2.0, 1.25), x0=(-3.7, 11.2, 0.5)), 2, 1),
    (lambda: W.bell3d(n=(10, 8, 6), ppc=4, seed=62), 2, 3),
    (lambda: W.gyro2d(nx=16, ny=16, ppc=4, seed=63), 0, 1),
])
def test_advance_matches_oracle(make, n_steps, n_sub):
    _need_gpu()
    wl = make()
    x, v, D = _advance([wl], n_steps, n_sub)
    o = oracle_run(wl)
    if n_steps:
        o.step(wl.B, wl.vg, wl.rho, wl.dt, n_steps, n_sub=n_sub)
    assert (D == o.D).all()
    assert_states_exact(x, v, o.positions(), o.v, "advance")


def test_advance_multi_box_matches_context_path():
    _need_gpu()
    wls = [W.gyro2d(nx=17, ny=40, ppc=3, seed=64), W.gyro2d(nx=8, ny=8, ppc=11, seed=65,
                                                           dx=(3.0, 0.75, 1.0), x0=(1.5, -2.0, 0.0))]
    x, v, D = _advance(wls, 4)
    g = DeviceRun(wls)
    g.step(4)
    Dg = np.concatenate(g.deposits(), axis=1)
    xg = np.concatenate([p[0] for p in g.particles()], axis=1)
    vg = np.concatenate([p[1] for p in g.particles()], axis=1)
    assert (D == Dg).all()
    assert (x == xg).all() and (v == vg).all()


def test_advance_precision_form_matches_context_path():
    _need_gpu()
    wl = W.bell3d(n=(12, 10, 8), ppc=3, seed=66)
    x, v, D = _advance([wl], 3, precision=1)
    g = DeviceRun(wl, precision=1)
    g.step(3)
    ((xg, vg),) = g.particles()
    (Dg,) = g.deposits()
    assert (D == Dg).all()
    assert (x == xg).all() and (v == vg).all()


def test_advance_reports_device_errors():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    wl = W.gyro2d(nx=8, ny=8, ppc=1, seed=67)
    wl.m = wl.m.copy()
    wl.m[3] = 1e5  # (q/mc) m 2^40 > 2^51
    with pytest.raises(M.MhdpicError) as e:
        _advance([wl], 1)
    assert e.value.code == M.ERANGE
