"""mhdpic_advance_noalloc (static device scratch, no allocation) against
mhdpic_advance (caller workspace) through the C ABI: deposits and states equal
bit for bit, on two calls in a row, the second with a smaller input."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1412_1087_amd import workloads as W  # noqa: E402

from gpu_helpers import gpu_box, to_dev  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(wl, n_steps, noalloc, precision=0, n_sub=1):
    from paper_1412_1087_amd import mhdpic as M
    out = M.advance([gpu_box(wl.box)], [wl.N], to_dev(wl.x), to_dev(wl.v), to_dev(wl.m),
                    to_dev(wl.qm), to_dev(wl.B), to_dev(wl.vg), to_dev(wl.rho), [wl.dt], n_steps,
                    n_sub=n_sub, precision=precision, noalloc=noalloc)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def test_noalloc_equals_workspace_entry_point_on_two_calls():
    _need_gpu()
    big = W.bell3d(n=(20, 12, 10), ppc=4, seed=90, dx=(0.5, 2.0, 1.25), x0=(-3.7, 11.2, 0.5))
    small = W.gyro2d(nx=13, ny=9, ppc=3, seed=91)
    for wl, n_steps in ((big, 3), (small, 2)):
        ref = _run(wl, n_steps, noalloc=False)
        got = _run(wl, n_steps, noalloc=True)
        for name, a, b in zip(("x", "v", "deposits"), got, ref):
            assert a.shape == b.shape and (a == b).all(), (wl.name, name)


def test_noalloc_precision_form_and_subcycling():
    _need_gpu()
    wl = W.bell3d(n=(12, 10, 8), ppc=3, seed=92)
    for prec, n_sub in ((1, 1), (0, 3)):
        ref = _run(wl, 2, noalloc=False, precision=prec, n_sub=n_sub)
        got = _run(wl, 2, noalloc=True, precision=prec, n_sub=n_sub)
        for a, b in zip(got, ref):
            assert (a == b).all()


def test_noalloc_rejects_inputs_beyond_the_scratch():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    # 128^3 cells need about 0.3 GB of workspace: refused before any device work
    box = M.Box(ndim=3, n=(128, 128, 128), C=20.0)
    N = 4
    z = torch.zeros((3, N), dtype=torch.float64, device="cuda")
    one = torch.ones(N, dtype=torch.float64, device="cuda")
    Bz = torch.zeros((3, 128 ** 3), dtype=torch.float64, device="cuda")
    with pytest.raises(M.MhdpicError) as e:
        M.advance([box], [N], z, z, one, one, Bz, Bz, None, 0.01, 1, noalloc=True)
    assert e.value.code == M.ENOMEM
    assert "static scratch" in str(e.value)
