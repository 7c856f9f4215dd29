"""Edge cases against the oracle, bit for bit: the method's degenerate inputs
and the largest grid extents the library's cell index can hold."""
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
        assert (D[ch] == o.D[ch]).all(), f"{tag}: channel {ch}"
    ((x, v),) = g.particles()
    assert_states_exact(x, v, o.positions(), o.v, tag)


@pytest.mark.parametrize("ndim", [2, 3])
def test_degenerate_fields_and_particles(ndim):
    """B = 0 (no E-parallel removal), v_g = 0 (E0 = 0), cells without CRs
    (R = 0 in the Hall term), particles at rest, massless particles, offsets
    exactly on a cell boundary, and positions just below the upper box edge."""
    _need_gpu()
    if ndim == 2:
        wl = W.gyro2d(nx=40, ny=24, ppc=3, seed=1400)
    else:
        wl = W.bell3d(n=(20, 12, 12), ppc=2, seed=1401)
    wl.box.hall = 1
    nx, ny = wl.box.n[0], wl.box.n[1]
    cx = np.arange(wl.box.n_cells) % nx
    wl.B = wl.B.copy()
    wl.vg = wl.vg.copy()
    wl.B[:, (cx >= 4) & (cx < 9)] = 0.0          # field-free slab
    wl.vg[:, (cx >= 12) & (cx < 16)] = 0.0       # gas at rest
    x, v, m = wl.x.copy(), wl.v.copy(), wl.m.copy()
    rng = np.random.default_rng(1402)
    k = 40
    v[:, :k] = 0.0                                # at rest
    m[k:2 * k] = 0.0                              # no mass: nothing to deposit
    on = slice(2 * k, 3 * k)                      # exactly on cell boundaries
    for d in range(ndim):
        x[d, on] = rng.integers(0, wl.box.n[d], size=k) * wl.box.dx[d]
    edge = slice(3 * k, 4 * k)                    # just below the upper edge
    x[0, edge] = nx * wl.box.dx[0] * (1.0 - 1e-12)
    x[1, edge] = ny * wl.box.dx[1] * (1.0 - 1e-12)
    # CRs only in the left half: the right half has n_CR = 0
    far = x[0] > 0.75 * nx * wl.box.dx[0]
    x[0, far] -= 0.5 * nx * wl.box.dx[0]
    wl.x, wl.v, wl.m = x, v, m
    g = DeviceRun(wl)
    o = oracle_run(wl)
    (D0,) = g.deposits()
    assert (D0 == o.D).all(), "initial deposit"
    for rep in range(3):
        g.step(1)
        o.step(wl.B, wl.vg, wl.rho, wl.dt, 1)
        _compare(wl, g, o, f"step {rep}")
    g.ctx.check()


@pytest.mark.parametrize("shape", [(65536, 2, 1), (2048, 4, 4), (4, 2048, 4), (4, 4, 1024)])
def test_largest_grid_extents(shape):
    """The cell index packs 16 + 16 bits in 2D and 11 + 11 + 10 bits in 3D:
    boxes at those extents, with particles up to the last cell."""
    _need_gpu()
    if shape[2] == 1:
        wl = W.gyro2d(nx=shape[0], ny=shape[1], ppc=1, seed=1410)
    else:
        wl = W.bell3d(n=shape, ppc=1, seed=1411, hall=0)
    # a few particles in the last cells of every dimension
    x = wl.x.copy()
    nd = wl.box.ndim
    for d in range(nd):
        x[d, :16] = (wl.box.n[d] - 0.5 - 0.3 * np.arange(16) / 16.0) * wl.box.dx[d]
    wl.x = x
    g = DeviceRun(wl)
    o = oracle_run(wl)
    for rep in range(2):
        g.step(1)
        o.step(wl.B, wl.vg, wl.rho, wl.dt, 1)
        _compare(wl, g, o, f"step {rep}")
