"""Full-size checks, in the launch configuration the benchmark times (default
tiles, one step from the initial state).

The oracle cannot step millions of particles within a test, so it checks
samples it can compute exactly:
  * cells: every particle that can reach a sampled cell in one step (its
    initial cell within 4 cells, periodically) is stepped by the oracle, so the
    oracle's deposits at the sampled cells are complete and must equal the
    GPU's bit for bit;
  * particles: the states of all those particles against the GPU's;
  * with the Hall term, E at a cell depends on n_CR, J_CR of that cell only, so
    the n_CR, J_CR the stepped particles see (cells within 5 of a sampled cell)
    come from an oracle initialisation of every particle within 7 cells.
The precision form and the batched form are checked on properties that hold
at any size, and on sampled boxes.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from paper_1412_1087_amd import workloads as W  # noqa: E402

from gpu_helpers import DeviceRun, assert_states_exact, oracle_box, oracle_run  # noqa: E402

EPS32 = 2.0 ** -24


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cells_of(wl):
    nd = wl.box.ndim
    return np.stack([np.floor((wl.x[d] - wl.box.x0[d]) / wl.box.dx[d]).astype(np.int64) % wl.box.n[d]
                     for d in range(nd)])


def _near(ci, n, cells, r):
    """Particles whose cell is within r cells (periodic, per dimension) of any
    of the given cells."""
    keep = np.zeros(ci.shape[1], dtype=bool)
    for c in cells:
        ok = np.ones(ci.shape[1], dtype=bool)
        for d in range(ci.shape[0]):
            dd = np.abs(ci[d] - c[d])
            dd = np.minimum(dd, n[d] - dd)
            ok &= dd <= r
        keep |= ok
    return np.flatnonzero(keep)


def _flat(c, n):
    return c[0] + n[0] * (c[1] + n[1] * (c[2] if len(c) > 2 else 0))


def _sampled_cell_parity(wl, cells):
    nd = wl.box.ndim
    n = wl.box.n
    g = DeviceRun(wl)
    (D0,) = g.deposits()
    g.step(1)
    (D1,) = g.deposits()
    ((xg, vg),) = g.particles()
    g.ctx.check()
    del g
    torch.cuda.empty_cache()

    ci = _cells_of(wl)
    box = oracle_box(wl.box)
    step_idx = _near(ci, n, cells, 4)
    sub = O.System(box, wl.x[:, step_idx], wl.v[:, step_idx], wl.m[step_idx], wl.qm[step_idx])
    if wl.box.hall:
        init_idx = _near(ci, n, cells, 7)
        full = O.System(box, wl.x[:, init_idx], wl.v[:, init_idx], wl.m[init_idx], wl.qm[init_idx])
        # n_CR, J_CR are complete within 6 cells of the sampled cells
        ring = np.array([_flat(c, n) for c in _cells_within(cells, n, nd, 5)])
        assert (D0[:4, ring] == full.D[:4, ring]).all(), "initial n_CR, J_CR differ"
        sub.D[:4] = full.D[:4]
    sub.step(wl.B, wl.vg, wl.rho, wl.dt, 1)
    flat = np.array([_flat(c, n) for c in cells])
    for ch in range(8):
        assert (D1[ch, flat] == sub.D[ch, flat]).all(), f"channel {ch} at sampled cells"
    assert_states_exact(xg[:, step_idx], vg[:, step_idx], sub.positions(), sub.v, "sampled particles")
    return len(step_idx)


def _cells_within(cells, n, nd, r):
    out = set()
    rng = range(-r, r + 1)
    for c in cells:
        for ox in rng:
            for oy in rng:
                for oz in (rng if nd == 3 else [0]):
                    out.add(((c[0] + ox) % n[0], (c[1] + oy) % n[1], (c[2] + oz) % n[2] if nd == 3 else 0))
    return sorted(out)


def test_full_size_beam_box_sampled_cells_and_particles():
    """64^3 cells, 16 per cell, Hall term on: the headline configuration."""
    _need_gpu()
    wl = W.bell3d()
    rng = np.random.default_rng(71)
    cells = [(0, 0, 0), (63, 63, 63), (7, 3, 3), (8, 4, 4), (31, 0, 63)]
    cells += [tuple(int(a) for a in rng.integers(0, 64, size=3)) for _ in range(3)]
    assert _sampled_cell_parity(wl, cells) > 50_000


def test_full_size_strip_sampled_cells_and_particles():
    """8192 x 32 cells, 16.8M particles, 80 % in the band around x = 0.3 L."""
    _need_gpu()
    wl = W.shock2d()
    cells = [(2458, 0, 0), (2457, 31, 0), (2470, 16, 0), (2600, 5, 0),   # band
             (0, 0, 0), (8191, 31, 0), (100, 17, 0), (6000, 8, 0)]
    assert _sampled_cell_parity(wl, cells) > 100_000


def test_full_size_batched_graph_sampled_boxes():
    """256 boxes in one context, two steps as one HIP graph launch: sampled
    boxes against the oracle (binary64) and the precision form of each sampled
    box against the same box run alone."""
    _need_gpu()
    wls = W.batch2d(n_boxes=256, seed0=5000)
    sizes = np.array([w.N for w in wls])
    pick = sorted({int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), 3, 77, 200})
    stream = torch.cuda.Stream()
    dts = [w.dt for w in wls]
    g = DeviceRun(wls)
    with torch.cuda.stream(stream):
        g.ctx.step_graph(g.B, g.vg, g.rho, dts, 2, stream)
    stream.synchronize()
    torch.cuda.synchronize()
    D = g.deposits()
    P = g.particles()
    g.ctx.check()
    for b in pick:
        o = oracle_run(wls[b])
        o.step(wls[b].B, wls[b].vg, wls[b].rho, wls[b].dt, 2)
        assert (D[b] == o.D).all(), f"box {b}"
        assert_states_exact(P[b][0], P[b][1], o.positions(), o.v, f"box {b}")
    del g
    torch.cuda.empty_cache()
    g32 = DeviceRun(wls, precision=1)
    with torch.cuda.stream(stream):
        g32.ctx.step_graph(g32.B, g32.vg, g32.rho, dts, 2, stream)
    stream.synchronize()
    torch.cuda.synchronize()
    D32 = g32.deposits()
    P32 = g32.particles()
    for b in pick:
        s = DeviceRun(wls[b], precision=1)
        s.step(2)
        (Ds,) = s.deposits()
        ((xs, vs),) = s.particles()
        assert (D32[b] == Ds).all(), f"box {b}"
        assert (P32[b][1] == vs).all(), f"box {b}"


def test_full_size_precision_form_properties():
    """128^3 cells, 32 per cell, one step of the precision form against the
    binary64 path (itself bit-identical to the oracle) on the same input:
    positions and velocities within binary32 rounding; n_CR, J_CR within
    binary32 rounding of the amounts; -dM and -dE_k within bounds made of the
    terms of each particle's change (the rotation half-angle theta times |v|,
    the kick he, the change itself), not of |v|, summed over the particles
    that can reach each cell."""
    _need_gpu()
    wl = W.bell3d(n=128, ppc=32, seed=4001, n_steps=100)
    g32 = DeviceRun(wl, precision=1)
    g32.step(1)
    (D32,) = g32.deposits()
    ((x32, v32),) = g32.particles()
    g32.ctx.check()
    del g32
    torch.cuda.empty_cache()
    g64 = DeviceRun(wl)
    (D0,) = g64.deposits()
    g64.step(1)
    (D64,) = g64.deposits()
    ((x64, v64),) = g64.particles()
    del g64
    torch.cuda.empty_cache()
    L = 128.0
    dx = x32 - x64
    dx -= L * np.round(dx / L)
    vmax = np.abs(v64).max()
    assert np.abs(dx).max() <= 10 * EPS32
    assert np.abs(v32 - v64).max() <= 20 * EPS32 * vmax
    slack = 2 * 27 * 0.5 * 64
    for ch in range(4):
        assert np.abs(D32[ch] - D64[ch]).max() <= 10 * EPS32 * np.abs(D64[ch]).max() + slack, ch
    # E at cell centres from the initial n_CR, J_CR (eq. emfcr2; v_g = 0 here)
    S = 2.0 ** 40
    n = D0[0] / S
    J = D0[1:4] / S
    ng = wl.box.qomc_gas * wl.rho
    R = n / (ng + n)
    E = -((1.0 - R) * np.cross(J.T, wl.B.T).T) / ng
    Emax = np.sqrt((E * E).sum(axis=0)).max()
    C = wl.box.C
    vabs = np.sqrt((wl.v * wl.v).sum(axis=0))
    gam = np.sqrt(1.0 + vabs ** 2 / C ** 2)
    hq = 0.5 * abs(wl.dt) * np.abs(wl.qm)
    theta = hq * np.sqrt((wl.B ** 2).sum(axis=0)).max() / gam
    he = hq * Emax
    dv = np.sqrt(((v64 - wl.v) ** 2).sum(axis=0))
    mS = np.abs(wl.m) * S
    bM = (32 * EPS32 * mS * (theta * vabs + 2 * he + dv)).max()
    bE = (32 * EPS32 * mS * (2 * he * (vabs + dv) / gam + dv * vabs / gam)).max()
    del dv, vabs, gam
    # particles whose corrector stencil can reach each cell: initial cell +-2
    ci = [np.floor(wl.x[d]).astype(np.int64) % 128 for d in range(3)]
    cnt = np.bincount(ci[0] + 128 * (ci[1] + 128 * ci[2]), minlength=128 ** 3).reshape(128, 128, 128)
    reach = np.zeros_like(cnt)
    for oz in range(-2, 3):
        for oy in range(-2, 3):
            for ox in range(-2, 3):
                reach += np.roll(cnt, (oz, oy, ox), axis=(0, 1, 2))
    reach = reach.ravel().astype(np.float64)
    for ch in range(4, 7):
        err = np.abs(D32[ch] - D64[ch]).astype(np.float64)
        assert (err <= reach * (bM + 27)).all(), (ch, (err / (reach * (bM + 27))).max())
    err = np.abs(D32[7] - D64[7]).astype(np.float64)
    assert (err <= reach * (bE + 27)).all(), (err / (reach * (bE + 27))).max()
