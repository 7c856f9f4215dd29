"""GPU parity: the HIP library against the oracle, through the C ABI.

Deposits must be bit-identical (64-bit fixed point).  Particle states are
compared element by element and must be identical too: both sides perform the
same binary64 operations in the same order, so a cell index, an offset or a
velocity component that differs in any bit is a defect (the goal allows
1e-12 relative; nothing needs it).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1412_1087_amd import workloads as W  # noqa: E402

from gpu_helpers import DeviceRun, oracle_run, to_dev  # noqa: E402

def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _assert_states(wl, sysO, x_g, v_g):
    """Positions (read back as x0 + dx((i + 1/2) + d) on both sides) and
    four-velocities equal the oracle's in every bit, particle by particle."""
    xo = sysO.positions()
    vo = sysO.v
    badx = np.argwhere(x_g != xo)
    assert len(badx) == 0, (f"{len(badx)} position components differ, first (comp, particle) "
                            f"{tuple(badx[0])}: {x_g[tuple(badx[0])]!r} vs {xo[tuple(badx[0])]!r}")
    badv = np.argwhere(v_g != vo)
    assert len(badv) == 0, (f"{len(badv)} velocity components differ, first (comp, particle) "
                            f"{tuple(badv[0])}: {v_g[tuple(badv[0])]!r} vs {vo[tuple(badv[0])]!r}")


def _parity(wl, n_steps=1, tile=(0, 0, 0), steps_per_call=1, moves=0):
    _need_gpu()
    g = DeviceRun(wl, tile=tile, moves=moves)
    o = oracle_run(wl)
    (D0,) = g.deposits()
    assert (D0 == o.D).all(), "init deposit differs"
    done = 0
    while done < n_steps:
        k = min(steps_per_call, n_steps - done)
        g.step(k)
        o.step(wl.B, wl.vg, wl.rho, wl.dt, k)
        done += k
        (D,) = g.deposits()
        for ch in range(8):
            bad = np.nonzero(D[ch] != o.D[ch])[0]
            assert len(bad) == 0, f"channel {ch} differs in {len(bad)} cells after {done} steps"
        ((x, v),) = g.particles()
        _assert_states(wl, o, x, v)
    g.ctx.check()
    return g, o


def test_arith_selftest_matches_host_ieee():
    """Device sqrt, division and fma round exactly as IEEE binary64 (the host)."""
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    rng = np.random.default_rng(1)
    n = 1 << 20
    a = np.abs(rng.normal(size=n)) * 10.0 ** rng.uniform(-30, 30, size=n)
    b = rng.normal(size=n) * 10.0 ** rng.uniform(-30, 30, size=n)
    c = rng.normal(size=n) * 10.0 ** rng.uniform(-30, 30, size=n)
    # ranges the step uses: C^2 + v^2 with C = 20
    a[: n // 4] = 400.0 + rng.uniform(0, 1e6, size=n // 4)
    out = M.selftest_arith(to_dev(a), to_dev(b), to_dev(c)).cpu().numpy()
    assert (out[0] == np.sqrt(a)).all()
    assert (out[1] == a / b).all()
    # fma: a*b + c rounded once; float(Fraction) rounds to nearest-even
    from fractions import Fraction
    sel = rng.integers(0, n, size=20000)
    for i in sel:
        exact = Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i]))
        assert out[2][i] == float(exact)
    ints = c.view(np.int64)
    assert (out[3] == ints.astype(np.float64)).all()


def test_parity_gyro2d_full_size_one_step():
    _parity(W.gyro2d(), n_steps=1)


def test_parity_gyro2d_multi_step_one_call():
    _parity(W.gyro2d(nx=16, ny=16, ppc=8, seed=5), n_steps=6, steps_per_call=3)


def test_parity_bell3d_hall_small():
    _parity(W.bell3d(n=16, ppc=4, seed=7), n_steps=2)


def test_parity_bell3d_no_hall_ragged():
    # 13 x 9 x 6 cells: ragged edge tiles in every dimension
    _parity(W.bell3d(n=(13, 9, 6), ppc=3, seed=8, hall=0), n_steps=2)


def test_parity_shock2d_small():
    _parity(W.shock2d(nx=512, ny=32, n_particles=512 * 32 * 8, seed=9), n_steps=2)


@pytest.mark.parametrize("tile", [(8, 8, 1), (16, 16, 1), (32, 32, 1), (64, 16, 1)])
def test_parity_2d_tiles(tile):
    _parity(W.gyro2d(nx=37, ny=23, ppc=5, seed=10), n_steps=2, tile=tile)


@pytest.mark.parametrize("tile", [(4, 4, 4), (8, 8, 4), (16, 4, 4)])
def test_parity_3d_tiles(tile):
    _parity(W.bell3d(n=(11, 10, 9), ppc=2, seed=11), n_steps=1, tile=tile)


def test_parity_many_tiles_initial_sort_large_histogram():
    # 256 x 33 tiles of 16 x 16 cells: an LDS histogram of more than 32 KB
    _parity(W.shock2d(nx=4096, ny=528, n_particles=100_000, seed=14), n_steps=1, tile=(16, 16, 1))


def test_parity_many_tiles_initial_sort_fallback():
    # 512 x 65 tiles of 8 x 8 cells: more tiles than the initial sort's LDS
    # histograms hold (32768), so it counts with per-wave global atomics
    _parity(W.shock2d(nx=4096, ny=520, n_particles=100_000, seed=16), n_steps=1, tile=(8, 8, 1))


@pytest.mark.parametrize("order", ["sorted", "reversed", "one_tile_first"])
def test_parity_input_order(order):
    # the initial sort sees long runs of one tile (sorted input), runs in
    # descending tile order, or one tile's particles packed into few blocks
    import dataclasses
    wl = W.bell3d(n=(24, 16, 12), ppc=6, seed=15)
    box = wl.box
    cell = [np.floor(wl.x[d] / box.dx[d]).astype(np.int64) for d in range(3)]
    key = (cell[2] * box.n[1] + cell[1]) * box.n[0] + cell[0]
    if order == "sorted":
        perm = np.argsort(key, kind="stable")
    elif order == "reversed":
        perm = np.argsort(-key, kind="stable")
    else:
        first = (cell[0] < 8) & (cell[1] < 4) & (cell[2] < 4)
        perm = np.r_[np.flatnonzero(first), np.flatnonzero(~first)]
    wl = dataclasses.replace(wl, x=np.ascontiguousarray(wl.x[:, perm]), v=np.ascontiguousarray(wl.v[:, perm]),
                             m=wl.m[perm].copy(), qm=wl.qm[perm].copy())
    _parity(wl, n_steps=2)


def test_parity_tiny_boxes_wrap_onto_themselves():
    # boxes smaller than a tile and its ghost layers
    _parity(W.gyro2d(nx=3, ny=2, ppc=7, seed=12), n_steps=3)
    _parity(W.bell3d(n=(2, 3, 1), ppc=5, seed=13), n_steps=2)


def test_parity_multi_box_context():
    _need_gpu()
    wls = [W.gyro2d(nx=17, ny=40, ppc=3, seed=20), W.gyro2d(nx=8, ny=8, ppc=11, seed=21),
           W.gyro2d(nx=64, ny=16, ppc=2, seed=22)]
    g = DeviceRun(wls)
    os_ = [oracle_run(w) for w in wls]
    for st in range(2):
        g.step(1)
        for w, o in zip(wls, os_):
            o.step(w.B, w.vg, w.rho, w.dt, 1)
        Ds = g.deposits()
        ps = g.particles()
        for b, (w, o) in enumerate(zip(wls, os_)):
            assert (Ds[b] == o.D).all(), f"box {b} deposits differ"
            _assert_states(w, o, *ps[b])


def test_empty_box_and_no_particles():
    _need_gpu()
    wl = W.gyro2d(nx=8, ny=8, ppc=1, seed=23)
    empty = W.gyro2d(nx=8, ny=8, ppc=1, seed=24)
    for k in ("x", "v"):
        setattr(empty, k, getattr(empty, k)[:, :0])
    empty.m = empty.m[:0]
    empty.qm = empty.qm[:0]
    g = DeviceRun([wl, empty])
    o = oracle_run(wl)
    g.step(2)
    o.step(wl.B, wl.vg, wl.rho, wl.dt, 2)
    D = g.deposits()
    assert (D[0] == o.D).all()
    assert (D[1] == 0).all()


def test_deposit_read_reset_and_accumulate():
    _need_gpu()
    wl = W.gyro2d(nx=12, ny=12, ppc=4, seed=25)
    g = DeviceRun(wl)
    o = oracle_run(wl)
    g.step(2)
    o.step(wl.B, wl.vg, wl.rho, wl.dt, 2)
    D = g.ctx.deposit_read(reset_accumulated=True).cpu().numpy()
    assert (D == o.D).all()
    o.clear_accumulated()
    g.step(1)
    o.step(wl.B, wl.vg, wl.rho, wl.dt, 1)
    (D,) = g.deposits()
    assert (D == o.D).all()


def test_negative_dt_reverses():
    _need_gpu()
    wl = W.gyro2d(nx=12, ny=12, ppc=4, seed=26)
    g = DeviceRun(wl)
    ((x0, v0),) = g.particles()
    g.step(10)
    g.step(10, dts=[-wl.dt])
    ((x1, v1),) = g.particles()
    L = np.array([12.0, 12.0, 1.0])[:, None]
    d = x1 - x0
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-10
    assert np.abs(v1 - v0).max() < 1e-10 * np.abs(v0).max()


def test_move_limit_rejected():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    wl = W.gyro2d(nx=8, ny=8, ppc=1, seed=27)
    g = DeviceRun(wl)
    with pytest.raises(M.MhdpicError) as e:
        g.ctx.step(g.B, g.vg, g.rho, [0.2], 1)  # C*dt/dx = 4 > 2
    assert e.value.code == M.ERANGE


def test_nonfinite_velocity_rejected_at_init():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    wl = W.gyro2d(nx=8, ny=8, ppc=1, seed=28)
    wl.v = wl.v.copy()
    wl.v[1, 5] = np.nan
    with pytest.raises(M.MhdpicError) as e:
        DeviceRun(wl)
    assert e.value.code == M.ENONFINITE


def test_amount_overflow_flagged():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    wl = W.gyro2d(nx=8, ny=8, ppc=1, seed=29)
    wl.m = wl.m.copy()
    wl.m[3] = 1e5  # (q/mc) m 2^40 > 2^51
    with pytest.raises(M.MhdpicError) as e:
        DeviceRun(wl)
    assert e.value.code == M.ERANGE


def test_parity_sides_one_more_than_tiles():
    # n % tile == 1 in every dimension: the last tile is shifted to two cells
    _parity(W.gyro2d(nx=33, ny=17, ppc=4, seed=30), n_steps=4, tile=(16, 16, 1))
    _parity(W.bell3d(n=(17, 9, 5), ppc=3, seed=31), n_steps=3, tile=(8, 4, 4))


def test_parity_many_steps_stays_bit_exact():
    # particles cross many tiles; binning and deposits must stay exact
    _parity(W.shock2d(nx=256, ny=32, n_particles=256 * 32 * 4, seed=32), n_steps=24,
            steps_per_call=8)


def test_parity_dt_changes_between_calls():
    _need_gpu()
    wl = W.gyro2d(nx=20, ny=20, ppc=5, seed=33)
    g = DeviceRun(wl)
    o = oracle_run(wl)
    for f in (1.0, 0.5, -0.7, 1.0):
        g.step(3, dts=[f * wl.dt])
        o.step(wl.B, wl.vg, wl.rho, f * wl.dt, 3)
        (D,) = g.deposits()
        assert (D == o.D).all()
        ((x, v),) = g.particles()
        _assert_states(wl, o, x, v)


# ---------------------------------------------------------------------------
# a lower corner away from zero and a different cell size along each axis
# ---------------------------------------------------------------------------

X0 = (-3.7, 11.2, 0.5)
DX = (0.5, 2.0, 1.25)


def test_parity_2d_offset_origin_anisotropic_cells():
    _parity(W.gyro2d(nx=37, ny=23, ppc=5, seed=50, dx=DX, x0=X0), n_steps=4, steps_per_call=2)


def test_parity_3d_hall_offset_origin_anisotropic_cells():
    _parity(W.bell3d(n=(13, 9, 7), ppc=3, seed=51, dx=DX, x0=X0, hall=1), n_steps=3)


def test_parity_3d_hall_offset_origin_anisotropic_full_tiles():
    # several whole 8x4x4 tiles plus ragged ones, Hall term on
    _parity(W.bell3d(n=(20, 12, 10), ppc=4, seed=52, dx=(1.25, 0.5, 2.0), x0=(7.3, -0.9, -12.6),
                     hall=1), n_steps=2)


def test_parity_multi_box_origins_and_cell_sizes():
    _need_gpu()
    wls = [W.gyro2d(nx=17, ny=40, ppc=3, seed=53, dx=(0.5, 2.0, 1.0), x0=(-3.7, 11.2, 0.0)),
           W.gyro2d(nx=8, ny=8, ppc=11, seed=54, dx=(3.0, 0.75, 1.0), x0=(100.25, -40.5, 0.0)),
           W.gyro2d(nx=64, ny=16, ppc=2, seed=55)]
    g = DeviceRun(wls)
    os_ = [oracle_run(w) for w in wls]
    for b, o in enumerate(os_):
        assert (g.deposits()[b] == o.D).all(), f"box {b} init deposit differs"
    for st in range(3):
        g.step(1)
        for w, o in zip(wls, os_):
            o.step(w.B, w.vg, w.rho, w.dt, 1)
        Ds = g.deposits()
        ps = g.particles()
        for b, (w, o) in enumerate(zip(wls, os_)):
            assert (Ds[b] == o.D).all(), f"box {b} deposits differ after {st + 1} steps"
            _assert_states(w, o, *ps[b])


def test_parity_3d_multi_box_origins_and_cell_sizes_hall():
    _need_gpu()
    wls = [W.bell3d(n=(9, 8, 6), ppc=3, seed=56, dx=DX, x0=X0, hall=1),
           W.bell3d(n=(6, 10, 5), ppc=2, seed=57, dx=(2.0, 1.0, 0.75), x0=(-50.0, 3.3, 8.125), hall=1)]
    g = DeviceRun(wls)
    os_ = [oracle_run(w) for w in wls]
    for st in range(2):
        g.step(1)
        for w, o in zip(wls, os_):
            o.step(w.B, w.vg, w.rho, w.dt, 1)
        Ds = g.deposits()
        ps = g.particles()
        for b, (w, o) in enumerate(zip(wls, os_)):
            assert (Ds[b] == o.D).all(), f"box {b} deposits differ after {st + 1} steps"
            _assert_states(w, o, *ps[b])


def test_position_too_far_from_origin_rejected_at_init():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    wl = W.gyro2d(nx=8, ny=8, ppc=1, seed=58, dx=(0.5, 2.0, 1.0), x0=(-3.7, 11.2, 0.0))
    wl.x = wl.x.copy()
    wl.x[0, 7] = -3.7 + 0.5 * 2.0 ** 31 + 1.0
    with pytest.raises(M.MhdpicError) as e:
        DeviceRun(wl)
    assert e.value.code == M.ERANGE


# ---------------------------------------------------------------------------
# the particles moved to their new slots by the binning or by the push
# ---------------------------------------------------------------------------

MOVES = [pytest.param(1, id="in_binning"), pytest.param(2, id="in_push")]


@pytest.mark.parametrize("moves", MOVES)
def test_parity_moves_2d_many_steps(moves):
    # relativistic isotropic particles crossing tiles every few steps
    _parity(W.shock2d(nx=256, ny=32, n_particles=256 * 32 * 4, seed=60), n_steps=12,
            steps_per_call=4, moves=moves)


@pytest.mark.parametrize("moves", MOVES)
def test_parity_moves_3d_hall_ragged(moves):
    _parity(W.bell3d(n=(13, 9, 6), ppc=3, seed=61, hall=1), n_steps=4, steps_per_call=2,
            moves=moves)


@pytest.mark.parametrize("moves", MOVES)
def test_parity_moves_3d_tiles_and_subcycling(moves):
    _need_gpu()
    wl = W.bell3d(n=(11, 10, 9), ppc=2, seed=62)
    g = DeviceRun(wl, tile=(4, 4, 4), moves=moves)
    o = oracle_run(wl)
    for _ in range(2):
        g.step(2, n_sub=3)
        o.step(wl.B, wl.vg, wl.rho, wl.dt, 2, n_sub=3)
    (D,) = g.deposits()
    assert (D == o.D).all()
    ((x, v),) = g.particles()
    _assert_states(wl, o, x, v)
    g.ctx.check()


def test_parity_moves_switched_between_calls():
    _need_gpu()
    for wl in (W.gyro2d(nx=37, ny=23, ppc=5, seed=63), W.bell3d(n=(13, 9, 6), ppc=3, seed=64)):
        g = DeviceRun(wl)
        o = oracle_run(wl)
        for moves in (2, 1, 0, 2, 2, 1):
            g.ctx.set_particle_moves(moves)
            g.step(2)
            o.step(wl.B, wl.vg, wl.rho, wl.dt, 2)
            (D,) = g.deposits()
            assert (D == o.D).all(), f"moves {moves}"
            ((x, v),) = g.particles()
            _assert_states(wl, o, x, v)
        g.ctx.check()


def test_particle_moves_rejects_unknown_setting():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    g = DeviceRun(W.gyro2d(nx=8, ny=8, ppc=2, seed=65))
    with pytest.raises(M.MhdpicError):
        g.ctx.set_particle_moves(3)


def test_parity_3d_long_run_stays_bit_exact():
    # 200 steps of a small beam box: particles cross tiles and the periodic
    # wrap many times, with the particles moved by the push through the map
    _parity(W.bell3d(n=(12, 10, 9), ppc=4, seed=66, hall=1), n_steps=200, steps_per_call=50)


def test_parity_2d_dense_band_long_run_stays_bit_exact():
    # a dense band (tiles of several work items) over 120 steps, the
    # particles moved by the push in chunked level order
    _parity(W.shock2d(nx=128, ny=32, n_particles=128 * 32 * 6, seed=67), n_steps=120,
            steps_per_call=40)
