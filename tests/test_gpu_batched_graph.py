"""Batched form: many independent boxes in one context, stepped through one
HIP graph launch; plus the tile autotuner."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1412_1087_amd import workloads as W  # noqa: E402

from gpu_helpers import DeviceRun, assert_states_exact, oracle_run  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _boxes(n=10, seed0=900):
    return W.batch2d(n_boxes=n, seed0=seed0, side=(16, 40), ppc=(2, 8))


def test_batched_fp64_graph_replays_match_eager_and_oracle():
    _need_gpu()
    wls = _boxes()
    eager = DeviceRun(wls)
    graph = DeviceRun(wls)
    oracles = [oracle_run(w) for w in wls]
    stream = torch.cuda.Stream()
    dts = [w.dt for w in wls]
    for rep in range(3):
        eager.step(4, dts=dts)
        with torch.cuda.stream(stream):
            graph.ctx.step_graph(graph.B, graph.vg, graph.rho, dts, 4, stream)
        stream.synchronize()
        torch.cuda.synchronize()
        for w, o in zip(wls, oracles):
            o.step(w.B, w.vg, w.rho, w.dt, 4)
        De = eager.deposits()
        Dg = graph.deposits()
        pe = eager.particles()
        pg = graph.particles()
        for b, o in enumerate(oracles):
            assert (Dg[b] == De[b]).all(), f"replay {rep}: box {b} graph != eager"
            assert (Dg[b] == o.D).all(), f"replay {rep}: box {b} graph != oracle"
            assert (pg[b][1] == pe[b][1]).all()
        graph.ctx.check()


def test_batched_fp32_each_box_equals_its_single_box_run():
    _need_gpu()
    wls = _boxes(n=8, seed0=950)
    many = DeviceRun(wls, precision=1)
    singles = [DeviceRun(w, precision=1) for w in wls]
    stream = torch.cuda.Stream()
    dts = [w.dt for w in wls]
    with torch.cuda.stream(stream):
        many.ctx.step_graph(many.B, many.vg, many.rho, dts, 6, stream)
    stream.synchronize()
    torch.cuda.synchronize()
    for s in singles:
        s.step(6)
    Dm = many.deposits()
    pm = many.particles()
    for b, s in enumerate(singles):
        (Ds,) = s.deposits()
        ((xs, vs),) = s.particles()
        assert (Dm[b] == Ds).all(), b
        assert (pm[b][1] == vs).all(), b


def test_graph_rejects_odd_steps_and_default_stream():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    wl = W.gyro2d(nx=16, ny=16, ppc=2, seed=960)
    g = DeviceRun(wl)
    s = torch.cuda.Stream()
    with pytest.raises(M.MhdpicError):
        g.ctx.step_graph(g.B, g.vg, g.rho, [wl.dt], 3, s)
    with pytest.raises(M.MhdpicError):
        g.ctx.step_graph(g.B, g.vg, g.rho, [wl.dt], 2, torch.cuda.default_stream())


def test_autotune_picks_a_compiled_shape_that_stays_exact():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    from gpu_helpers import gpu_box, to_dev
    wl = W.bell3d(n=(16, 12, 12), ppc=4, seed=970)
    box = gpu_box(wl.box)
    tile, ms = M.autotune([box], [wl.N], to_dev(wl.x), to_dev(wl.v), to_dev(wl.m), to_dev(wl.qm),
                          to_dev(wl.B), to_dev(wl.vg), to_dev(wl.rho), wl.dt, n_steps=4)
    assert tile in [(8, 4, 4), (8, 8, 4), (4, 4, 4), (16, 4, 4)]
    assert ms > 0
    g = DeviceRun(wl, tile=tile)
    o = oracle_run(wl)
    g.step(2)
    o.step(wl.B, wl.vg, wl.rho, wl.dt, 2)
    (D,) = g.deposits()
    assert (D == o.D).all()


def test_boxes_with_different_tile_shapes_match_oracle_eager_and_graph():
    """One context whose boxes use three tile shapes (one push launch per
    shape), eager and graph-captured, bit-exact against the oracle."""
    _need_gpu()
    wls = _boxes(n=9, seed0=990)
    shapes = [(16, 16, 1), (32, 16, 1), (8, 8, 1)]
    tiles = [shapes[b % 3] for b in range(len(wls))]
    eager = DeviceRun(wls, tile=tiles)
    graph = DeviceRun(wls, tile=tiles)
    oracles = [oracle_run(w) for w in wls]
    stream = torch.cuda.Stream()
    dts = [w.dt for w in wls]
    for rep in range(2):
        eager.step(2, dts=dts)
        with torch.cuda.stream(stream):
            graph.ctx.step_graph(graph.B, graph.vg, graph.rho, dts, 2, stream)
        stream.synchronize()
        torch.cuda.synchronize()
        for w, o in zip(wls, oracles):
            o.step(w.B, w.vg, w.rho, w.dt, 2)
        De, Dg = eager.deposits(), graph.deposits()
        pe, pg = eager.particles(), graph.particles()
        for b, o in enumerate(oracles):
            assert (De[b] == o.D).all(), f"replay {rep}: box {b} eager != oracle"
            assert (Dg[b] == o.D).all(), f"replay {rep}: box {b} graph != oracle"
            assert_states_exact(pe[b][0], pe[b][1], o.positions(), o.v, f"box {b}")
            assert (pg[b][1] == pe[b][1]).all()
    eager.ctx.check()
    graph.ctx.check()


def test_class_autotuner_gives_compiled_shapes_per_box_that_stay_exact():
    _need_gpu()
    from paper_1412_1087_amd import mhdpic as M
    from gpu_helpers import gpu_box, to_dev
    wls = W.batch2d(n_boxes=12, seed0=1990, side=(16, 96), ppc=(2, 6))
    cat = lambda f: np.concatenate([f(w) for w in wls], axis=-1)
    tiles, ms = M.autotune_classes([gpu_box(w.box) for w in wls], [w.N for w in wls],
                                   to_dev(cat(lambda w: w.x)), to_dev(cat(lambda w: w.v)),
                                   to_dev(cat(lambda w: w.m)), to_dev(cat(lambda w: w.qm)),
                                   to_dev(cat(lambda w: w.B)), to_dev(cat(lambda w: w.vg)),
                                   to_dev(cat(lambda w: w.rho)), [w.dt for w in wls], n_steps=4)
    assert len(tiles) == len(wls) and ms > 0
    compiled = [(16, 16, 1), (32, 16, 1), (8, 8, 1), (32, 32, 1), (64, 16, 1)]
    assert all(t in compiled for t in tiles)
    # boxes of one size class share a shape
    cls = [int(np.log2(w.box.n_cells) // 2) for w in wls]
    for k in set(cls):
        assert len({t for t, c in zip(tiles, cls) if c == k}) == 1
    g = DeviceRun(wls, tile=tiles)
    oracles = [oracle_run(w) for w in wls]
    g.step(2)
    for w, o in zip(wls, oracles):
        o.step(w.B, w.vg, w.rho, w.dt, 2)
    D = g.deposits()
    for b, o in enumerate(oracles):
        assert (D[b] == o.D).all(), b


def test_graph_subcycled_replays_match_eager_and_oracle():
    _need_gpu()
    wls = _boxes(n=4, seed0=980)
    eager = DeviceRun(wls)
    graph = DeviceRun(wls)
    oracles = [oracle_run(w) for w in wls]
    stream = torch.cuda.Stream()
    dts = [w.dt for w in wls]
    for rep in range(2):
        eager.step(2, dts=dts, n_sub=3)
        with torch.cuda.stream(stream):
            graph.ctx.step_graph(graph.B, graph.vg, graph.rho, dts, 2, stream, n_sub=3)
        stream.synchronize()
        torch.cuda.synchronize()
        for w, o in zip(wls, oracles):
            o.step(w.B, w.vg, w.rho, w.dt, 2, n_sub=3)
        De, Dg = eager.deposits(), graph.deposits()
        pe, pg = eager.particles(), graph.particles()
        for b, o in enumerate(oracles):
            assert (Dg[b] == De[b]).all(), f"replay {rep}: box {b} graph != eager"
            assert (Dg[b] == o.D).all(), f"replay {rep}: box {b} graph != oracle"
            assert (pg[b][1] == pe[b][1]).all()


def test_graph_and_eager_calls_mix_in_one_context():
    """Eager calls between graph launches may change dt and leave the
    particle and work-list buffers swapped: the next graph call must see both
    (it re-uploads the step constants and recaptures)."""
    _need_gpu()
    wl = W.gyro2d(nx=24, ny=20, ppc=4, seed=990)
    g = DeviceRun(wl)
    o = oracle_run(wl)
    stream = torch.cuda.Stream()
    dt1, dt2 = wl.dt, 0.7 * wl.dt
    plan = [("graph", dt1, 2), ("eager", dt2, 1), ("graph", dt1, 2), ("eager", dt1, 3), ("graph", dt1, 2)]
    for kind, dt, n in plan:
        if kind == "graph":
            with torch.cuda.stream(stream):
                g.ctx.step_graph(g.B, g.vg, g.rho, [dt], n, stream)
            stream.synchronize()
            torch.cuda.synchronize()
        else:
            g.step(n, dts=[dt])
        o.step(wl.B, wl.vg, wl.rho, dt, n)
        (D,) = g.deposits()
        assert (D == o.D).all(), (kind, dt, n)
    ((x, v),) = g.particles()
    assert_states_exact(x, v, o.positions(), o.v, "after graph and eager steps")


def test_user_captured_step_replays_match_the_oracle():
    """mhdpic_step captured by the caller (torch.cuda.graph) and replayed,
    with eager steps and synchronisations between the replays."""
    _need_gpu()
    wl = W.gyro2d(nx=20, ny=24, ppc=4, seed=995)
    g = DeviceRun(wl)
    o = oracle_run(wl)
    g.step(2)                      # uploads this dt before the capture
    o.step(wl.B, wl.vg, wl.rho, wl.dt, 2)
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        g.ctx.step(g.B, g.vg, g.rho, [wl.dt], 2, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        o.step(wl.B, wl.vg, wl.rho, wl.dt, 2)
        (D,) = g.deposits()
        assert (D == o.D).all(), f"replay {rep}"
        g.step(2)                  # eager work between replays (even n_steps)
        o.step(wl.B, wl.vg, wl.rho, wl.dt, 2)
        (D,) = g.deposits()
        assert (D == o.D).all(), f"eager after replay {rep}"


@pytest.mark.parametrize("moves", [1, 2], ids=["in_binning", "in_push"])
@pytest.mark.parametrize("dim", [2, 3])
def test_graph_replays_match_eager_for_both_move_settings(moves, dim):
    _need_gpu()
    wls = _boxes(n=6, seed0=1700) if dim == 2 else [W.bell3d(n=(13, 9, 6), ppc=3, seed=1701, hall=1)]
    eager = DeviceRun(wls, moves=moves)
    graph = DeviceRun(wls, moves=moves)
    oracles = [oracle_run(w) for w in wls]
    stream = torch.cuda.Stream()
    dts = [w.dt for w in wls]
    for rep in range(3):
        eager.step(2, dts=dts)
        with torch.cuda.stream(stream):
            graph.ctx.step_graph(graph.B, graph.vg, graph.rho, dts, 2, stream)
        stream.synchronize()
        torch.cuda.synchronize()
        for w, o in zip(wls, oracles):
            o.step(w.B, w.vg, w.rho, w.dt, 2)
        De, Dg = eager.deposits(), graph.deposits()
        pe, pg = eager.particles(), graph.particles()
        for b, o in enumerate(oracles):
            assert (De[b] == o.D).all(), f"replay {rep}: box {b} eager != oracle"
            assert (Dg[b] == o.D).all(), f"replay {rep}: box {b} graph != oracle"
            assert_states_exact(pg[b][0], pg[b][1], o.positions(), o.v, f"box {b}")
    eager.ctx.check()
    graph.ctx.check()
