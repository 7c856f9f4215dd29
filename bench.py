#!/usr/bin/env python3
"""Throughput of the CR particle step (gather + push + deposit) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints ONE JSON line on stdout.  The headline workload is the 3D Bell-style
box: 64^3 cells, 16 particles per cell (4,194,304 particles), CR-Hall term on,
binary64 path, C = 20.  Inputs are seeded and synthetic; they are resident in
HBM before the timed region starts.  A step is one pass of the whole hot
path: binning, cell-centred E, the fused gather/push/deposit kernel.

Extra legs:
  * roofline: the fused push kernel's algorithmic bytes per launch divided by
    its average launch duration, measured with HIP events recorded by the
    library on the launch stream over the timed region;
  * cpu_baseline: the reference oracle (single-threaded binary64 C) timed on
    the host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1412_1087_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

DATA_NOTE = {
    "bell3d": "synthetic (seeded; shapes of the paper's Bell-instability test box)",
    "shock2d": "synthetic (seeded; shapes of the paper's 2D shock runs: upstream/downstream "
               "gas, CR band near the shock)",
    "gyro2d": "synthetic (seeded; the paper's gyration-test settings on a 32x32 box)",
    "bell3d128": "synthetic (seeded; the Bell-instability test box at 128^3, 32 per cell)",
}


def make_workload(name: str):
    from paper_1412_1087_amd import workloads as W
    if name == "bell3d":
        wl = W.bell3d()
        label = "bell3d-64^3-ppc16-hall"
    elif name == "shock2d":
        wl = W.shock2d()
        label = "shock2d-8192x32-16.8M"
    elif name == "gyro2d":
        wl = W.gyro2d()
        label = "gyro2d-32x32-ppc16"
    elif name == "bell3d128":
        wl = W.bell3d(n=128, ppc=32, seed=4001, n_steps=100)
        label = "bell3d-128^3-ppc32-hall"
    else:
        raise SystemExit(f"unknown workload {name}")
    return wl, label


def algorithmic_bytes(ndim: int, N: int, NC: int, fsz: int = 8, msz: int = 8,
                      moves_in_push: bool = False) -> dict:
    """Bytes the fused push kernel must move per launch.

    Per particle: read cell index (4), offsets (ndim*fsz), four-velocity
    (3*fsz), m and q/mc (2*msz); write cell index, offsets, four-velocity.
    When the push also moves the particles to their new slots, it reads the
    slot map (4) and writes m and q/mc (2*msz) as well.
    Per cell: read E and B (6*fsz), read+write the accumulated -dM, -dE_k
    (2*32), write n_CR, J_CR (32)."""
    p_read = 4 + ndim * fsz + 3 * fsz + 2 * msz + (4 if moves_in_push else 0)
    p_write = 4 + ndim * fsz + 3 * fsz + (2 * msz if moves_in_push else 0)
    c_bytes = 6 * fsz + 64 + 32
    return dict(per_particle=p_read + p_write, per_cell=c_bytes,
                per_launch=N * (p_read + p_write) + NC * c_bytes)


# --------------------------------------------------------------------------
# GPU leg
# --------------------------------------------------------------------------

def moves_in_push(ndim: int, moves: int) -> bool:
    """Whether the push moves the particles (the library's automatic choice)."""
    return moves != 1


def run_gpu(wl, steps: int, warmup: int, calibrate_copy: bool, tile=(0, 0, 0), precision=0,
            moves=0):
    import torch
    from paper_1412_1087_amd import mhdpic as M

    dev = torch.device("cuda:0")
    if calibrate_copy:
        # a plain copy of known size, for scaling the HBM byte counters
        a = torch.empty(512 * 1024 * 1024 // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 536870912 bytes read, 536870912 bytes written")
        del a, b

    def t(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    box = M.Box(ndim=wl.box.ndim, n=wl.box.n, dx=wl.box.dx, x0=wl.box.x0, C=wl.box.C,
                qomc_gas=wl.box.qomc_gas, hall=wl.box.hall, frac_bits=wl.box.frac_bits,
                max_move_cells=wl.box.max_move_cells, tile=tile)
    B, vg, rho = t(wl.B), t(wl.vg), t(wl.rho)
    xs, vs, ms_, qs = t(wl.x), t(wl.v), t(wl.m), t(wl.qm)
    torch.cuda.synchronize()
    t_init = time.perf_counter()
    ctx = M.Context([box], [wl.N], xs, vs, ms_, qs, precision=precision)
    torch.cuda.synchronize()
    init_ms = 1e3 * (time.perf_counter() - t_init)
    if moves:
        ctx.set_particle_moves(moves)
    del xs, vs, ms_, qs
    log(f"init done: N={wl.N} cells={box.n_cells}, context creation {init_ms:.1f} ms")
    if warmup > 0:
        ctx.step(B, vg, rho, wl.dt, warmup)
    ctx.check()
    torch.cuda.synchronize()
    log("warmup done")

    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # inside the timed region only the push launches carry event pairs (each
    # recorded event costs stream time); the other phases are timed after it
    ctx.timing(True, phases=("push",))
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    ctx.step(B, vg, rho, wl.dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    ctx.timing(False)
    push = ctx.timing_read()["push"]
    ctx.check()
    ms = e0.elapsed_time(e1)
    log(f"timed {steps} steps: {ms:.3f} ms (events), {1e3 * (w1 - w0):.3f} ms (wall)")
    log(f"  push     : {push[0]:9.3f} ms over {push[1]} launches")
    # breakdown: a separate, fully instrumented pass (not part of the timed region)
    nb = max(2, min(steps, 20))
    ctx.timing(True)
    ctx.step(B, vg, rho, wl.dt, nb)
    torch.cuda.synchronize()
    ctx.timing(False)
    phases = ctx.timing_read()
    ctx.check()
    log(f"instrumented pass of {nb} steps (every phase timed):")
    for p, (pm, pn) in phases.items():
        log(f"  phase {p:9s}: {pm:9.3f} ms over {pn} launches")
    D = ctx.deposit_read().cpu()
    ctx.destroy()
    return dict(ms=ms, wall_ms=1e3 * (w1 - w0), push=push, phases=phases, breakdown_steps=nb,
                checksum=int(D.sum().item()), n_cells=box.n_cells, init_ms=init_ms)


# --------------------------------------------------------------------------
# the two other forms
# --------------------------------------------------------------------------

def _to(dev, a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _gpu_box(spec, tile=(0, 0, 0)):
    from paper_1412_1087_amd import mhdpic as M
    return M.Box(ndim=spec.ndim, n=spec.n, dx=spec.dx, x0=spec.x0, C=spec.C,
                 qomc_gas=spec.qomc_gas, hall=spec.hall, frac_bits=spec.frac_bits,
                 max_move_cells=spec.max_move_cells, tile=tile)


def _time_steps(ctx, B, vg, rho, dt, steps, warmup, n_sub=1):
    import torch
    ctx.step(B, vg, rho, dt, warmup, n_sub=n_sub)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.step(B, vg, rho, dt, steps, n_sub=n_sub)
    e1.record()
    torch.cuda.synchronize()
    ctx.check()
    return e0.elapsed_time(e1)


def run_subcycled_form(steps: int, warmup: int, n_sub: int = 5):
    """Particle sub-cycling on the 64^3 beam box: steps of n_sub particle
    sub-steps (n_CR, J_CR deposited once per step), against the same number
    of particle steps of the same size taken one step per field update."""
    import torch
    from paper_1412_1087_amd import mhdpic as M
    wl, label = make_workload("bell3d")
    dev = torch.device("cuda:0")
    B, vg, rho = _to(dev, wl.B), _to(dev, wl.vg), _to(dev, wl.rho)
    ctx = M.Context([_gpu_box(wl.box)], [wl.N], *(_to(dev, a) for a in (wl.x, wl.v, wl.m, wl.qm)))
    ms_sub = _time_steps(ctx, B, vg, rho, wl.dt * n_sub, steps, warmup, n_sub=n_sub)
    ms_one = _time_steps(ctx, B, vg, rho, wl.dt, steps * n_sub, warmup)
    ctx.destroy()
    n_upd = wl.N * steps * n_sub
    out = {"workload": label, "n_sub": n_sub, "steps": steps, "particle_step_dt": wl.dt,
           "value": round(n_upd / (ms_sub * 1e-3), 1), "unit": "particle sub-step updates/s",
           "nsub1_value": round(n_upd / (ms_one * 1e-3), 1),
           "speedup_vs_nsub1": round(ms_one / ms_sub, 3)}
    log(f"sub-cycled n_sub={n_sub}: {out['value']:.4g}/s vs {out['nsub1_value']:.4g}/s unsub-cycled")
    return out


def run_strip_form(steps: int, warmup: int):
    """The FP64 path on the 2D shock-like strip (8192 x 32 cells, 16.8 M
    particles, 80 % of them in a band of a tenth of the strip)."""
    wl, label = make_workload("shock2d")
    g = run_gpu(wl, steps, warmup, False)
    alg = algorithmic_bytes(wl.box.ndim, wl.N, g["n_cells"], moves_in_push=moves_in_push(2, 0))
    push_ms, push_n = g["push"]
    push_s = push_ms * 1e-3 / max(push_n, 1)
    out = {"workload": label, "particles": wl.N, "cells": g["n_cells"], "steps": steps,
           "value": round(wl.N * steps / (g["ms"] * 1e-3), 1),
           "ms_per_step": round(g["ms"] / steps, 5),
           "push_avg_launch_us": round(push_s * 1e6, 2),
           "push_hbm_frac": round(alg["per_launch"] / push_s / 1e9 / HBM_PEAK_GBS, 4),
           "hbm_frac_whole_step": round(alg["per_launch"] / (g["ms"] * 1e-3 / steps) / 1e9
                                        / HBM_PEAK_GBS, 4),
           "phases_ms_instrumented_pass": {k: round(v[0], 3) for k, v in g["phases"].items()},
           "instrumented_pass_steps": g["breakdown_steps"],
           "traffic": load_traffic(label, alg["per_launch"])}
    log(f"strip: {out['value']:.4g}/s, push {out['push_avg_launch_us']} us")
    return out


def run_shock_wall_form(steps: int, warmup: int):
    """The particle side of the Sec. 5 shock set-up: a 2D box of 8192 x 256
    cells of 12 ion inertial lengths with a conducting (reflecting) wall at
    x = 0 and an inflow (absorbing) face at x = L_x, the downstream gas at rest
    behind the front and the upstream flow at -v0, 2M CRs around the front,
    and CRs injected at the moving front every step (mhdpic_inject, tagged
    with the injection time, 4 per cell of swept gas).  Throughput counts the
    particle updates of the timed steps; the time includes the injections."""
    import torch
    from paper_1412_1087_amd import mhdpic as M
    from paper_1412_1087_amd import workloads as W
    dev = torch.device("cuda:0")
    st = W.shock_wall2d(nx=8192, ny=256, front_cell=2048)
    N0 = 2_000_000
    x, v, m, qm, _ = W.shock_population(st, N0, seed=7002)
    per_step = max(1, int(round(4 * st.box.n[1] * st.v_sh * st.dt / st.box.dx[0])))
    total = warmup + steps
    batches = [W.shock_injection(st, per_step, k * st.dt, seed=7100 + k) for k in range(total)]
    cap = N0 + per_step * total + 1024
    box = M.Box(ndim=2, n=st.box.n, dx=st.box.dx, x0=st.box.x0, C=st.box.C, hall=0,
                boundary=st.boundary, capacity=cap)
    B, vg, rho = _to(dev, st.B), _to(dev, st.vg), _to(dev, st.rho)
    ctx = M.Context([box], [N0], *(_to(dev, a) for a in (x, v, m, qm)))
    dbat = [tuple(_to(dev, a) for a in b) for b in batches]
    torch.cuda.synchronize()

    def run(ks):
        inj = 0.0
        for k in ks:
            bx, bv, bm, bq, bt = dbat[k]
            t0 = time.perf_counter()
            ctx.inject([bx.shape[1]], bx, bv, bm, bq, bt)
            inj += time.perf_counter() - t0
            ctx.step(B, vg, rho, st.dt, 1)
        return inj

    run(list(range(warmup)))
    torch.cuda.synchronize()
    n_start = sum(ctx.counts())
    t0 = time.perf_counter()
    inj = run(list(range(warmup, total)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_end = sum(ctx.counts())
    ctx.check()
    ctx.destroy()
    n_upd = 0.5 * (n_start + n_end) * steps
    out = {"workload": "shockwall2d-8192x256-2M", "particles_start": n_start, "particles_end": n_end,
           "injected_per_step": per_step, "steps": steps,
           "value": round(n_upd / wall, 1), "unit": "particle-updates/s",
           "ms_per_step": round(1e3 * wall / steps, 4),
           "inject_ms_per_step": round(1e3 * inj / steps, 4),
           "note": "wall clock of inject + step per step (each inject waits for the stream)"}
    log(f"shock wall: {out['value']:.4g}/s, {out['ms_per_step']} ms/step, "
        f"inject {out['inject_ms_per_step']} ms/step")
    return out


FEEDBACK_BYTES_PER_CELL = 168  # read n_CR, J_CR (32), B, v_g (48), rho (8); write 10 doubles


def measure_copy_gbps(nbytes: int = 1 << 31, reps: int = 5):
    """Device-to-device copy bandwidth (bytes read + written per second), the
    median of reps copies of nbytes: the HBM rate a streaming kernel reaches
    on this GPU, beside the published 8 TB/s peak."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    t = sorted(times)[len(times) // 2]
    return round(2 * nbytes / t / 1e9, 1)


def time_feedback(ctx, B, vg, rho, n_cells: int, reps: int = 20):
    """Average launch time of the cell-centred feedback kernel and its share
    of the HBM peak at 168 algorithmic bytes per cell."""
    import torch
    out = torch.empty((10, n_cells), dtype=torch.float64, device=B.device)
    ctx.feedback(B, vg, rho, out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.feedback(B, vg, rho, out)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    gbs = FEEDBACK_BYTES_PER_CELL * n_cells / (us * 1e-6) / 1e9
    log(f"feedback: {n_cells} cells, {us:.1f} us per launch, {gbs:.0f} GB/s")
    return {"cells": n_cells, "avg_launch_us": round(us, 2),
            "bytes_per_cell": FEEDBACK_BYTES_PER_CELL, "achieved_GBs": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


def run_precision_form(steps: int, warmup: int):
    """Precision form on the 128^3, 32-per-cell beam box, against the binary64
    path on the same seed: throughput of both and the one-step error."""
    import torch
    from paper_1412_1087_amd import mhdpic as M
    from paper_1412_1087_amd import workloads as W
    dev = torch.device("cuda:0")
    wl = W.bell3d(n=128, ppc=32, seed=4001, n_steps=100)
    label = "bell3d-128^3-ppc32-hall"
    box = _gpu_box(wl.box)
    B, vg, rho = _to(dev, wl.B), _to(dev, wl.vg), _to(dev, wl.rho)
    x, v, m, qm = (_to(dev, a) for a in (wl.x, wl.v, wl.m, wl.qm))
    out = {"workload": label, "particles": wl.N, "cells": box.n_cells, "steps": steps}
    ctx64 = M.Context([box], [wl.N], x, v, m, qm, precision=M.FP64)
    ctx32 = M.Context([box], [wl.N], x, v, m, qm, precision=M.FP32_MIXED)
    del x, v, m, qm
    # one step from the same state: error of the precision form
    ctx64.step(B, vg, rho, wl.dt, 1)
    ctx32.step(B, vg, rho, wl.dt, 1)
    x64, v64 = ctx64.particles_read()
    x32, v32 = ctx32.particles_read()
    D64 = ctx64.deposit_read()
    D32 = ctx32.deposit_read()
    torch.cuda.synchronize()
    Lb = torch.tensor([128.0, 128.0, 128.0], device=dev, dtype=torch.float64)[:, None]
    dx = x32 - x64
    dx = dx - Lb * torch.round(dx / Lb)
    vmax = v64.abs().max().item()
    err = {"pos_max_abs_cells": dx.abs().max().item(),
           "v_max_abs_rel": ((v32 - v64).abs().max().item()) / vmax}
    names = ["n", "Jx", "Jy", "Jz", "-dMx", "-dMy", "-dMz", "-dEk"]
    for ch, nm in enumerate(names):
        a = D64[ch].double()
        err[f"dep_{nm}_max_abs_rel"] = ((D32[ch].double() - a).abs().max() /
                                        a.abs().max().clamp(min=1)).item()
    out["one_step_error_vs_fp64"] = err
    del x64, v64, x32, v32, D64, D32
    ms64 = _time_steps(ctx64, B, vg, rho, wl.dt, steps, warmup)
    out["feedback"] = time_feedback(ctx64, B, vg, rho, box.n_cells)
    ctx64.destroy()
    del ctx64
    torch.cuda.empty_cache()
    ms32 = _time_steps(ctx32, B, vg, rho, wl.dt, steps, warmup)
    ctx32.destroy()
    out["fp64_value"] = round(wl.N * steps / (ms64 * 1e-3), 1)
    out["value"] = round(wl.N * steps / (ms32 * 1e-3), 1)
    out["speedup_vs_fp64"] = round(ms64 / ms32, 3)
    alg = algorithmic_bytes(3, wl.N, box.n_cells, fsz=4, msz=4, moves_in_push=moves_in_push(3, 0))
    out["hbm_frac_whole_step"] = round(alg["per_launch"] / (ms32 * 1e-3 / steps) / 1e9 / HBM_PEAK_GBS, 4)
    log(f"precision form: fp32 {out['value']:.4g}/s, fp64 {out['fp64_value']:.4g}/s, err {err}")
    return out


def run_batched_form(steps: int):
    """256 independent 2D boxes (sides log-uniform in 16..128, 4..64 per cell),
    tile picked by the library autotuner, steps run as one HIP graph launch;
    precision form, with the binary64 path on the same boxes for comparison."""
    import torch
    from paper_1412_1087_amd import mhdpic as M
    from paper_1412_1087_amd import workloads as W
    dev = torch.device("cuda:0")
    wls = W.batch2d(n_boxes=256, seed0=5000, n_steps=100)
    N = sum(w.N for w in wls)
    NC = sum(w.box.n_cells for w in wls)
    cat = lambda f: np.concatenate([f(w) for w in wls], axis=-1)
    B, vg, rho = _to(dev, cat(lambda w: w.B)), _to(dev, cat(lambda w: w.vg)), _to(dev, cat(lambda w: w.rho))
    x, v = _to(dev, cat(lambda w: w.x)), _to(dev, cat(lambda w: w.v))
    m, qm = _to(dev, cat(lambda w: w.m)), _to(dev, cat(lambda w: w.qm))
    dts = [w.dt for w in wls]
    nps = [w.N for w in wls]
    out = {"workload": "batch2d-256-boxes", "boxes": len(wls), "particles": N, "cells": NC,
           "steps": steps}
    res = {}

    def graph_ms(boxes, prec):
        ctx = M.Context(boxes, nps, x, v, m, qm, precision=prec)
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        ctx.step_graph(B, vg, rho, dts, steps, stream)  # capture + first launch
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.step_graph(B, vg, rho, dts, steps, stream)
        e1.record(stream)
        stream.synchronize()
        ctx.check(stream)
        ctx.destroy()
        return e0.elapsed_time(e1)

    for prec, name in ((M.FP32_MIXED, "fp32"), (M.FP64, "fp64")):
        boxes0 = [_gpu_box(w.box) for w in wls]
        tile, _ = M.autotune(boxes0, nps, x, v, m, qm, B, vg, rho, dts, n_steps=10, precision=prec)
        ms_one = graph_ms([_gpu_box(w.box, tile) for w in wls], prec)
        tiles, _ = M.autotune_classes(boxes0, nps, x, v, m, qm, B, vg, rho, dts, n_steps=10,
                                      precision=prec)
        ms_cls = graph_ms([_gpu_box(w.box, t) for w, t in zip(wls, tiles)], prec)
        shapes = sorted({t for t in tiles})
        by_class = {}
        for w, t in zip(wls, tiles):
            k = int(np.log2(w.box.n_cells) // 2)
            by_class.setdefault(f"4^{k}..4^{k + 1} cells", set()).add(t)
        best = min(ms_one, ms_cls)
        res[name] = dict(value=round(N * steps / (best * 1e-3), 1),
                         ms_per_step=round(best / steps, 5),
                         one_tile=dict(tile=list(tile), ms_per_step=round(ms_one / steps, 5)),
                         per_class=dict(tiles={k: [list(t) for t in sorted(v)] for k, v in by_class.items()},
                                        shapes=[list(t) for t in shapes],
                                        ms_per_step=round(ms_cls / steps, 5)),
                         per_class_gain=round(ms_one / ms_cls, 3))
        log(f"batched {name}: one tile {tile} {ms_one / steps:.4f} ms/step, per class "
            f"{shapes} {ms_cls / steps:.4f} ms/step")
    out["value"] = res["fp32"]["value"]
    out["fp32"] = res["fp32"]
    out["fp64_value"] = res["fp64"]["value"]
    out["fp64"] = res["fp64"]
    out["speedup_vs_fp64"] = round(res["fp32"]["value"] / res["fp64"]["value"], 3)
    out["launch"] = "one hipGraph launch per call of %d steps" % steps
    return out


# --------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample
# --------------------------------------------------------------------------

def _oracle_box(wl):
    from oracle import oracle as O
    return O.Box(ndim=wl.box.ndim, n=tuple(wl.box.n), dx=tuple(wl.box.dx), x0=tuple(wl.box.x0),
                 C=wl.box.C, qomc_gas=wl.box.qomc_gas, hall=wl.box.hall,
                 frac_bits=wl.box.frac_bits, max_move_cells=wl.box.max_move_cells)


def _oracle_part(conn, wl, idx, pin):
    """Child process: the oracle on one disjoint subset of the particles.  Each
    step it receives the n_CR, J_CR of all subsets (the Hall term's E depends
    on every particle), steps once and returns its own n_CR, J_CR, its
    accumulated -dM, -dE_k and the seconds the step took."""
    from oracle import oracle as O
    if pin is not None:
        os.sched_setaffinity(0, {pin})
    sysO = O.System(_oracle_box(wl), wl.x[:, idx].copy(), wl.v[:, idx].copy(), wl.m[idx].copy(),
                    wl.qm[idx].copy())
    conn.send(sysO.D[:4].copy())
    while True:
        nJ = conn.recv()
        if nJ is None:
            break
        sysO.D[:4] = nJ
        t0 = time.perf_counter()
        sysO.step(wl.B, wl.vg, wl.rho, wl.dt, 1)
        conn.send((sysO.D.copy(), time.perf_counter() - t0))
    conn.close()


def _oracle_parallel(wl, subsets, steps, pins):
    """The oracle over disjoint particle subsets, one process each, with the
    n_CR, J_CR summed over the subsets before every step.  Returns the summed
    deposits and the wall seconds of the slowest subset per step, summed."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")  # before the GPU is touched in this process
    procs, conns = [], []
    for k, idx in enumerate(subsets):
        a, b = ctx.Pipe()
        pr = ctx.Process(target=_oracle_part, args=(b, wl, idx, pins[k % len(pins)] if pins else None))
        pr.start()
        procs.append(pr)
        conns.append(a)
    nJ = sum(c.recv() for c in conns)
    wall = 0.0
    acc = None
    for _ in range(steps):
        for c in conns:
            c.send(nJ)
        outs = [c.recv() for c in conns]
        Ds = sum(o[0] for o in outs)
        wall += max(o[1] for o in outs)
        nJ = Ds[:4].copy()
        acc = Ds
    for c in conns:
        c.send(None)
    for pr in procs:
        pr.join()
    return acc, wall


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(wl, label: str, per_core: int = 65536, steps: int = 3, check_per: int = 4096):
    """The oracle as it stands (single-threaded binary64 C) on the host:
    1 core pinned, and all usable cores as one process per core on disjoint
    particle subsets (n_CR, J_CR summed across the subsets before each step,
    so the Hall field is that of all particles).  First, on a small set, the
    per-core split is checked to give the same integers as one process."""
    from oracle import oracle as O
    O.build(force=not os.path.exists(O.LIB))
    avail = sorted(os.sched_getaffinity(0))
    P = max(1, min(16, len(avail)))  # at most 16 host cores (the host's share per GPU)
    rng = np.random.default_rng(11)
    # equality of the split with one process on P * check_per particles
    pick = rng.choice(wl.N, size=min(wl.N, P * check_per), replace=False)
    one, _ = _oracle_parallel(wl, [pick], 2, None)
    split, _ = _oracle_parallel(wl, np.array_split(pick, P), 2, None)
    identical = bool((one == split).all())
    log(f"oracle split over {P} processes: deposits identical to one process: {identical}")
    # timing: per_core particles on each core
    sel = rng.choice(wl.N, size=min(wl.N, P * per_core), replace=False)
    _, wall1 = _oracle_parallel(wl, [sel[:per_core]], steps, [avail[0]])
    rate1 = per_core * steps / wall1
    _, wallP = _oracle_parallel(wl, np.array_split(sel, P), steps, avail[:P])
    rateP = len(sel) * steps / wallP
    log(f"oracle: 1 core {rate1:.4g} updates/s, {P} cores {rateP:.4g} updates/s ({cpu_model()})")
    return dict(value=rateP, unit="particle-updates/s", cores=P, kind="oracle",
                single_core_value=rate1, cpu_model=cpu_model(),
                split_deposits_identical_to_one_process=identical,
                sample=f"{per_core} particles per core drawn from {label} on its full grid, "
                       f"{steps} steps; one process per core, pinned, n_CR and J_CR summed "
                       f"over the processes before each step; 1-core leg: {per_core} "
                       f"particles on one pinned core")


# --------------------------------------------------------------------------

def load_traffic(label: str, per_launch_alg: float):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get(label)
    if not ent or ent.get("kernel_hash") != kernel_hash():
        return None
    return ent.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="bell3d")
    ap.add_argument("--tile", default="0,0,0")
    ap.add_argument("--moves", choices=("auto", "binning", "push"), default="auto",
                    help="where the particles move to their new slots (library default: auto)")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64",
                    help="fp32: the precision form on the chosen workload (profiling runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision-form and batched-form legs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 512 MiB device copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "shockwall":
        out = run_shock_wall_form(args.steps, args.warmup)
        print(json.dumps({"metric": "particle-updates/s (gather+push+deposit)", "value": out["value"],
                          "unit": "particle-updates/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "higher_is_better": True, "dtype": "f64",
                          "data": "synthetic (seeded; the shock set-up of Sec. 5)",
                          "config": {"workload": out["workload"]}, "shock_wall": out}), flush=True)
        return
    if args.workload == "precision":
        # the precision form alone (profiling runs): binary32 and binary64 on
        # the 128^3 box, the one-step error, and the feedback kernel
        out = run_precision_form(args.steps, args.warmup)
        print(json.dumps({"metric": "particle-updates/s (gather+push+deposit)", "value": out["value"],
                          "unit": "particle-updates/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "higher_is_better": True, "dtype": "f32",
                          "data": DATA_NOTE["bell3d128"],
                          "config": {"workload": out["workload"]}, "fp32_mixed": out}), flush=True)
        return
    if args.workload == "batch2d":
        # the batched form alone (profiling runs): steps as one graph launch
        out = run_batched_form(args.steps)
        print(json.dumps({"metric": "particle-updates/s (gather+push+deposit)", "value": out["value"],
                          "unit": "particle-updates/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": 0, "higher_is_better": True, "dtype": "f32",
                          "data": "synthetic (seeded; 256 gyration-test boxes)",
                          "config": {"workload": out["workload"]}, "batched": out}), flush=True)
        return
    wl, label = make_workload(args.workload)
    tile = tuple(int(a) for a in args.tile.split(","))
    # the oracle's processes are forked before this process touches the GPU
    cpu = None if args.no_cpu else run_cpu_baseline(wl, label)
    prec = 1 if args.precision == "fp32" else 0
    moves = {"auto": 0, "binning": 1, "push": 2}[args.moves]
    g = run_gpu(wl, args.steps, args.warmup, args.calibrate_copy, tile=tile, precision=prec,
                moves=moves)
    N = wl.N
    ms = g["ms"]
    value = N * args.steps / (ms * 1e-3)
    push_ms, push_n = g["push"]
    fsz = 4 if prec else 8
    mip = moves_in_push(wl.box.ndim, moves)
    alg = algorithmic_bytes(wl.box.ndim, N, g["n_cells"], fsz=fsz, msz=fsz, moves_in_push=mip)
    push_avg_s = push_ms * 1e-3 / max(push_n, 1)
    achieved = alg["per_launch"] / push_avg_s / 1e9
    traffic = load_traffic(label + ("/fp32" if prec else "") + (f"/moves-{args.moves}" if moves else ""),
                           alg["per_launch"])
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel="k_push_f32" if prec else "k_push_f64",
                    avg_launch_us=round(push_avg_s * 1e6, 2),
                    alg_bytes_per_launch=alg["per_launch"],
                    alg_bytes_per_particle=alg["per_particle"], alg_bytes_per_cell=alg["per_cell"])
    forms = None
    if not args.no_forms:
        import torch
        torch.cuda.empty_cache()
        forms = {"fp32_mixed": run_precision_form(100, 5), "batched": run_batched_form(100)}
        torch.cuda.empty_cache()
        forms["subcycled"] = run_subcycled_form(20, 2)
        torch.cuda.empty_cache()
        forms["strip2d"] = run_strip_form(20, 3)
        torch.cuda.empty_cache()
        forms["shock_wall"] = run_shock_wall_form(20, 3)
    # (a counter-collection run keeps its one calibration copy alone)
    copy_gbps = None if args.calibrate_copy else measure_copy_gbps()
    log(f"device copy: {copy_gbps} GB/s (read + written)")
    phases = {k: dict(ms=round(v[0], 3), launches=v[1]) for k, v in g["phases"].items()}
    phases["steps"] = g["breakdown_steps"]
    out = {
        "metric": "particle-updates/s (gather+push+deposit)",
        "value": round(value, 1),
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec else "f64",
        "data": DATA_NOTE.get(args.workload, "synthetic (seeded)"),
        "config": {"workload": label, "cells": g["n_cells"], "particles": N, "ndim": wl.box.ndim,
                   "hall": wl.box.hall, "C": wl.box.C, "dt": wl.dt, "tile": list(tile),
                   "precision": args.precision,
                   "particle_moves": "in_push" if mip else "in_binning"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases_ms_instrumented_pass": phases,
        "context_creation_ms": round(g["init_ms"], 2),
        "forms": forms,
        "hbm_frac_whole_step": round(
            (alg["per_launch"] / (ms * 1e-3 / args.steps)) / 1e9 / HBM_PEAK_GBS, 4),
        "copy_GBps_measured": copy_gbps,
        "checksum": g["checksum"],
        "kernel_hash": kernel_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
