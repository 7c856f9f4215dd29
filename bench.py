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
    else:
        raise SystemExit(f"unknown workload {name}")
    return wl, label


def algorithmic_bytes(ndim: int, N: int, NC: int, fsz: int = 8, msz: int = 8) -> dict:
    """Bytes the fused push kernel must move per launch.

    Per particle: read cell index (4), offsets (ndim*fsz), four-velocity
    (3*fsz), m and q/mc (2*msz); write cell index, offsets, four-velocity.
    Per cell: read E and B (6*fsz), read+write the accumulated -dM, -dE_k
    (2*32), write n_CR, J_CR (32)."""
    p_read = 4 + ndim * fsz + 3 * fsz + 2 * msz
    p_write = 4 + ndim * fsz + 3 * fsz
    c_bytes = 6 * fsz + 64 + 32
    return dict(per_particle=p_read + p_write, per_cell=c_bytes,
                per_launch=N * (p_read + p_write) + NC * c_bytes)


# --------------------------------------------------------------------------
# GPU leg
# --------------------------------------------------------------------------

def run_gpu(wl, steps: int, warmup: int, calibrate_copy: bool, tile=(0, 0, 0), precision=0):
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
    ctx = M.Context([box], [wl.N], t(wl.x), t(wl.v), t(wl.m), t(wl.qm), precision=precision)
    torch.cuda.synchronize()
    log(f"init done: N={wl.N} cells={box.n_cells}")
    if warmup > 0:
        ctx.step(B, vg, rho, wl.dt, warmup)
    ctx.check()
    torch.cuda.synchronize()
    log("warmup done")

    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ctx.timing(True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    ctx.step(B, vg, rho, wl.dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    ctx.timing(False)
    phases = ctx.timing_read()
    ctx.check()
    ms = e0.elapsed_time(e1)
    log(f"timed {steps} steps: {ms:.3f} ms (events), {1e3 * (w1 - w0):.3f} ms (wall)")
    for p, (pm, pn) in phases.items():
        log(f"  phase {p:9s}: {pm:9.3f} ms over {pn} launches")
    D = ctx.deposit_read().cpu()
    ctx.destroy()
    return dict(ms=ms, wall_ms=1e3 * (w1 - w0), phases=phases, checksum=int(D.sum().item()),
                n_cells=box.n_cells)


# --------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample
# --------------------------------------------------------------------------

def run_cpu_baseline(wl, label: str, sample_div: int = 16, steps: int = 3):
    from oracle import oracle as O
    O.build(force=not os.path.exists(O.LIB))
    ns = max(1, wl.N // sample_div)
    box = O.Box(ndim=wl.box.ndim, n=tuple(wl.box.n), dx=tuple(wl.box.dx), x0=tuple(wl.box.x0),
                C=wl.box.C, qomc_gas=wl.box.qomc_gas, hall=wl.box.hall,
                frac_bits=wl.box.frac_bits, max_move_cells=wl.box.max_move_cells)
    sysO = O.System(box, wl.x[:, :ns].copy(), wl.v[:, :ns].copy(), wl.m[:ns].copy(),
                    wl.qm[:ns].copy())
    t0 = time.perf_counter()
    sysO.step(wl.B, wl.vg, wl.rho, wl.dt, steps)
    el = time.perf_counter() - t0
    rate = ns * steps / el
    log(f"oracle: {ns} particles x {steps} steps in {el:.2f} s -> {rate:.4g} updates/s")
    return dict(value=rate, unit="particle-updates/s", cores=1, kind="oracle",
                sample=f"first {ns} of {wl.N} particles of {label} on its full grid, "
                       f"{steps} steps, single thread, {el:.1f} s")


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
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 512 MiB device copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    wl, label = make_workload(args.workload)
    tile = tuple(int(a) for a in args.tile.split(","))
    g = run_gpu(wl, args.steps, args.warmup, args.calibrate_copy, tile=tile)
    N = wl.N
    ms = g["ms"]
    value = N * args.steps / (ms * 1e-3)
    push_ms, push_n = g["phases"]["push"]
    alg = algorithmic_bytes(wl.box.ndim, N, g["n_cells"])
    push_avg_s = push_ms * 1e-3 / max(push_n, 1)
    achieved = alg["per_launch"] / push_avg_s / 1e9
    traffic = load_traffic(label, alg["per_launch"])
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel="k_push_f64", avg_launch_us=round(push_avg_s * 1e6, 2),
                    alg_bytes_per_launch=alg["per_launch"],
                    alg_bytes_per_particle=alg["per_particle"], alg_bytes_per_cell=alg["per_cell"])
    cpu = None if args.no_cpu else run_cpu_baseline(wl, label)
    phases = {k: dict(ms=round(v[0], 3), launches=v[1]) for k, v in g["phases"].items()}
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
        "dtype": "f64",
        "data": "synthetic (seeded; shapes of the paper's Bell-instability test box)",
        "config": {"workload": label, "cells": g["n_cells"], "particles": N, "ndim": wl.box.ndim,
                   "hall": wl.box.hall, "C": wl.box.C, "dt": wl.dt, "tile": list(tile),
                   "precision": "fp64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases_ms": phases,
        "hbm_frac_whole_step": round(
            (alg["per_launch"] / (ms * 1e-3 / args.steps)) / 1e9 / HBM_PEAK_GBS, 4),
        "checksum": g["checksum"],
        "kernel_hash": kernel_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
