"""Helpers shared by the GPU tests: run one workload through the HIP library
(via the C ABI binding) and through the oracle, from the same input bits."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_1412_1087_amd import workloads as W


PERIODIC_FACES = ((0, 0), (0, 0), (0, 0))


def oracle_box(spec: W.BoxSpec, boundary=PERIODIC_FACES) -> O.Box:
    return O.Box(ndim=spec.ndim, n=tuple(spec.n), dx=tuple(spec.dx), x0=tuple(spec.x0), C=spec.C,
                 qomc_gas=spec.qomc_gas, hall=spec.hall, frac_bits=spec.frac_bits,
                 max_move_cells=spec.max_move_cells, bc=tuple(tuple(f) for f in boundary))


def gpu_box(spec: W.BoxSpec, tile=(0, 0, 0), boundary=PERIODIC_FACES, capacity=0):
    from paper_1412_1087_amd import mhdpic as M
    return M.Box(ndim=spec.ndim, n=tuple(spec.n), dx=tuple(spec.dx), x0=tuple(spec.x0), C=spec.C,
                 qomc_gas=spec.qomc_gas, hall=spec.hall, frac_bits=spec.frac_bits,
                 max_move_cells=spec.max_move_cells, tile=tuple(tile),
                 boundary=tuple(tuple(f) for f in boundary), capacity=int(capacity))


def to_dev(a: np.ndarray, dev="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


class DeviceRun:
    """One or more workloads as the boxes of one GPU context."""

    def __init__(self, wls, tile=(0, 0, 0), precision=0, moves=0):
        import torch
        from paper_1412_1087_amd import mhdpic as M
        if not isinstance(wls, (list, tuple)):
            wls = [wls]
        self.wls = list(wls)
        # tile: one shape for every box, or a list with one shape per box
        tiles = tile if (len(tile) and isinstance(tile[0], (tuple, list))) else [tile] * len(self.wls)
        self.boxes = [gpu_box(w.box, t) for w, t in zip(self.wls, tiles)]
        x = np.concatenate([w.x for w in self.wls], axis=1)
        v = np.concatenate([w.v for w in self.wls], axis=1)
        m = np.concatenate([w.m for w in self.wls])
        qm = np.concatenate([w.qm for w in self.wls])
        self.B = to_dev(np.concatenate([w.B for w in self.wls], axis=1))
        self.vg = to_dev(np.concatenate([w.vg for w in self.wls], axis=1))
        self.rho = to_dev(np.concatenate([w.rho for w in self.wls]))
        self.ctx = M.Context(self.boxes, [w.N for w in self.wls], to_dev(x), to_dev(v), to_dev(m),
                             to_dev(qm), precision=precision)
        if moves:
            self.ctx.set_particle_moves(moves)
        self.cell_off = np.cumsum([0] + [w.box.n_cells for w in self.wls])
        self.part_off = np.cumsum([0] + [w.N for w in self.wls])
        torch.cuda.synchronize()

    def step(self, n_steps=1, dts=None, n_sub=1):
        import torch
        if dts is None:
            dts = [w.dt for w in self.wls]
        self.ctx.step(self.B, self.vg, self.rho, dts, n_steps, n_sub=n_sub)
        torch.cuda.synchronize()

    def deposits(self):
        import torch
        D = self.ctx.deposit_read().cpu().numpy()
        torch.cuda.synchronize()
        return [D[:, self.cell_off[b]:self.cell_off[b + 1]] for b in range(len(self.wls))]

    def particles(self):
        x, v = self.ctx.particles_read()
        x = x.cpu().numpy()
        v = v.cpu().numpy()
        return [(x[:, self.part_off[b]:self.part_off[b + 1]], v[:, self.part_off[b]:self.part_off[b + 1]])
                for b in range(len(self.wls))]


def oracle_run(wl: W.Workload) -> O.System:
    return O.System(oracle_box(wl.box), wl.x, wl.v, wl.m, wl.qm)


def assert_states_exact(x_g, v_g, x_o, v_o, tag=""):
    """Binary64 particle states equal the oracle's in every bit, element by
    element: both sides perform the same operations in the same order."""
    for name, a, b in (("position", x_g, x_o), ("velocity", v_g, v_o)):
        bad = np.argwhere(a != b)
        assert len(bad) == 0, (f"{tag}: {len(bad)} {name} components differ, first (comp, particle) "
                               f"{tuple(bad[0])}: {a[tuple(bad[0])]!r} vs {b[tuple(bad[0])]!r}")
