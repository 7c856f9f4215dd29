"""Thin ctypes binding of ``libmhdpic.so`` (the C ABI in ``include/mhdpic.h``).

Argument marshalling only: every step of the particle update runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.  If
the library has not been built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass, field
from typing import Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# MHDPIC_LIB selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("MHDPIC_LIB") or os.path.join(HERE, "libmhdpic.so")

OK, EINVAL, ENOMEM, EDEVICE, ERANGE, ENONFINITE, ESTATE, ENOTSUP = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32_MIXED = 0, 1
PERIODIC, REFLECT, ABSORB = 0, 1, 2
MOVES_AUTO, MOVES_IN_BINNING, MOVES_IN_PUSH = 0, 1, 2

EXPORTED = [
    "mhdpic_workspace_size", "mhdpic_init", "mhdpic_step", "mhdpic_deposit_read",
    "mhdpic_particles_read", "mhdpic_check", "mhdpic_destroy", "mhdpic_last_error",
    "mhdpic_selftest_arith", "mhdpic_timing_enable", "mhdpic_timing_read",
    "mhdpic_step_graph", "mhdpic_autotune_workspace_size", "mhdpic_autotune", "mhdpic_step_sub",
    "mhdpic_feedback", "mhdpic_step_graph_sub", "mhdpic_advance", "mhdpic_advance_noalloc",
    "mhdpic_particles_read_ids", "mhdpic_counts", "mhdpic_inject", "mhdpic_remove_tagged",
    "mhdpic_autotune_classes_workspace_size", "mhdpic_autotune_classes", "mhdpic_set_particle_moves",
]


class MhdpicBox(ct.Structure):
    _fields_ = [("ndim", ct.c_int32), ("n", ct.c_int32 * 3), ("dx", ct.c_double * 3),
                ("x0", ct.c_double * 3), ("C", ct.c_double), ("qomc_gas", ct.c_double),
                ("hall", ct.c_int32), ("frac_bits", ct.c_int32), ("max_move_cells", ct.c_int32),
                ("tile", ct.c_int32 * 3), ("boundary", ct.c_int32 * 6), ("capacity", ct.c_int64)]


class MhdpicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mhdpic error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1412_1087_amd/build.py")
        L = ct.CDLL(LIB_PATH)
        vp, sz = ct.c_void_p, ct.c_size_t
        L.mhdpic_workspace_size.restype = ct.c_int
        L.mhdpic_workspace_size.argtypes = [ct.POINTER(MhdpicBox), ct.c_int32,
                                            ct.POINTER(ct.c_int64), ct.c_int32, ct.POINTER(sz)]
        L.mhdpic_init.restype = ct.c_int
        L.mhdpic_init.argtypes = [ct.POINTER(MhdpicBox), ct.c_int32, ct.POINTER(ct.c_int64),
                                  ct.c_int32, vp, vp, vp, vp, vp, sz, vp, ct.POINTER(vp)]
        L.mhdpic_step.restype = ct.c_int
        L.mhdpic_step.argtypes = [vp, vp, vp, vp, ct.POINTER(ct.c_double), ct.c_int32, vp]
        L.mhdpic_step_sub.restype = ct.c_int
        L.mhdpic_step_sub.argtypes = [vp, vp, vp, vp, ct.POINTER(ct.c_double), ct.c_int32,
                                      ct.c_int32, vp]
        L.mhdpic_step_graph_sub.restype = ct.c_int
        L.mhdpic_step_graph_sub.argtypes = [vp, vp, vp, vp, ct.POINTER(ct.c_double), ct.c_int32,
                                            ct.c_int32, vp]
        L.mhdpic_feedback.restype = ct.c_int
        L.mhdpic_feedback.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mhdpic_deposit_read.restype = ct.c_int
        L.mhdpic_deposit_read.argtypes = [vp, vp, ct.c_int32, vp]
        L.mhdpic_particles_read.restype = ct.c_int
        L.mhdpic_particles_read.argtypes = [vp, vp, vp, vp]
        L.mhdpic_particles_read_ids.restype = ct.c_int
        L.mhdpic_particles_read_ids.argtypes = [vp, vp, vp, vp, vp, ct.c_int64,
                                                ct.POINTER(ct.c_int64), vp]
        L.mhdpic_counts.restype = ct.c_int
        L.mhdpic_counts.argtypes = [vp, ct.POINTER(ct.c_int64), vp]
        L.mhdpic_inject.restype = ct.c_int
        L.mhdpic_inject.argtypes = [vp, ct.POINTER(ct.c_int64), vp, vp, vp, vp, vp, vp]
        L.mhdpic_remove_tagged.restype = ct.c_int
        L.mhdpic_remove_tagged.argtypes = [vp, ct.c_double, ct.c_double, vp]
        L.mhdpic_check.restype = ct.c_int
        L.mhdpic_check.argtypes = [vp, vp]
        L.mhdpic_destroy.restype = ct.c_int
        L.mhdpic_destroy.argtypes = [vp]
        L.mhdpic_last_error.restype = ct.c_char_p
        L.mhdpic_last_error.argtypes = []
        L.mhdpic_timing_enable.restype = ct.c_int
        L.mhdpic_timing_enable.argtypes = [vp, ct.c_int32]
        L.mhdpic_set_particle_moves.restype = ct.c_int
        L.mhdpic_set_particle_moves.argtypes = [vp, ct.c_int32]
        L.mhdpic_timing_read.restype = ct.c_int
        L.mhdpic_timing_read.argtypes = [vp, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64)]
        L.mhdpic_step_graph.restype = ct.c_int
        L.mhdpic_step_graph.argtypes = [vp, vp, vp, vp, ct.POINTER(ct.c_double), ct.c_int32, vp]
        L.mhdpic_autotune_workspace_size.restype = ct.c_int
        L.mhdpic_autotune_workspace_size.argtypes = [ct.POINTER(MhdpicBox), ct.c_int32,
                                                     ct.POINTER(ct.c_int64), ct.c_int32,
                                                     ct.POINTER(sz)]
        L.mhdpic_autotune.restype = ct.c_int
        L.mhdpic_autotune.argtypes = [ct.POINTER(MhdpicBox), ct.c_int32, ct.POINTER(ct.c_int64),
                                      ct.c_int32, vp, vp, vp, vp, vp, vp, vp,
                                      ct.POINTER(ct.c_double), ct.c_int32, vp, sz, vp,
                                      ct.POINTER(ct.c_int32), ct.POINTER(ct.c_double)]
        L.mhdpic_autotune_classes_workspace_size.restype = ct.c_int
        L.mhdpic_autotune_classes_workspace_size.argtypes = [ct.POINTER(MhdpicBox), ct.c_int32,
                                                             ct.POINTER(ct.c_int64), ct.c_int32,
                                                             ct.POINTER(sz)]
        L.mhdpic_autotune_classes.restype = ct.c_int
        L.mhdpic_autotune_classes.argtypes = [ct.POINTER(MhdpicBox), ct.c_int32,
                                              ct.POINTER(ct.c_int64), ct.c_int32, vp, vp, vp, vp,
                                              vp, vp, vp, ct.POINTER(ct.c_double), ct.c_int32, vp,
                                              sz, vp, ct.POINTER(ct.c_int32),
                                              ct.POINTER(ct.c_double)]
        L.mhdpic_advance.restype = ct.c_int
        L.mhdpic_advance.argtypes = [ct.POINTER(MhdpicBox), ct.c_int32, ct.POINTER(ct.c_int64),
                                     ct.c_int32, vp, vp, vp, vp, vp, vp, vp,
                                     ct.POINTER(ct.c_double), ct.c_int32, ct.c_int32, vp, vp, vp,
                                     vp, sz, vp]
        L.mhdpic_advance_noalloc.restype = ct.c_int
        L.mhdpic_advance_noalloc.argtypes = [ct.POINTER(MhdpicBox), ct.c_int32,
                                             ct.POINTER(ct.c_int64), ct.c_int32, vp, vp, vp, vp, vp,
                                             vp, vp, ct.POINTER(ct.c_double), ct.c_int32,
                                             ct.c_int32, vp, vp, vp, vp]
        L.mhdpic_selftest_arith.restype = ct.c_int
        L.mhdpic_selftest_arith.argtypes = [vp, vp, vp, vp, ct.c_int64, vp]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise MhdpicError(rc, lib().mhdpic_last_error().decode())


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ct.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


@dataclass
class Box:
    """Host description of one periodic box (mirrors ``mhdpic_box``)."""
    ndim: int
    n: Sequence[int]
    dx: Sequence[float] = (1.0, 1.0, 1.0)
    x0: Sequence[float] = (0.0, 0.0, 0.0)
    C: float = 20.0
    qomc_gas: float = 1.0
    hall: int = 0
    frac_bits: int = 40
    max_move_cells: int = 2
    tile: Sequence[int] = field(default_factory=lambda: (0, 0, 0))
    # per axis (low, high): PERIODIC, REFLECT or ABSORB
    boundary: Sequence[Sequence[int]] = ((0, 0), (0, 0), (0, 0))
    capacity: int = 0  # particle slots for injection (0: the initial count)

    def c_struct(self) -> MhdpicBox:
        n = list(self.n) + [1] * (3 - len(self.n))
        if self.ndim == 2:
            n[2] = 1
        b = MhdpicBox()
        b.ndim = self.ndim
        b.n = (ct.c_int32 * 3)(*n)
        b.dx = (ct.c_double * 3)(*[float(a) for a in self.dx])
        b.x0 = (ct.c_double * 3)(*[float(a) for a in self.x0])
        b.C = float(self.C)
        b.qomc_gas = float(self.qomc_gas)
        b.hall = int(self.hall)
        b.frac_bits = int(self.frac_bits)
        b.max_move_cells = int(self.max_move_cells)
        t = list(self.tile) + [0] * (3 - len(self.tile))
        b.tile = (ct.c_int32 * 3)(*t)
        b.boundary = (ct.c_int32 * 6)(*[int(f) for ax in self.boundary for f in ax])
        b.capacity = int(self.capacity)
        return b

    @property
    def n_cells(self) -> int:
        return int(self.n[0] * self.n[1] * (self.n[2] if self.ndim == 3 else 1))


def _boxes_array(boxes: Sequence[Box]):
    arr = (MhdpicBox * len(boxes))()
    for i, b in enumerate(boxes):
        arr[i] = b.c_struct()
    return arr


def workspace_size(boxes: Sequence[Box], n_particles: Sequence[int], precision: int = FP64) -> int:
    arr = _boxes_array(boxes)
    npart = (ct.c_int64 * len(boxes))(*[int(a) for a in n_particles])
    out = ct.c_size_t()
    _check(lib().mhdpic_workspace_size(arr, len(boxes), npart, int(precision), ct.byref(out)))
    return int(out.value)


class Context:
    """A set of boxes and their CR particles resident on one GPU."""

    def __init__(self, boxes: Sequence[Box], n_particles: Sequence[int], x: torch.Tensor,
                 v: torch.Tensor, m: torch.Tensor, qm: torch.Tensor, precision: int = FP64,
                 stream=None):
        self.boxes = list(boxes)
        self.n_particles = [int(a) for a in n_particles]
        self.N = sum(self.n_particles)
        self.n_cells = sum(b.n_cells for b in self.boxes)
        self.precision = precision
        dev = x.device
        for t in (x, v, m, qm):
            assert t.dtype == torch.float64 and t.device == dev
        nbytes = workspace_size(self.boxes, self.n_particles, precision)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        self._arr = _boxes_array(self.boxes)
        npart = (ct.c_int64 * len(self.boxes))(*self.n_particles)
        h = ct.c_void_p()
        _check(lib().mhdpic_init(self._arr, len(self.boxes), npart, int(precision), _ptr(x), _ptr(v),
                                 _ptr(m), _ptr(qm), _ptr(self.workspace), nbytes, _stream(stream),
                                 ct.byref(h)))
        self._h = h
        self.device = dev

    def step(self, B: torch.Tensor, vg: torch.Tensor, rho: torch.Tensor | None, dt, n_steps: int = 1,
             stream=None, n_sub: int = 1):
        """n_steps steps of dt; with n_sub > 1 each takes n_sub particle
        sub-steps of dt/n_sub through the field formed at its start."""
        if isinstance(dt, (int, float)):
            dt = [float(dt)] * len(self.boxes)
        dts = (ct.c_double * len(self.boxes))(*[float(a) for a in dt])
        if n_sub == 1:
            _check(lib().mhdpic_step(self._h, _ptr(B), _ptr(vg), _ptr(rho), dts, int(n_steps),
                                     _stream(stream)))
        else:
            _check(lib().mhdpic_step_sub(self._h, _ptr(B), _ptr(vg), _ptr(rho), dts, int(n_steps),
                                         int(n_sub), _stream(stream)))

    def step_graph(self, B: torch.Tensor, vg: torch.Tensor, rho: torch.Tensor | None, dt,
                   n_steps: int, stream, n_sub: int = 1):
        """n_steps (even) steps as one cached HIP graph launch on a non-default
        stream; with n_sub > 1 each step takes n_sub particle sub-steps."""
        if isinstance(dt, (int, float)):
            dt = [float(dt)] * len(self.boxes)
        dts = (ct.c_double * len(self.boxes))(*[float(a) for a in dt])
        if n_sub == 1:
            _check(lib().mhdpic_step_graph(self._h, _ptr(B), _ptr(vg), _ptr(rho), dts,
                                           int(n_steps), _stream(stream)))
        else:
            _check(lib().mhdpic_step_graph_sub(self._h, _ptr(B), _ptr(vg), _ptr(rho), dts,
                                               int(n_steps), int(n_sub), _stream(stream)))

    def feedback(self, B: torch.Tensor, vg: torch.Tensor, rho: torch.Tensor,
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """[10][cells] doubles: -F_CR, -(1-R) J_CR.E0, (E-E0)xB, Lambda from the
        current n_CR, J_CR (the predictor step's cell-centred feedback)."""
        if out is None:
            out = torch.empty((10, self.n_cells), dtype=torch.float64, device=self.device)
        _check(lib().mhdpic_feedback(self._h, _ptr(B), _ptr(vg), _ptr(rho), _ptr(out),
                                     _stream(stream)))
        return out

    def deposit_read(self, reset_accumulated: bool = False, out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty((8, self.n_cells), dtype=torch.int64, device=self.device)
        _check(lib().mhdpic_deposit_read(self._h, _ptr(out), int(bool(reset_accumulated)),
                                         _stream(stream)))
        return out

    def particles_read(self, stream=None):
        x = torch.empty((3, self.N), dtype=torch.float64, device=self.device)
        v = torch.empty((3, self.N), dtype=torch.float64, device=self.device)
        _check(lib().mhdpic_particles_read(self._h, _ptr(x), _ptr(v), _stream(stream)))
        return x, v

    def particles_read_ids(self, n_max: int | None = None, stream=None):
        """Current particles (compacted, any order): x, v [3][n], ids [n] and
        tags [n] (+inf for particles without one)."""
        if n_max is None:
            n_max = sum(self.counts(stream))
        x = torch.empty((3, max(n_max, 1)), dtype=torch.float64, device=self.device)
        v = torch.empty_like(x)
        ids = torch.empty(max(n_max, 1), dtype=torch.int32, device=self.device)
        tags = torch.empty(max(n_max, 1), dtype=torch.float64, device=self.device)
        n = ct.c_int64()
        _check(lib().mhdpic_particles_read_ids(self._h, _ptr(x), _ptr(v), _ptr(ids), _ptr(tags),
                                               int(n_max), ct.byref(n), _stream(stream)))
        k = int(n.value)
        return x[:, :k], v[:, :k], ids[:k], tags[:k]

    def counts(self, stream=None):
        """Current particles per box."""
        out = (ct.c_int64 * len(self.boxes))()
        _check(lib().mhdpic_counts(self._h, out, _stream(stream)))
        return [int(a) for a in out]

    def inject(self, n_new, x, v, m, qm, tags=None, stream=None):
        """Adds particles: n_new per box, global positions and four-velocities
        [3][sum], m, qm (and optional tags) [sum]."""
        nn = (ct.c_int64 * len(self.boxes))(*[int(a) for a in n_new])
        _check(lib().mhdpic_inject(self._h, nn, _ptr(x), _ptr(v), _ptr(m), _ptr(qm), _ptr(tags),
                                   _stream(stream)))

    def remove_tagged(self, t_cut: float, t_now: float, stream=None):
        """Removes particles with tag < t_cut once t_now >= 2 tag (Sec. 5)."""
        _check(lib().mhdpic_remove_tagged(self._h, float(t_cut), float(t_now), _stream(stream)))

    def set_particle_moves(self, where: int):
        """Where a step moves the particles to their new slots: MOVES_AUTO,
        MOVES_IN_BINNING or MOVES_IN_PUSH (same results, different cost)."""
        _check(lib().mhdpic_set_particle_moves(self._h, int(where)))

    PHASES = ("bin", "fieldprep", "push", "clear")

    def timing(self, enable: bool, phases=None):
        """Event timing of the named phases (all four if None) from now on;
        timing(False) stops."""
        mask = 0
        if enable:
            names = self.PHASES if phases is None else phases
            for p in names:
                mask |= 1 << self.PHASES.index(p)
        _check(lib().mhdpic_timing_enable(self._h, mask))

    def timing_read(self) -> dict:
        ms = (ct.c_double * 4)()
        n = (ct.c_int64 * 4)()
        _check(lib().mhdpic_timing_read(self._h, ms, n))
        return {p: (float(ms[k]), int(n[k])) for k, p in enumerate(self.PHASES)}

    def check(self, stream=None):
        _check(lib().mhdpic_check(self._h, _stream(stream)))

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mhdpic_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def autotune(boxes: Sequence[Box], n_particles: Sequence[int], x, v, m, qm, B, vg, rho, dt,
             n_steps: int = 10, precision: int = FP64, stream=None):
    """Tile shape with the shortest measured step for this workload (library autotuner)."""
    arr = _boxes_array(boxes)
    npart = (ct.c_int64 * len(boxes))(*[int(a) for a in n_particles])
    size = ct.c_size_t()
    _check(lib().mhdpic_autotune_workspace_size(arr, len(boxes), npart, int(precision),
                                                ct.byref(size)))
    ws = torch.empty(max(int(size.value), 256), dtype=torch.uint8, device=x.device)
    if isinstance(dt, (int, float)):
        dt = [float(dt)] * len(boxes)
    dts = (ct.c_double * len(boxes))(*[float(a) for a in dt])
    tile = (ct.c_int32 * 3)()
    ms = ct.c_double()
    _check(lib().mhdpic_autotune(arr, len(boxes), npart, int(precision), _ptr(x), _ptr(v), _ptr(m),
                                 _ptr(qm), _ptr(B), _ptr(vg), _ptr(rho), dts, int(n_steps),
                                 _ptr(ws), int(size.value), _stream(stream), tile, ct.byref(ms)))
    del ws
    return (int(tile[0]), int(tile[1]), int(tile[2])), float(ms.value)


def autotune_classes(boxes: Sequence[Box], n_particles: Sequence[int], x, v, m, qm, B, vg, rho,
                     dt, n_steps: int = 10, precision: int = FP64, stream=None):
    """Tile shape per box (per box-size class) and the chosen step time in ms
    (library autotuner of the batched form)."""
    arr = _boxes_array(boxes)
    nb = len(boxes)
    npart = (ct.c_int64 * nb)(*[int(a) for a in n_particles])
    size = ct.c_size_t()
    _check(lib().mhdpic_autotune_classes_workspace_size(arr, nb, npart, int(precision),
                                                        ct.byref(size)))
    ws = torch.empty(max(int(size.value), 256), dtype=torch.uint8, device=x.device)
    if isinstance(dt, (int, float)):
        dt = [float(dt)] * nb
    dts = (ct.c_double * nb)(*[float(a) for a in dt])
    tiles = (ct.c_int32 * (3 * nb))()
    ms = ct.c_double()
    _check(lib().mhdpic_autotune_classes(arr, nb, npart, int(precision), _ptr(x), _ptr(v), _ptr(m),
                                         _ptr(qm), _ptr(B), _ptr(vg), _ptr(rho), dts, int(n_steps),
                                         _ptr(ws), int(size.value), _stream(stream), tiles,
                                         ct.byref(ms)))
    del ws
    return [tuple(int(tiles[3 * b + k]) for k in range(3)) for b in range(nb)], float(ms.value)


def advance(boxes: Sequence[Box], n_particles: Sequence[int], x, v, m, qm, B, vg, rho, dt,
            n_steps: int, n_sub: int = 1, precision: int = FP64, workspace=None, stream=None,
            noalloc: bool = False):
    """One call without a context (mhdpic_advance): returns the final global
    positions and four-velocities [3][N] and the deposits [8][cells].  The
    workspace (a uint8 device tensor of at least workspace_size bytes) is
    allocated here if not given.  With noalloc, mhdpic_advance_noalloc runs
    the same step in the library's static scratch (no workspace)."""
    arr = _boxes_array(boxes)
    nps = [int(a) for a in n_particles]
    npart = (ct.c_int64 * len(boxes))(*nps)
    N = sum(nps)
    NC = sum(b.n_cells for b in boxes)
    dev = x.device
    if isinstance(dt, (int, float)):
        dt = [float(dt)] * len(boxes)
    dts = (ct.c_double * len(boxes))(*[float(a) for a in dt])
    x_out = torch.empty((3, N), dtype=torch.float64, device=dev)
    v_out = torch.empty((3, N), dtype=torch.float64, device=dev)
    D = torch.empty((8, NC), dtype=torch.int64, device=dev)
    if noalloc:
        _check(lib().mhdpic_advance_noalloc(arr, len(boxes), npart, int(precision), _ptr(x), _ptr(v),
                                            _ptr(m), _ptr(qm), _ptr(B), _ptr(vg), _ptr(rho), dts,
                                            int(n_steps), int(n_sub), _ptr(x_out), _ptr(v_out),
                                            _ptr(D), _stream(stream)))
        return x_out, v_out, D
    if workspace is None:
        workspace = torch.empty(max(workspace_size(boxes, nps, precision), 256), dtype=torch.uint8,
                                device=dev)
    _check(lib().mhdpic_advance(arr, len(boxes), npart, int(precision), _ptr(x), _ptr(v), _ptr(m),
                                _ptr(qm), _ptr(B), _ptr(vg), _ptr(rho), dts, int(n_steps),
                                int(n_sub), _ptr(x_out), _ptr(v_out), _ptr(D), _ptr(workspace),
                                workspace.numel(), _stream(stream)))
    return x_out, v_out, D


def selftest_arith(a: torch.Tensor, b: torch.Tensor, c: torch.Tensor, stream=None) -> torch.Tensor:
    n = a.numel()
    out = torch.empty((4, n), dtype=torch.float64, device=a.device)
    _check(lib().mhdpic_selftest_arith(_ptr(a), _ptr(b), _ptr(c), _ptr(out), n, _stream(stream)))
    return out
