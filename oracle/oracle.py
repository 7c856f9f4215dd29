"""Python driver for the C reference oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this module.  The GPU library never does.

The oracle is plain single-threaded binary64 C (``mhdpic_oracle.c``); this
module builds it with gcc and exposes numpy-friendly wrappers.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mhdpic_oracle.c")
LIB = os.path.join(HERE, "libmhdpic_oracle.so")

OK, EINVAL, ERANGE, ENONFINITE = 0, -1, -4, -5
PERIODIC, REFLECT, ABSORB = 0, 1, 2


def build(force: bool = True) -> str:
    """Compiles the oracle with contraction off and no fast-math."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=HERE)
        os.replace(tmp, LIB)
    return LIB


class OracleBox(ct.Structure):
    _fields_ = [("ndim", ct.c_int32), ("n", ct.c_int32 * 3), ("dx", ct.c_double * 3),
                ("x0", ct.c_double * 3), ("C", ct.c_double), ("qomc_gas", ct.c_double),
                ("hall", ct.c_int32), ("frac_bits", ct.c_int32),
                ("max_move_cells", ct.c_int32), ("bc", ct.c_int32 * 6)]


class OracleParticles(ct.Structure):
    _fields_ = [("N", ct.c_int64), ("cell", ct.POINTER(ct.c_int32)),
                ("delta", ct.POINTER(ct.c_double)), ("v", ct.POINTER(ct.c_double)),
                ("m", ct.POINTER(ct.c_double)), ("qm", ct.POINTER(ct.c_double)),
                ("alive", ct.POINTER(ct.c_int32))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ct.CDLL(LIB)
        dp = ct.POINTER(ct.c_double)
        i64p = ct.POINTER(ct.c_int64)
        L.oracle_rne_product.restype = ct.c_int64
        L.oracle_rne_product.argtypes = [ct.c_double, ct.c_double]
        L.oracle_quantize.restype = ct.c_int64
        L.oracle_quantize.argtypes = [ct.c_double, ct.c_double]
        L.oracle_lorentz.restype = None
        L.oracle_lorentz.argtypes = [dp, ct.c_double, dp, dp, dp]
        L.oracle_clean_E.restype = None
        L.oracle_clean_E.argtypes = [dp, dp]
        L.oracle_boris_kick_rotate_kick.restype = None
        L.oracle_boris_kick_rotate_kick.argtypes = [dp, dp, dp, ct.c_double, ct.c_double, dp]
        L.oracle_tsc_weights.restype = None
        L.oracle_tsc_weights.argtypes = [ct.c_double, dp]
        L.oracle_fieldprep.restype = ct.c_int
        L.oracle_fieldprep.argtypes = [ct.POINTER(OracleBox), dp, dp, dp, i64p, dp]
        L.oracle_init.restype = ct.c_int
        L.oracle_init.argtypes = [ct.POINTER(OracleBox), ct.POINTER(OracleParticles), dp, dp, dp,
                                  dp, i64p]
        L.oracle_add.restype = ct.c_int
        L.oracle_add.argtypes = [ct.POINTER(OracleBox), ct.POINTER(OracleParticles), ct.c_int64,
                                 dp, dp, dp, dp, i64p]
        L.oracle_remove.restype = ct.c_int
        L.oracle_remove.argtypes = [ct.POINTER(OracleBox), ct.POINTER(OracleParticles), ct.c_int64,
                                    i64p]
        L.oracle_check_dt.restype = ct.c_int
        L.oracle_check_dt.argtypes = [ct.POINTER(OracleBox), ct.c_double]
        L.oracle_step.restype = ct.c_int
        L.oracle_step.argtypes = [ct.POINTER(OracleBox), ct.POINTER(OracleParticles), dp, dp, dp,
                                  ct.c_double, ct.c_int, i64p, i64p, dp]
        L.oracle_step_sub.restype = ct.c_int
        L.oracle_step_sub.argtypes = [ct.POINTER(OracleBox), ct.POINTER(OracleParticles), dp, dp, dp,
                                      ct.c_double, ct.c_int, ct.c_int, i64p, i64p, dp]
        L.oracle_feedback.restype = ct.c_int
        L.oracle_feedback.argtypes = [ct.POINTER(OracleBox), dp, dp, dp, i64p, dp]
        L.oracle_positions.restype = ct.c_int
        L.oracle_positions.argtypes = [ct.POINTER(OracleBox), ct.POINTER(OracleParticles), dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _i64p(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_int64))


def _i32p(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_int32))


# --------------------------------------------------------------------------
# scalar pieces
# --------------------------------------------------------------------------

def rne_product(a: float, b: float) -> int:
    return int(lib().oracle_rne_product(float(a), float(b)))


def quantize(W: float, V: float) -> int:
    return int(lib().oracle_quantize(float(W), float(V)))


def lorentz(v, C):
    v = np.ascontiguousarray(v, dtype=np.float64)
    g = ct.c_double()
    u = np.zeros(3)
    ek = ct.c_double()
    lib().oracle_lorentz(_dp(v), float(C), ct.byref(g), _dp(u), ct.byref(ek))
    return g.value, u, ek.value


def clean_E(E, B):
    E = np.array(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    lib().oracle_clean_E(_dp(E), _dp(B))
    return E


def boris_kick_rotate_kick(v, E, B, hq, C):
    v = np.ascontiguousarray(v, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    out = np.zeros(3)
    lib().oracle_boris_kick_rotate_kick(_dp(v), _dp(E), _dp(B), float(hq), float(C), _dp(out))
    return out


def tsc_weights(d: float):
    w = np.zeros(3)
    lib().oracle_tsc_weights(float(d), _dp(w))
    return w


# --------------------------------------------------------------------------
# the particle system of one periodic box
# --------------------------------------------------------------------------

@dataclass
class Box:
    ndim: int
    n: tuple
    dx: tuple = (1.0, 1.0, 1.0)
    x0: tuple = (0.0, 0.0, 0.0)
    C: float = 20.0
    qomc_gas: float = 1.0
    hall: int = 0
    frac_bits: int = 40
    max_move_cells: int = 2
    # per axis (low, high): PERIODIC, REFLECT or ABSORB
    bc: tuple = ((PERIODIC, PERIODIC), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC))

    @property
    def n_cells(self) -> int:
        n = list(self.n) + [1] * (3 - len(self.n))
        return int(n[0] * n[1] * (n[2] if self.ndim == 3 else 1))

    def c_struct(self) -> OracleBox:
        n = list(self.n) + [1] * (3 - len(self.n))
        if self.ndim == 2:
            n[2] = 1
        b = OracleBox()
        b.ndim = self.ndim
        b.n = (ct.c_int32 * 3)(*n)
        b.dx = (ct.c_double * 3)(*[float(a) for a in self.dx])
        b.x0 = (ct.c_double * 3)(*[float(a) for a in self.x0])
        b.C = float(self.C)
        b.qomc_gas = float(self.qomc_gas)
        b.hall = int(self.hall)
        b.frac_bits = int(self.frac_bits)
        b.max_move_cells = int(self.max_move_cells)
        b.bc = (ct.c_int32 * 6)(*[int(f) for ax in self.bc for f in ax])
        return b


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned {code}")
        self.code = code


class System:
    """One box of particles advanced by the oracle.

    Arrays follow the [comp][N] / [comp][cells] layout; grid arrays are
    flattened with x fastest.  ``D`` holds the 8 deposit channels:
    n_CR, J_CR (x,y,z) at the current positions, then the accumulated
    -dM (x,y,z) and -dE_k.  Particle j keeps index j for its whole life;
    ``alive[j]`` is 0 once it has left through an absorbing face or been
    removed.  Added particles take the next indices.
    """

    def __init__(self, box: Box, x, v, m, qm):
        self.box = box
        self._cb = box.c_struct()
        nc = box.n_cells
        self.N = 0
        self.cell = np.zeros((3, 0), dtype=np.int32)
        self.delta = np.zeros((3, 0), dtype=np.float64)
        self.v = np.zeros((3, 0), dtype=np.float64)
        self.m = np.zeros(0, dtype=np.float64)
        self.qm = np.zeros(0, dtype=np.float64)
        self.alive = np.zeros(0, dtype=np.int32)
        self.D = np.zeros((8, nc), dtype=np.int64)
        self._nJ = np.zeros((4, nc), dtype=np.int64)
        self.E = np.zeros((3, nc), dtype=np.float64)
        self._add(x, v, m, qm, init=True)

    def _grow(self, k: int):
        N = self.N + k
        def ext(a, shape):
            b = np.zeros(shape, dtype=a.dtype)
            if a.ndim == 2:
                b[:, :self.N] = a
            else:
                b[:self.N] = a
            return b
        self.cell = ext(self.cell, (3, N))
        self.delta = ext(self.delta, (3, N))
        self.v = ext(self.v, (3, N))
        self.m = ext(self.m, (N,))
        self.qm = ext(self.qm, (N,))
        self.alive = ext(self.alive, (N,))
        self.N = N
        self._P = OracleParticles(N, _i32p(self.cell), _dp(self.delta), _dp(self.v), _dp(self.m),
                                  _dp(self.qm), _i32p(self.alive))

    def _add(self, x, v, m, qm, init=False):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(3, -1)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(3, -1)
        m = np.ascontiguousarray(m, dtype=np.float64)
        qm = np.ascontiguousarray(qm, dtype=np.float64)
        first = self.N
        self._grow(x.shape[1])
        if init:
            rc = lib().oracle_init(ct.byref(self._cb), ct.byref(self._P), _dp(x), _dp(v), _dp(m),
                                   _dp(qm), _i64p(self.D))
        else:
            rc = lib().oracle_add(ct.byref(self._cb), ct.byref(self._P), first, _dp(x), _dp(v),
                                  _dp(m), _dp(qm), _i64p(self.D))
        if rc:
            raise OracleError(rc)
        return np.arange(first, self.N)

    def inject(self, x, v, m, qm):
        """Adds particles (global positions, four-velocities); their n_CR, J_CR
        join D[0..3].  Returns their indices."""
        return self._add(x, v, m, qm)

    def remove(self, idx):
        """Removes particles: their n_CR, J_CR leave D[0..3]."""
        for j in np.atleast_1d(idx):
            rc = lib().oracle_remove(ct.byref(self._cb), ct.byref(self._P), int(j), _i64p(self.D))
            if rc:
                raise OracleError(rc)

    def step(self, B, vg, rho, dt: float, n_steps: int = 1, n_sub: int = 1):
        """n_steps MHD steps of dt, each of n_sub particle steps of dt/n_sub
        with the field prepared at the MHD step's start."""
        B = np.ascontiguousarray(B, dtype=np.float64)
        vg = np.ascontiguousarray(vg, dtype=np.float64)
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        rc = lib().oracle_step_sub(ct.byref(self._cb), ct.byref(self._P), _dp(B), _dp(vg),
                                   _dp(rho), float(dt), int(n_steps), int(n_sub),
                                   _i64p(self.D), _i64p(self._nJ), _dp(self.E))
        if rc:
            raise OracleError(rc)

    def fieldprep(self, B, vg, rho):
        B = np.ascontiguousarray(B, dtype=np.float64)
        vg = np.ascontiguousarray(vg, dtype=np.float64)
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        E = np.zeros((3, self.box.n_cells))
        rc = lib().oracle_fieldprep(ct.byref(self._cb), _dp(B), _dp(vg), _dp(rho),
                                    _i64p(self.D), _dp(E))
        if rc:
            raise OracleError(rc)
        return E

    def feedback(self, B, vg, rho):
        """The 10 cell-centred predictor feedback channels from the current
        n_CR, J_CR (see the function feedback)."""
        return feedback(self.box, B, vg, rho, self.D)

    def positions(self):
        x = np.zeros((3, self.N))
        lib().oracle_positions(ct.byref(self._cb), ct.byref(self._P), _dp(x))
        return x

    def clear_accumulated(self):
        self.D[4:] = 0


def fieldprep(box: Box, B, vg, rho, D):
    cb = box.c_struct()
    B = np.ascontiguousarray(B, dtype=np.float64)
    vg = np.ascontiguousarray(vg, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.int64)
    E = np.zeros((3, box.n_cells))
    rc = lib().oracle_fieldprep(ct.byref(cb), _dp(B), _dp(vg), _dp(rho), _i64p(D), _dp(E))
    if rc:
        raise OracleError(rc)
    return E


def feedback(box: Box, B, vg, rho, D):
    """[10][cells]: -F_CR, -(1-R) J_CR.E0, (E-E0)xB, Lambda (App. A.3 predictor)."""
    cb = box.c_struct()
    B = np.ascontiguousarray(B, dtype=np.float64)
    vg = np.ascontiguousarray(vg, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.int64)
    out = np.zeros((10, box.n_cells))
    rc = lib().oracle_feedback(ct.byref(cb), _dp(B), _dp(vg), _dp(rho), _i64p(D), _dp(out))
    if rc:
        raise OracleError(rc)
    return out


def check_dt(box: Box, dt: float) -> int:
    cb = box.c_struct()
    return int(lib().oracle_check_dt(ct.byref(cb), float(dt)))
