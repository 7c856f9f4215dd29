"""Precision form (binary32 offsets, velocities, fields, weights and rotation;
binary64 Lorentz factors, energy differences and fixed-point quantisation)
against the binary64 oracle.

Bounds follow from binary32 rounding, eps = 2^-24:
  * positions: the offset is stored in binary32 (|d| <= 1/2) and each drift
    adds a move of at most one cell, so one step is off by at most ~10 eps
    cells;
  * four-velocities: the kick and the rotation are a few binary32 operations
    on |v|, so ~20 eps |v|max;
  * n_CR, J_CR deposits: binary32 mass, weights (3 roundings) and u, so
    ~10 eps of the amount, plus the half-quantum roundings of up to 27
    contributions per particle on each side;
  * -dM, -dE_k: the differences v' - v of binary32 velocities carry the
    velocity error, ~40 eps |v|max (|v|max^2 for the energy) per unit mass.
Exact on the precision form's own numbers: the -dM integers sum to
round-half-even of -m (v' - v) 2^40 taken from its binary32 states.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1412_1087_amd import workloads as W  # noqa: E402

from gpu_helpers import DeviceRun, oracle_run  # noqa: E402

EPS32 = 2.0 ** -24


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rne(x: float) -> int:
    f = Fraction(x)
    fl = math.floor(f)
    r = f - fl
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and fl % 2 == 1):
        return fl + 1
    return fl


@pytest.mark.parametrize("make", [
    lambda: W.bell3d(n=16, ppc=4, seed=41),
    lambda: W.gyro2d(nx=32, ny=24, ppc=8, seed=42),
    lambda: W.shock2d(nx=256, ny=32, n_particles=256 * 32 * 4, seed=43),
])
def test_fp32_form_one_step_within_bounds(make):
    _need_gpu()
    wl = make()
    g = DeviceRun(wl, precision=1)
    o = oracle_run(wl)
    g.step(1)
    o.step(wl.B, wl.vg, wl.rho, wl.dt, 1)
    ((x, v),) = g.particles()
    (D,) = g.deposits()
    vmax = np.abs(o.v).max()
    L = np.array([wl.box.n[d] * wl.box.dx[d] for d in range(3)])[:, None]
    dx = x - o.positions()
    dx -= L * np.round(dx / L)
    assert np.abs(dx).max() <= 10 * EPS32 * max(wl.box.dx)
    assert np.abs(v - o.v).max() <= 20 * EPS32 * vmax
    Dn = o.D[0].astype(np.float64)
    slack = 2 * 27 * 0.5 * 64  # half-quantum roundings, generous count per cell
    for ch in range(4):
        scale = np.abs(o.D[ch]).max()
        assert np.abs(D[ch] - o.D[ch]).max() <= 10 * EPS32 * scale + slack, ch
    for ch in range(4, 7):
        assert np.abs(D[ch] - o.D[ch]).max() <= 40 * EPS32 * vmax * Dn.max() + slack, ch
    assert np.abs(D[7] - o.D[7]).max() <= 40 * EPS32 * vmax * vmax * Dn.max() + slack


def test_fp32_form_momentum_deposit_is_exact_on_its_own_states():
    _need_gpu()
    wl = W.gyro2d(nx=16, ny=16, ppc=6, seed=44)
    g = DeviceRun(wl, precision=1)
    v0 = wl.v.astype(np.float32).astype(np.float64)
    m32 = wl.m.astype(np.float32).astype(np.float64)
    g.step(1)
    ((x, v1),) = g.particles()
    (D,) = g.deposits()
    S = 2.0 ** 40
    for d in range(3):
        want = sum(_rne((-(m32[j] * (v1[d, j] - v0[d, j]))) * S) for j in range(wl.N))
        assert int(D[4 + d].sum()) == want


def test_fp32_form_is_deterministic_and_order_free():
    _need_gpu()
    wl = W.bell3d(n=(12, 10, 8), ppc=3, seed=45)
    a = DeviceRun(wl, precision=1)
    perm = np.random.default_rng(5).permutation(wl.N)
    wl2 = W.bell3d(n=(12, 10, 8), ppc=3, seed=45)
    wl2.x, wl2.v, wl2.m, wl2.qm = wl.x[:, perm], wl.v[:, perm], wl.m[perm], wl.qm[perm]
    b = DeviceRun(wl2, precision=1)
    a.step(4)
    b.step(4)
    (Da,) = a.deposits()
    (Db,) = b.deposits()
    assert (Da == Db).all()
    ((xa, va),) = a.particles()
    ((xb, vb),) = b.particles()
    assert (va[:, perm] == vb).all()


def test_fp32_form_multi_step_drift_is_bounded():
    """Orbits diverge over many steps; the precision form's error growth over
    20 steps stays at the level of binary32 rounding accumulated per step."""
    _need_gpu()
    wl = W.gyro2d(nx=32, ny=32, ppc=4, seed=46)
    g = DeviceRun(wl, precision=1)
    o = oracle_run(wl)
    g.step(20)
    o.step(wl.B, wl.vg, wl.rho, wl.dt, 20)
    ((x, v),) = g.particles()
    vmax = np.abs(o.v).max()
    assert np.abs(v - o.v).max() <= 20 * 20 * EPS32 * vmax * 10
