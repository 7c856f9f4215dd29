"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs: grid fields at cell centres (rho, v_g, B),
particle positions, four-velocities, masses and charge-to-mass ratios, and a
time step.  It holds none of the particle method's arithmetic, and both the
GPU library's tests and the oracle's tests take their inputs from here, so
both sides see the same bits.

Units are the paper's code units: rho0 = B0 = (q/mc) = 1, so the Alfven speed,
the ion inertial length and the ion cyclotron frequency are all 1 (Sec. 5).
Cells are one ion inertial length wide.

Workloads (sizes are parameters so that tests can shrink them):

* ``gyro2d`` -- 2D periodic box, uniform gas rho = 1 drifting at v_g = (0.1,0,0),
  B = (1, 0.5, 0) plus a 10 % divergence-free perturbation on integer modes
  1 <= |m| <= 4; isotropic CR three-velocities with |u| uniform in [1, 10];
  C = 20; Hall term off.  Default 32x32 cells, 16 particles per cell.
* ``bell3d`` -- 3D periodic box, gas at rest with rho = 1, B = (1,0,0) plus a 1 %
  perturbation on 1 <= |m| <= 8; a CR beam along B0 with four-velocity
  (gamma_D * 0.8 C, 0, 0) plus a Gaussian spread of 0.1 C per component;
  CR charge density 5 % of the gas ion charge (the Bell-instability setting of
  App. B.2); Hall term on; C = 20.  Default 64^3 cells, 16 per cell.
* ``shock2d`` -- 2D strip of 8192 x 32 cells shaped like the shock runs of Sec. 5:
  80 % of the particles in a band 0.25 L <= x < 0.35 L, 20 % elsewhere;
  v_g = (4,0,0) upstream of x = 0.3 L and (1,0,0) downstream (rho 1 and 4,
  mass-flux continuity); B at 45 degrees to x; isotropic momenta with
  f(p) ~ p^-4 for p in [1, 1000] m C (dN/dp ~ p^-2); Hall term off.
* ``batch2d`` -- many independent ``gyro2d`` boxes with side lengths and
  particles per cell drawn log-uniformly.

The time step follows the Larmor-time rule of App. A.4 with a gyro-phase of
0.05 per step: dt = 0.05 * min(gamma) / ((q/mc) max|B|), capped so that a
particle moving at C crosses at most ``max_move_cells`` cells per step.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class BoxSpec:
    ndim: int
    n: tuple                     # (nx, ny, nz); nz = 1 in 2D
    dx: tuple = (1.0, 1.0, 1.0)
    x0: tuple = (0.0, 0.0, 0.0)
    C: float = 20.0
    qomc_gas: float = 1.0
    hall: int = 0
    frac_bits: int = 40
    max_move_cells: int = 2

    @property
    def n_cells(self) -> int:
        return int(self.n[0] * self.n[1] * (self.n[2] if self.ndim == 3 else 1))

    @property
    def grid_shape(self):
        """numpy shape of one grid component, x fastest."""
        return (self.n[2], self.n[1], self.n[0]) if self.ndim == 3 else (self.n[1], self.n[0])


@dataclass
class Workload:
    name: str
    box: BoxSpec
    B: np.ndarray            # [3][cells]
    vg: np.ndarray           # [3][cells]
    rho: np.ndarray          # [cells]
    x: np.ndarray            # [3][N] global positions
    v: np.ndarray            # [3][N] four-velocities gamma*u
    m: np.ndarray            # [N]
    qm: np.ndarray           # [N]
    dt: float
    n_steps: int
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.m.shape[0])


# --------------------------------------------------------------------------
# helpers (input drawing only)
# --------------------------------------------------------------------------

def _cell_centres(box: BoxSpec):
    axes = []
    for d in range(box.ndim):
        axes.append(box.x0[d] + (np.arange(box.n[d]) + 0.5) * box.dx[d])
    return axes


def _perturbation(box: BoxSpec, rng, m_max: int, rms: float) -> np.ndarray:
    """Divergence-free field sum_m (k_m x a_m) cos(k_m . x + phi_m) over integer
    modes 1 <= |m| <= m_max in one half-space, evaluated at cell centres and
    scaled to the given rms magnitude.  Returns [3][cells]."""
    nd = box.ndim
    rngs = [np.arange(-m_max, m_max + 1)] * nd
    grids = np.meshgrid(*rngs, indexing="ij")
    ms = np.stack([g.ravel() for g in grids], axis=1)
    r2 = (ms ** 2).sum(axis=1)
    keep = (r2 >= 1) & (r2 <= m_max * m_max)
    # half-space: first nonzero component positive
    first = np.zeros(len(ms), dtype=bool)
    decided = np.zeros(len(ms), dtype=bool)
    for d in range(nd):
        pos = (~decided) & (ms[:, d] > 0)
        neg = (~decided) & (ms[:, d] < 0)
        first |= pos
        decided |= pos | neg
    ms = ms[keep & first]
    L = np.array([box.n[d] * box.dx[d] for d in range(nd)])
    spec = np.zeros((3,) + tuple(box.n[d] for d in range(nd)), dtype=np.complex128)
    for mv in ms:
        k = np.zeros(3)
        k[:nd] = 2.0 * np.pi * mv / L
        a = rng.normal(size=3)
        amp = np.cross(k, a)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        # cell centres sit half a cell above the FFT sample points
        shift = sum(k[d] * (box.x0[d] + 0.5 * box.dx[d]) for d in range(nd))
        idx = tuple(int(mv[d]) % box.n[d] for d in range(nd))
        spec[(slice(None),) + idx] += amp * np.exp(1j * (phi + shift))
    axes = tuple(range(1, nd + 1))
    ncell = int(np.prod([box.n[d] for d in range(nd)]))
    fld = np.real(np.fft.ifftn(spec, axes=axes)) * ncell  # [3][nx][ny](..)
    # reorder spatial axes to x fastest
    fld = np.transpose(fld, (0,) + tuple(range(nd, 0, -1)))
    fld = fld.reshape(3, -1)
    cur = np.sqrt(np.mean((fld ** 2).sum(axis=0)))
    if cur > 0:
        fld = fld * (rms / cur)
    return np.ascontiguousarray(fld)


def _cell_volume(box: BoxSpec) -> float:
    v = 1.0
    for d in range(box.ndim):
        v = v * box.dx[d]
    return v


def _isotropic(rng, mag: np.ndarray) -> np.ndarray:
    n = mag.shape[0]
    mu = rng.uniform(-1.0, 1.0, size=n)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n)
    s = np.sqrt(1.0 - mu * mu)
    return np.stack([mag * s * np.cos(ph), mag * s * np.sin(ph), mag * mu])


def _uniform_positions(box: BoxSpec, rng, N: int) -> np.ndarray:
    x = np.zeros((3, N))
    for d in range(box.ndim):
        x[d] = box.x0[d] + rng.uniform(0.0, box.n[d] * box.dx[d], size=N)
    return x


def choose_dt(box: BoxSpec, v: np.ndarray, qm: np.ndarray, B: np.ndarray, phase: float = 0.05):
    """Larmor-time rule (App. A.4) with the move limit as a cap."""
    gam = np.sqrt(1.0 + (v * v).sum(axis=0) / (box.C * box.C))
    bmax = float(np.sqrt((B * B).sum(axis=0)).max())
    qmax = float(np.abs(qm).max())
    dt = phase * float(gam.min()) / (qmax * bmax)
    dxmin = min(box.dx[d] for d in range(box.ndim))
    cap = 0.98 * box.max_move_cells * dxmin / box.C
    return min(dt, cap)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def gyro2d(nx=32, ny=32, ppc=16, seed=1001, C=20.0, n_steps=100, eta=2e-3,
           dx=(1.0, 1.0, 1.0), x0=(0.0, 0.0, 0.0)) -> Workload:
    box = BoxSpec(ndim=2, n=(nx, ny, 1), dx=tuple(dx), x0=tuple(x0), C=C, hall=0)
    rng = np.random.default_rng(seed)
    nc = box.n_cells
    rho = np.ones(nc)
    vg = np.zeros((3, nc))
    vg[0] = 0.1
    B0 = np.array([1.0, 0.5, 0.0])
    B = B0[:, None] + _perturbation(box, rng, 4, 0.1 * float(np.linalg.norm(B0)))
    N = nc * ppc
    x = _uniform_positions(box, rng, N)
    umag = rng.uniform(1.0, 10.0, size=N)
    u = _isotropic(rng, umag)
    gam = 1.0 / np.sqrt(1.0 - (umag / C) ** 2)
    v = u * gam[None, :]
    # CR mass density eta * rho: m = eta rho dV / ppc
    m = np.full(N, eta * _cell_volume(box) / ppc)
    qm = np.ones(N)
    dt = choose_dt(box, v, qm, B)
    return Workload("gyro2d", box, np.ascontiguousarray(B), vg, rho, x, np.ascontiguousarray(v), m,
                    qm, dt, n_steps, dict(ppc=ppc, seed=seed))


def bell3d(n=64, ppc=16, seed=2001, C=20.0, n_steps=200, ncr_frac=0.05, hall=1,
           dx=(1.0, 1.0, 1.0), x0=(0.0, 0.0, 0.0)) -> Workload:
    if isinstance(n, int):
        n = (n, n, n)
    box = BoxSpec(ndim=3, n=tuple(n), dx=tuple(dx), x0=tuple(x0), C=C, hall=hall)
    rng = np.random.default_rng(seed)
    nc = box.n_cells
    rho = np.ones(nc)
    vg = np.zeros((3, nc))
    B0 = np.array([1.0, 0.0, 0.0])
    B = B0[:, None] + _perturbation(box, rng, 8, 0.01)
    N = nc * ppc
    x = _uniform_positions(box, rng, N)
    vD = 0.8 * C
    gD = 1.0 / np.sqrt(1.0 - 0.64)
    v = rng.normal(0.0, 0.1 * C, size=(3, N))
    v[0] += gD * vD
    qm = np.ones(N)
    # n_CR = (q/mc) m ppc / dV = ncr_frac * (q/mc)_g rho
    m = np.full(N, ncr_frac * _cell_volume(box) / ppc)
    dt = choose_dt(box, v, qm, B)
    return Workload("bell3d", box, np.ascontiguousarray(B), vg, rho, x, np.ascontiguousarray(v), m,
                    qm, dt, n_steps, dict(ppc=ppc, seed=seed))


def shock2d(nx=8192, ny=32, n_particles=16_777_216, seed=3001, C=20.0, n_steps=100,
            eta=2e-3, band_frac=0.8) -> Workload:
    box = BoxSpec(ndim=2, n=(nx, ny, 1), C=C, hall=0)
    rng = np.random.default_rng(seed)
    nc = box.n_cells
    L = nx * box.dx[0]
    xc = (np.arange(nx) + 0.5) * box.dx[0]
    up = np.broadcast_to(xc[None, :] < 0.3 * L, (ny, nx)).ravel()
    rho = np.where(up, 1.0, 4.0)
    vg = np.zeros((3, nc))
    vg[0] = np.where(up, 4.0, 1.0)
    B = np.zeros((3, nc))
    B[0] = 1.0 / np.sqrt(2.0)
    B[1] = 1.0 / np.sqrt(2.0)
    N = int(n_particles)
    nb = int(round(band_frac * N))
    x = np.zeros((3, N))
    x[0, :nb] = rng.uniform(0.25 * L, 0.35 * L, size=nb)
    # the rest: uniform over the strip outside the band
    r = rng.uniform(0.0, 0.9 * L, size=N - nb)
    x[0, nb:] = np.where(r < 0.25 * L, r, r + 0.1 * L)
    x[1] = rng.uniform(0.0, ny * box.dx[1], size=N)
    perm = rng.permutation(N)
    x = np.ascontiguousarray(x[:, perm])
    # dN/dp ~ p^-2 on [1, 1000]: inverse CDF
    U = rng.uniform(0.0, 1.0, size=N)
    p = 1.0 / (1.0 - U * (1.0 - 1.0 / 1000.0))
    v = _isotropic(rng, p * C)
    qm = np.ones(N)
    ppc_mean = N / nc
    m = np.full(N, eta * 1.0 * 1.0 / ppc_mean)
    dt = choose_dt(box, v, qm, B)
    return Workload("shock2d", box, B, vg, rho, x, np.ascontiguousarray(v), m, qm, dt, n_steps,
                    dict(seed=seed, band_frac=band_frac))


# faces of a box (per axis, low and high): periodic, reflecting, absorbing
PERIODIC, REFLECT, ABSORB = 0, 1, 2


@dataclass
class ShockSetup:
    """The shock set-up of Sec. 5 at test size: a conducting (reflecting) wall
    at x = x0, an inflow (absorbing) face at the far end, periodic in y; the
    downstream gas at rest with density 4 rho0 behind the shock front x_s,
    the upstream gas flowing at -v0 toward the wall; B along the shock normal
    (a parallel shock); CRs injected at the front each step."""
    box: BoxSpec
    boundary: tuple
    B: np.ndarray
    vg: np.ndarray
    rho: np.ndarray
    x_s: float          # shock front
    v0: float           # upstream flow speed (M_A v_A)
    v_sh: float         # front speed in the downstream frame, v0/3
    dt: float
    eta: float          # injected CR mass per unit swept gas mass


def shock_wall2d(nx=96, ny=8, dx=12.0, M_A=30.0, C=None, seed=7001, eta=2e-3,
                 front_cell=32) -> ShockSetup:
    """Gas and fields of the shock set-up, with the front at cell front_cell.
    C defaults to the paper's reduced speed of light 10 sqrt(2) v0 (run
    R2-REL); dt keeps a particle moving at C within the move limit."""
    v0 = float(M_A)
    if C is None:
        C = 10.0 * np.sqrt(2.0) * v0
    box = BoxSpec(ndim=2, n=(nx, ny, 1), dx=(dx, dx, 1.0), C=C, hall=0)
    nc = box.n_cells
    xc = (np.arange(nx) + 0.5) * dx
    x_s = front_cell * dx
    up = np.broadcast_to(xc[None, :] >= x_s, (ny, nx)).ravel()
    rho = np.where(up, 1.0, 4.0)
    vg = np.zeros((3, nc))
    vg[0] = np.where(up, -v0, 0.0)
    rng = np.random.default_rng(seed)
    B = np.zeros((3, nc))
    B[0] = 1.0
    # a little transverse field, as the Bell modes the shock drives
    B[1] = 0.05 * rng.normal(size=nc)
    B[2] = 0.05 * rng.normal(size=nc)
    dt = 0.9 * 2.0 * dx / C
    return ShockSetup(box, ((REFLECT, ABSORB), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)),
                      B, vg, rho, x_s, v0, v0 / 3.0, dt, eta)


def shock_injection(setup: ShockSetup, n: int, t: float, seed: int, ppc_up=4.0):
    """One step's injected CRs (Sec. 5): at the front x_s + v_sh t, uniform
    in y, isotropic in the frame moving with the front with kinetic energy
    10 E_sh (E_sh = v0^2/2 per unit mass), boosted to the downstream frame at
    the reduced speed of light; their total mass is eta times the gas mass the
    front swept in one step, shared by n particles.  Returns x, v ([3][n]),
    m, qm ([n]) and the tags (the injection time t)."""
    rng = np.random.default_rng(seed)
    box = setup.box
    C = box.C
    x = np.zeros((3, n))
    # within a cell behind the front (the front moves less than a cell a step)
    front = setup.x_s + setup.v_sh * t
    x[0] = box.x0[0] + front - rng.uniform(0.0, box.dx[0], size=n)
    x[1] = box.x0[1] + rng.uniform(0.0, box.n[1] * box.dx[1], size=n)
    Esh = 0.5 * setup.v0 ** 2
    g = 1.0 + 10.0 * Esh / (C * C)
    vmag = C * np.sqrt(g * g - 1.0)
    v = _isotropic(rng, np.full(n, vmag))
    b = setup.v_sh / C
    gb = 1.0 / np.sqrt(1.0 - b * b)
    vx = gb * (v[0] + b * g * C)
    v[0] = vx
    # swept gas: rho0 (v0 + v_sh) per unit area and time, over the box height
    swept = 1.0 * (setup.v0 + setup.v_sh) * setup.dt * box.n[1] * box.dx[1]
    m = np.full(n, setup.eta * swept / n)
    qm = np.ones(n)
    return (np.ascontiguousarray(x), np.ascontiguousarray(v), m, qm, np.full(n, float(t)))


def shock_population(setup: ShockSetup, N: int, seed: int, width_cells: float = 170.0):
    """CRs accumulated around the front by the time of a run's middle: uniform
    within width_cells cells on either side of x_s (about 2000 ion inertial
    lengths at 12 per cell, the CR precursor of Sec. 6), uniform in y,
    isotropic, with |v| log-uniform between the injection four-velocity
    (10 E_sh) and 20 times it, each carrying the injected mass of one particle
    of a 4-per-cell injection.  Returns x, v, m, qm, tags (tag: 0, injected
    before the run's start)."""
    rng = np.random.default_rng(seed)
    box = setup.box
    C = box.C
    x = np.zeros((3, N))
    lo = max(0.0, setup.x_s - width_cells * box.dx[0])
    hi = min(box.n[0] * box.dx[0], setup.x_s + width_cells * box.dx[0])
    x[0] = box.x0[0] + rng.uniform(lo, hi, size=N)
    x[1] = box.x0[1] + rng.uniform(0.0, box.n[1] * box.dx[1], size=N)
    Esh = 0.5 * setup.v0 ** 2
    g = 1.0 + 10.0 * Esh / (C * C)
    v_inj = C * np.sqrt(g * g - 1.0)
    vmag = v_inj * np.exp(rng.uniform(0.0, np.log(20.0), size=N))
    v = _isotropic(rng, vmag)
    # 4 particles per cell at rho0 = 1: each carries eta rho0 dV / 4
    m = np.full(N, setup.eta * _cell_volume(box) / 4.0)
    return (np.ascontiguousarray(x), np.ascontiguousarray(v), m, np.ones(N), np.zeros(N))


def batch2d(n_boxes=256, seed0=5000, side=(16, 128), ppc=(4, 64), C=20.0, n_steps=100):
    """Independent gyro2d boxes with log-uniform sides and particles per cell."""
    out = []
    for b in range(n_boxes):
        rng = np.random.default_rng(seed0 + b)
        lx = int(round(np.exp(rng.uniform(np.log(side[0]), np.log(side[1])))))
        ly = int(round(np.exp(rng.uniform(np.log(side[0]), np.log(side[1])))))
        pc = int(round(np.exp(rng.uniform(np.log(ppc[0]), np.log(ppc[1])))))
        out.append(gyro2d(nx=lx, ny=ly, ppc=pc, seed=seed0 * 7 + b, C=C, n_steps=n_steps))
    return out
