"""Pins of the oracle's box geometry: a lower corner x0 away from zero and a
different cell size along each axis.

Each test compares the oracle with something fixed independently of it:
exact rational arithmetic for the cell index and offset of a position, the
quadratic B-spline for the deposit weights, closed-form orbits in physical
units (the gyration circle and the E x B drift), and the closed-form
cell-centred field of a uniform beam (Sec. 2.1, eq. emfcr1), which fixes the
cell volume.  A dimension mix-up, an origin added instead of subtracted, or a
cell volume missing a factor fails one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O

X0 = (-3.7, 11.2, 0.5)
DX = (0.5, 2.0, 1.25)


def _bspline2(x: Fraction) -> Fraction:
    ax = abs(x)
    if ax <= Fraction(1, 2):
        return Fraction(3, 4) - ax * ax
    if ax <= Fraction(3, 2):
        return (Fraction(3, 2) - ax) ** 2 / 2
    return Fraction(0)


def _rne(x: Fraction) -> int:
    fl = math.floor(x)
    r = x - fl
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and fl % 2 == 1):
        return fl + 1
    return fl


def _uniform(box, Bvec, vgvec, rho=1.0):
    nc = box.n_cells
    B = np.repeat(np.asarray(Bvec, float)[:, None], nc, axis=1).copy()
    vg = np.repeat(np.asarray(vgvec, float)[:, None], nc, axis=1).copy()
    return B, vg, np.full(nc, float(rho))


def _unwrap(track, L):
    tr = np.array(track)
    out = tr.copy()
    for i in range(1, len(tr)):
        d = tr[i] - tr[i - 1]
        d -= L * np.round(d / L)
        out[i] = out[i - 1] + d
    return out


# --------------------------------------------------------------------------
# position <-> (cell, offset)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ndim", [2, 3])
def test_cell_index_and_offset_of_positions_exact(ndim):
    """The cell of a position is floor((x - x0)/dx) mod n per axis, and the
    offset from that cell's centre is (x - x0)/dx - cell - 1/2, both taken
    with exact rationals; the read-back x0 + dx((i + 1/2) + d) returns the
    input position to rounding."""
    n = (6, 5, 4) if ndim == 3 else (7, 3, 1)
    box = O.Box(ndim=ndim, n=n, dx=DX, x0=X0, C=20.0)
    rng = np.random.default_rng(71)
    N = 400
    x = np.zeros((3, N))
    for d in range(ndim):
        # positions over three periods on either side of the box
        x[d] = X0[d] + rng.uniform(-3 * n[d], 4 * n[d], size=N) * DX[d]
    v = rng.normal(size=(3, N))
    sys = O.System(box, x, v, np.full(N, 1e-3), np.ones(N))
    for j in range(N):
        for d in range(ndim):
            s = (Fraction(float(x[d, j])) - Fraction(X0[d])) / Fraction(DX[d])
            fl = math.floor(s)
            frac = s - fl
            if min(frac, 1 - frac) < Fraction(1, 10 ** 9):
                continue  # within rounding of a cell face: either cell is right
            assert sys.cell[d, j] == fl % n[d], (j, d)
            assert abs(Fraction(float(sys.delta[d, j])) - (frac - Fraction(1, 2))) < Fraction(1, 10 ** 12)
    xb = sys.positions()
    L = np.array([n[d] * DX[d] for d in range(3)])[:, None]
    dd = xb[:ndim] - x[:ndim]
    dd -= L[:ndim] * np.round(dd / L[:ndim])
    scale = np.abs(x[:ndim]).max() + np.abs(np.array(X0)).max()
    assert np.abs(dd).max() <= 8 * np.finfo(float).eps * scale


def test_positions_too_far_from_the_origin_are_rejected():
    box = O.Box(ndim=2, n=(4, 4, 1), dx=(0.5, 2.0, 1.0), x0=(-3.7, 11.2, 0.0), C=20.0)
    v = np.zeros((3, 1))
    m, qm = np.array([1e-3]), np.array([1.0])
    ok = np.array([[-3.7 + 0.5 * (2.0 ** 31 - 2)], [12.0], [0.0]])
    O.System(box, ok, v, m, qm)
    for far in ([-3.7 + 0.5 * 2.0 ** 31 + 1.0, 12.0], [0.0, 11.2 - 2.0 * (2.0 ** 31 + 2)]):
        x = np.array([[far[0]], [far[1]], [0.0]])
        with pytest.raises(O.OracleError) as e:
            O.System(box, x, v, m, qm)
        assert e.value.code == O.ERANGE


# --------------------------------------------------------------------------
# deposit placement and the cell volume
# --------------------------------------------------------------------------

def test_single_particle_deposit_at_offset_origin_anisotropic_cells():
    """Each of the 27 stencil cells receives the B-spline weight of the
    particle's distance from the cell centre, measured in that axis's cell
    size from the box origin, times the amount."""
    n = (5, 4, 3)
    box = O.Box(ndim=3, n=n, dx=DX, x0=X0, C=20.0)
    nc = box.n_cells
    # physical position: cell (4, 0, 2) plus offsets, so the stencil wraps in x and z
    cell = (4, 0, 2)
    off = (Fraction(17, 64), Fraction(-23, 64), Fraction(5, 16))
    pos = [Fraction(X0[d]) + Fraction(DX[d]) * (cell[d] + Fraction(1, 2) + off[d]) for d in range(3)]
    x = np.array([[float(p)] for p in pos])
    sys = O.System(box, x, np.array([[1.0], [-2.0], [0.5]]), np.array([0.0123]), np.array([1.7]))
    S = 2.0 ** 40
    Vn = (1.7 * 0.0123) * S
    xr = [Fraction(float(p)) for p in pos]
    expect = np.zeros(nc)
    for cz in range(n[2]):
        for cy in range(n[1]):
            for cx in range(n[0]):
                w = Fraction(1)
                for d, c in enumerate((cx, cy, cz)):
                    centre = Fraction(X0[d]) + Fraction(DX[d]) * (c + Fraction(1, 2))
                    dist = (xr[d] - centre) / Fraction(DX[d])
                    dist -= n[d] * round(dist / n[d])
                    w *= _bspline2(dist)
                expect[(cz * n[1] + cy) * n[0] + cx] = float(w * Fraction(Vn))
    D = sys.D[0]
    assert D.sum() == _rne(Fraction(Vn))
    nz = np.flatnonzero(expect)
    assert len(nz) == 27 and set(np.flatnonzero(D)) <= set(nz)
    centre = (cell[2] * n[1] + cell[1]) * n[0] + cell[0]
    err = np.abs(D - expect)
    assert np.delete(err, centre).max() <= 0.5 + Vn * 2.0 ** -48
    assert err[centre] <= 0.5 * 27 + Vn * 2.0 ** -47


def test_uniform_beam_fixes_the_cell_volume_in_field_and_feedback():
    """One particle per cell at the same offset and four-velocity: n_CR is
    (q/mc) m / dV with dV = dx dy dz and u_CR = u, so the cell-centred field
    is E = -[(1-R) v_g + R u] x B (eq. emfcr1) and Lambda = R (u - v_g)/v_A
    (eq. lambda) in closed form."""
    n = (4, 3, 2)
    box = O.Box(ndim=3, n=n, dx=DX, x0=X0, C=20.0, hall=1, qomc_gas=1.3)
    nc = box.n_cells
    cz, cy, cx = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    cells = (cx.ravel(), cy.ravel(), cz.ravel())
    off = (0.21, -0.33, 0.07)
    x = np.stack([X0[d] + DX[d] * (cells[d] + 0.5 + off[d]) for d in range(3)])
    N = x.shape[1]
    vb = np.array([3.0, -1.5, 2.0])
    v = np.repeat(vb[:, None], N, axis=1).copy()
    m, qm = np.full(N, 0.04), np.full(N, 0.9)
    sys = O.System(box, x, v, m, qm)
    dV = DX[0] * DX[1] * DX[2]
    nq = 0.9 * 0.04 / dV
    gam = math.sqrt(1.0 + vb @ vb / 400.0)
    u = vb / gam
    Bv, gv, rho = np.array([0.8, 0.3, -0.4]), np.array([0.2, 0.1, -0.05]), 1.7
    B, vg, rhoa = _uniform(box, Bv, gv, rho)
    ng = 1.3 * rho
    R = nq / (ng + nq)
    Ewant = -np.cross((1 - R) * gv + R * u, Bv)
    E = sys.fieldprep(B, vg, rhoa)
    tol = 1e-9 * np.linalg.norm(Ewant)
    assert np.abs(E - Ewant[:, None]).max() <= tol
    F = sys.feedback(B, vg, rhoa)
    vA = np.linalg.norm(Bv) / math.sqrt(rho)
    Lam = R * (u - gv) / vA
    assert np.abs(F[7:10] - Lam[:, None]).max() <= 1e-9 * np.abs(Lam).max()
    # -F_CR = -(1-R)(n E0 + J x B) with J = n u
    E0 = -np.cross(gv, Bv)
    Fcr = (1 - R) * (nq * E0 + np.cross(nq * u, Bv))
    assert np.abs(F[0:3] + Fcr[:, None]).max() <= 1e-9 * np.abs(Fcr).max()


# --------------------------------------------------------------------------
# orbits in physical units
# --------------------------------------------------------------------------

def test_gyration_circle_2d_offset_origin_anisotropic_cells():
    """B along z: full-step positions lie on a circle of radius R_L about the
    guiding centre, in physical units, although the cells are four times as
    tall as they are wide."""
    C = 10.0
    n = (48, 12, 1)
    box = O.Box(ndim=2, n=n, dx=(0.5, 2.0, 1.0), x0=(-3.7, 11.2, 0.0), C=C)
    B, vg, rho = _uniform(box, (0.0, 0.0, 1.0), (0.0, 0.0, 0.0))
    L = np.array([n[0] * 0.5, n[1] * 2.0])
    x = np.array([[-3.7 + 0.37 * L[0]], [11.2 + 0.61 * L[1]], [0.0]])
    vperp = 3.0
    sys = O.System(box, x, np.array([[vperp], [0.0], [0.0]]), np.array([1.0]), np.array([1.0]))
    RL = vperp
    centre = np.array([x[0, 0], x[1, 0] - RL])
    track = [sys.positions()[:2, 0].copy()]
    for _ in range(300):
        sys.step(B, vg, rho, 0.09, 1)
        track.append(sys.positions()[:2, 0].copy())
    tr = _unwrap(track, L)
    r = np.sqrt(((tr - centre[None, :]) ** 2).sum(axis=1))
    assert np.abs(r / RL - 1.0).max() < 1e-11
    # the orbit covers the full circle, so both axes' scales enter
    assert tr[:, 0].max() - tr[:, 0].min() > 1.99 * RL
    assert tr[:, 1].max() - tr[:, 1].min() > 1.99 * RL


def test_gyration_3d_helix_offset_origin_anisotropic_cells():
    """B along y, cells (0.5, 2, 1.25): the orbit is a circle of radius R_L in
    the z-x plane, and the particle drifts along y at its parallel velocity,
    which the rotation leaves exactly unchanged."""
    C = 10.0
    n = (40, 8, 16)
    box = O.Box(ndim=3, n=n, dx=DX, x0=X0, C=C)
    B, vg, rho = _uniform(box, (0.0, 1.0, 0.0), (0.0, 0.0, 0.0))
    L = np.array([n[d] * DX[d] for d in range(3)])
    x0p = np.array([X0[0] + 0.4 * L[0], X0[1] + 0.2 * L[1], X0[2] + 0.7 * L[2]])
    vpar, vperp = 0.9, 2.5
    v = np.array([[vperp], [vpar], [0.0]])
    sys = O.System(box, x0p[:, None].copy(), v, np.array([1.0]), np.array([1.0]))
    g = math.sqrt(1.0 + (vpar ** 2 + vperp ** 2) / C ** 2)
    RL = vperp  # v_perp / ((q/mc) B), four-velocity units
    # u x B for u along +x and B along +y points along +z: centre at z + R_L
    centre = np.array([x0p[0], x0p[2] + RL])
    dt = 0.09
    track = [sys.positions()[:, 0].copy()]
    for _ in range(250):
        sys.step(B, vg, rho, dt, 1)
        assert sys.v[1, 0] == vpar
        track.append(sys.positions()[:, 0].copy())
    tr = _unwrap(track, L)
    r = np.hypot(tr[:, 0] - centre[0], tr[:, 2] - centre[1])
    assert np.abs(r / RL - 1.0).max() < 1e-11
    ypred = x0p[1] + np.arange(len(tr)) * dt * (vpar / g)
    assert np.abs(tr[:, 1] - ypred).max() < 1e-10 * L[1]


def test_exb_drift_oblique_anisotropic_cells():
    """Uniform B along z and v_g = (0.3, 0.4, 0): the guiding centre moves at
    v_g, along both axes, to second order in dt, with cells four times as tall
    as they are wide (large cells keep C dt within the move limit at C = 100)."""
    C = 100.0
    vd = np.array([0.3, 0.4])

    def slope(dt):
        n = (32, 8, 1)
        box = O.Box(ndim=2, n=n, dx=(32.0, 128.0, 1.0), x0=(-37.0, 112.0, 0.0), C=C)
        B, vg, rho = _uniform(box, (0.0, 0.0, 1.0), (vd[0], vd[1], 0.0))
        sys = O.System(box, np.array([[200.0], [600.0], [0.0]]), np.array([[2.0], [0.0], [0.0]]),
                       np.array([1.0]), np.array([1.0]))
        L = np.array([n[0] * 32.0, n[1] * 128.0])

        def gc():
            xx = sys.positions()[:2, 0]
            vv = sys.v[:, 0]
            gg = math.sqrt(1.0 + vv @ vv / C ** 2)
            w = vv / gg - np.array([vd[0], vd[1], 0.0])
            return np.array([xx[0] + w[1] * gg, xx[1] - w[0] * gg])

        nst = int(round(200.0 / dt))
        tr = [gc()]
        for _ in range(nst):
            sys.step(B, vg, rho, dt, 1)
            tr.append(gc())
        tr = _unwrap(tr, L)
        t = np.arange(len(tr)) * dt
        return np.array([np.polyfit(t, tr[:, k], 1)[0] for k in range(2)])

    e1, e2 = np.abs(slope(0.4) - vd), np.abs(slope(0.2) - vd)
    assert (e1 < 1e-6).all()
    # second order in dt along each axis
    assert (3.5 < e1 / e2).all() and (e1 / e2 < 4.5).all()
