"""Pins of the oracle's non-periodic faces, added particles and removed
particles (the shock set-up of Sec. 5: a conducting wall at x = 0, an inflow
boundary at x = L_x, injection at the shock and removal of early particles).

Each test compares the oracle with something fixed independently of it: the
straight-line motion of a free particle folded into the box by mirror
images, |v| conserved by reflections and the magnetic rotation, the exact
integer bookkeeping of deposits (nothing leaves through a mirrored stencil,
added and removed particles change n_CR, J_CR by exactly their own
integers), and the quadratic B-spline with the ghost cell's weight landing on
its mirror image.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O

P, R, A = O.PERIODIC, O.REFLECT, O.ABSORB
S = 2.0 ** 40


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


def _fields(box, Bvec=(0.0, 0.0, 0.0), vgvec=(0.0, 0.0, 0.0)):
    nc = box.n_cells
    B = np.repeat(np.asarray(Bvec, float)[:, None], nc, axis=1).copy()
    vg = np.repeat(np.asarray(vgvec, float)[:, None], nc, axis=1).copy()
    return B, vg, np.ones(nc)


def _fold(q, lo, L):
    """A free path q folded into [lo, lo + L] by mirrors at both faces."""
    t = (q - lo) % (2 * L)
    return lo + np.where(t <= L, t, 2 * L - t)


def test_free_particle_folds_between_two_reflecting_walls():
    """No fields: the particle moves on a straight line that the two walls
    fold back into the box, and its velocity reverses at every bounce."""
    C = 10.0
    box = O.Box(ndim=2, n=(7, 5, 1), dx=(0.5, 2.0, 1.0), x0=(-3.7, 11.2, 0.0), C=C,
                bc=((R, R), (P, P), (P, P)))
    B, vg, rho = _fields(box)
    x = np.array([[-3.7 + 1.3], [15.0], [0.0]])
    v = np.array([[6.0], [1.5], [0.0]])
    sys = O.System(box, x, v, np.array([0.01]), np.array([1.0]))
    g = math.sqrt(1.0 + (v[:, 0] @ v[:, 0]) / C ** 2)
    u = v[:, 0] / g
    dt = 0.09
    Lx = 7 * 0.5
    for n in range(1, 120):
        sys.step(B, vg, rho, dt, 1)
        xn = sys.positions()[:, 0]
        want = _fold(x[0, 0] + n * dt * u[0], -3.7, Lx)
        assert abs(xn[0] - want) < 1e-11 * Lx, n
        # the reflected axis reverses, the other keeps its value
        assert abs(sys.v[0, 0]) == v[0, 0] and sys.v[1, 0] == v[1, 0]
    # no fields: the push changes nothing, so the gas receives nothing, although
    # the walls reversed the particle many times (their impulse is the wall's)
    assert (sys.D[4:] == 0).all()


@pytest.mark.parametrize("side", [0, 1])
def test_gyration_against_a_wall_conserves_speed(side):
    """A gyrating particle bouncing off a reflecting face: |v| stays what it
    was to rounding (reflection negates a component, the rotation keeps the
    norm) and the particle stays inside the box."""
    C = 10.0
    box = O.Box(ndim=2, n=(8, 8, 1), dx=(0.5, 0.5, 1.0), C=C, bc=((R, R), (P, P), (P, P)))
    B, vg, rho = _fields(box, (0.0, 0.0, 1.0))
    # the orbit (radius 1.2) is centred beyond the face, so it keeps hitting it
    x0, vy = (0.4, -1.2) if side == 0 else (3.6, 1.2)
    sys = O.System(box, np.array([[x0], [2.0], [0.0]]), np.array([[0.0], [vy], [0.0]]),
                   np.array([1.0]), np.array([1.0]))
    v0 = np.linalg.norm(sys.v[:, 0])
    bounces = 0
    last = sys.v[0, 0]
    for _ in range(400):
        sys.step(B, vg, rho, 0.05, 1)
        assert abs(np.linalg.norm(sys.v[:, 0]) / v0 - 1.0) < 1e-13
        xx = sys.positions()[0, 0]
        assert 0.0 <= xx <= 4.0
        # a bounce reverses v_x while it is large; the rotation turns it through zero
        bounces += np.sign(sys.v[0, 0]) != np.sign(last) and min(abs(last), abs(sys.v[0, 0])) > 0.3
        last = sys.v[0, 0]
    assert bounces > 3


def test_deposit_next_to_a_wall_lands_on_the_mirror_cell():
    """The stencil cell beyond a reflecting face is its mirror image: its
    B-spline share is added to the cell at the face, so the integers still sum
    to the rounded amount."""
    n = (5, 4, 3)
    box = O.Box(ndim=3, n=n, dx=(1.0, 1.0, 1.0), C=20.0, bc=((R, A), (P, P), (R, R)))
    nc = box.n_cells
    cell = (0, 2, 2)
    off = (Fraction(-13, 64), Fraction(9, 64), Fraction(21, 64))
    pos = [cell[d] + Fraction(1, 2) + off[d] for d in range(3)]
    x = np.array([[float(p)] for p in pos])
    sys = O.System(box, x, np.array([[1.0], [0.5], [-0.25]]), np.array([0.02]), np.array([1.3]))
    Vn = (1.3 * 0.02) * S
    expect = np.zeros(nc)

    def mirror(c, d):
        if box.bc[d][0] == P:
            return c % n[d]
        return -1 - c if c < 0 else (2 * n[d] - 1 - c if c >= n[d] else c)

    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                c = (cell[0] + dx, cell[1] + dy, cell[2] + dz)
                w = Fraction(1)
                for d in range(3):
                    w *= _bspline2(Fraction(c[d]) + Fraction(1, 2) - pos[d])
                m = [mirror(c[d], d) for d in range(3)]
                expect[(m[2] * n[1] + m[1]) * n[0] + m[0]] += float(w * Fraction(Vn))
    D = sys.D[0]
    assert D.sum() == _rne(Fraction(Vn))
    assert np.abs(D - expect).max() <= 0.5 * 27 + Vn * 2.0 ** -47
    # the face cells carry the folded shares
    assert set(np.flatnonzero(D)) == set(np.flatnonzero(expect))


def test_absorbing_face_removes_the_particle_and_its_deposits():
    """Particles leaving through an absorbing face are gone and their n_CR,
    J_CR with them: after each step the channel sums are exactly those of the
    particles still in the box, at their own velocities."""
    C = 20.0
    box = O.Box(ndim=2, n=(12, 6, 1), C=C, hall=0, bc=((R, A), (P, P), (P, P)))
    rng = np.random.default_rng(3)
    N = 300
    x = np.stack([rng.uniform(8.0, 12.0, N), rng.uniform(0, 6.0, N), np.zeros(N)])
    v = np.stack([rng.uniform(5.0, 60.0, N), rng.normal(0, 3.0, N), rng.normal(0, 3.0, N)])
    m = np.full(N, 1e-3)
    qm = np.ones(N)
    B, vg, rho = _fields(box, (0.3, 0.0, 1.0), (0.2, 0.1, 0.0))
    sys = O.System(box, x, v, m, qm)
    for _ in range(6):
        sys.step(B, vg, rho, 0.09, 1)
        live = sys.alive == 1
        assert sys.D[0].sum() == int(live.sum()) * _rne(Fraction(1e-3 * S))
        g = np.sqrt(1.0 + (sys.v * sys.v).sum(axis=0) / C ** 2)
        for d in range(3):
            amounts = (1e-3 * (sys.v[d] / g)) * S
            assert abs(int(sys.D[1 + d].sum()) - amounts[live].sum()) <= live.sum() + 1e-9 * np.abs(amounts).sum()
    assert 0 < sys.alive.sum() < N  # the fast particles left through x = L_x


def test_absorption_in_either_half_drift_deposits_nothing_without_fields():
    """No fields, so the push changes nothing: a particle that crosses the
    absorbing face in the first half drift or in the second leaves nothing
    behind (no corrector change, no n_CR, J_CR), and particles far from the
    faces move exactly as in a periodic box."""
    C = 20.0
    box = O.Box(ndim=2, n=(12, 4, 1), C=C, bc=((R, A), (P, P), (P, P)))
    per = O.Box(ndim=2, n=(12, 4, 1), C=C)
    B, vg, rho = _fields(box)
    dt = 0.09
    vx = 15.0
    ux = vx / math.sqrt(1.0 + vx * vx / C ** 2)
    h = 0.5 * dt * ux  # cells per half drift (dx = 1)
    xs = [12.0 - 0.5 * h, 12.0 - 1.5 * h]  # crosses in the first, in the second half drift
    x = np.array([xs, [1.0, 2.0], [0.0, 0.0]])
    v = np.array([[vx, vx], [0.0, 0.0], [0.0, 0.0]])
    sys = O.System(box, x, v, np.full(2, 1e-3), np.ones(2))
    sys.step(B, vg, rho, dt, 1)
    assert (sys.alive == 0).all()
    assert (sys.D == 0).all()
    # interior particles: bit-identical to the periodic box
    rng = np.random.default_rng(4)
    xi = np.stack([rng.uniform(4.0, 8.0, 50), rng.uniform(0, 4.0, 50), np.zeros(50)])
    vi = rng.normal(0, 1.0, (3, 50))
    a = O.System(box, xi, vi, np.full(50, 1e-3), np.ones(50))
    b = O.System(per, xi, vi, np.full(50, 1e-3), np.ones(50))
    Bf, vgf, rhof = _fields(box, (0.2, 0.5, 1.0), (0.1, 0.0, 0.0))
    a.step(Bf, vgf, rhof, dt, 3)
    b.step(Bf, vgf, rhof, dt, 3)
    assert (a.D == b.D).all() and (a.v == b.v).all() and (a.positions() == b.positions()).all()


def test_added_and_removed_particles_change_nJ_by_exactly_their_own():
    """n_CR, J_CR after adding particles equal those of a system built with
    all of them at once; after removing some, those of a system built without
    them (integer sums are exact and order-free)."""
    from paper_1412_1087_amd import workloads as W
    wl = W.bell3d(n=(6, 5, 4), ppc=3, seed=31)
    bc = ((R, A), (P, P), (R, R))
    box = O.Box(ndim=3, n=wl.box.n, C=wl.box.C, hall=1, bc=bc)
    half = wl.N // 2
    a = O.System(box, wl.x[:, :half], wl.v[:, :half], wl.m[:half], wl.qm[:half])
    ids = a.inject(wl.x[:, half:], wl.v[:, half:], wl.m[half:], wl.qm[half:])
    assert (ids == np.arange(half, wl.N)).all()
    full = O.System(box, wl.x, wl.v, wl.m, wl.qm)
    assert (a.D == full.D).all()
    # step both, then remove every third particle from one
    a.step(wl.B, wl.vg, wl.rho, wl.dt, 2)
    full.step(wl.B, wl.vg, wl.rho, wl.dt, 2)
    assert (a.D == full.D).all()
    drop = np.flatnonzero(a.alive)[::3]
    a.remove(drop)
    keep = np.setdiff1d(np.flatnonzero(full.alive), drop)
    rest = O.System(box, full.positions()[:, keep], full.v[:, keep], wl.m[keep], wl.qm[keep])
    assert (a.D[:4] == rest.D[:4]).all()
    with pytest.raises(O.OracleError):
        a.remove(drop[:1])  # already gone


def test_particle_landing_on_the_upper_face_stays_inside():
    """The first half drift ends exactly on the upper reflecting face: the
    mirror image is the face itself, so the particle is kept in the last cell
    at the largest offset below 1/2, and the free path then folds back."""
    C = 16.0
    n = 4
    box = O.Box(ndim=2, n=(n, 4, 1), C=C, bc=((R, R), (P, P), (P, P)))
    B, vg, rho = _fields(box)
    vx = 40.0  # fast enough that C dt stays within the move limit
    # u and hdx as the step forms them; choose dt so that u*hdx is 3/8 exactly
    r = math.sqrt(C * C + vx * vx)
    u = vx * (C / r)
    hdt = 0.375 / u
    for _ in range(64):
        if u * hdt == 0.375:
            break
        hdt = math.nextafter(hdt, 0.0 if u * hdt > 0.375 else 1.0)
    assert u * hdt == 0.375
    dt = 2.0 * hdt
    sys = O.System(box, np.array([[n - 1 + 0.625], [1.5], [0.0]]), np.array([[vx], [0.0], [0.0]]),
                   np.array([1e-3]), np.array([1.0]))
    sys.step(B, vg, rho, dt, 1)
    # mirrored onto the face: offset just below 1/2, then drifted back by 3/8
    assert sys.cell[0, 0] == n - 1 and sys.delta[0, 0] == math.nextafter(0.5, 0.0) - 0.375
    # start n - 3/8, move +3/4 into the face and back: n - 3/8 again, to rounding
    assert abs(sys.positions()[0, 0] - (n - 0.375)) < 1e-15 * n
    assert sys.v[0, 0] == -vx


def test_faces_are_checked():
    with pytest.raises(O.OracleError):  # one face periodic, the other not
        O.System(O.Box(ndim=2, n=(4, 4, 1), bc=((P, R), (P, P), (P, P))), np.zeros((3, 1)) + 0.5,
                 np.zeros((3, 1)), np.ones(1), np.ones(1))
    with pytest.raises(O.OracleError):  # a wall needs two cells along its axis
        O.System(O.Box(ndim=2, n=(1, 4, 1), bc=((R, R), (P, P), (P, P))), np.zeros((3, 1)) + 0.5,
                 np.zeros((3, 1)), np.ones(1), np.ones(1))
    box = O.Box(ndim=2, n=(4, 4, 1), bc=((R, A), (P, P), (P, P)))
    with pytest.raises(O.OracleError) as e:  # outside a non-periodic axis
        O.System(box, np.array([[4.5], [1.0], [0.0]]), np.zeros((3, 1)), np.ones(1), np.ones(1))
    assert e.value.code == O.ERANGE
    # the periodic axis still wraps
    O.System(box, np.array([[1.5], [9.0], [0.0]]), np.zeros((3, 1)), np.ones(1), np.ones(1))
