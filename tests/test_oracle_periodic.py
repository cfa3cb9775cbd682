"""Periodic lateral boundaries in the oracle (Sec. 3.4 imposes periodic
conditions on the faces normal to x and y; reading R16): positions stay
lattice-anchored and unwrapped, the cell, field, deposition cell and grain
map take the wrapped position, and particles meet through their nearest
periodic images (one grain meets itself only through a non-zero period
shift).  Pinned by brute force over explicit images, by closed-form stop
steps of single-axis particles (a grain meeting its own image, two grains
meeting across a face), by nucleation and grain maps through a face, and by
the deposition of a ball that straddles a face."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2504_12858_amd import workloads as W

LAM = 5e-6
Q0 = np.array([[1.0, 0.0, 0.0, 0.0]])
VDT = (W.KIN_A[0] * 5.0 ** 2 + W.KIN_A[1] * 5.0 ** 3) * 1e-4   # v(5 K) dt, dt = 1e-4 s


def _orc(hi, periodic, box_exit=1, field=None):
    o = Oracle((0, 0, 0), hi, LAM, LAM, LAM, W.KIN_A, W.KIN_B, box_exit=box_exit,
               periodic=periodic)
    o.set_field(field or W.Field(W.FIELD_UNIFORM, dT=5.0))
    return o


def _cloud(seed, L, n_grains=4, per=400, m=25):
    """Grains anywhere in the periodic box with particles up to m sites away
    (clouds that reach through the faces; each grain spans more than half a
    period, so a grain also meets its own images)."""
    g = W.rng(seed)
    centre = g.random((n_grains, 3)) * L
    quat = W.shoemake_quaternions(g, n_grains)
    grain = np.repeat(np.arange(n_grains, dtype=np.int32), per)
    site = g.integers(-m, m + 1, size=(grain.size, 3)).astype(np.int32)
    d = g.integers(0, 6, size=grain.size).astype(np.int32)
    s = g.random(grain.size) * LAM
    state = np.where(g.random(grain.size) < 0.3, 1, 0).astype(np.int32)
    return centre, quat, dict(grain=grain, site=site, dir=d, s=s, state=state)


_EMPTY = dict(grain=np.zeros(0, np.int32), site=np.zeros((0, 3), np.int32),
              flags=np.zeros(0, np.uint8))


@pytest.mark.parametrize("periodic", [1, 3, 7])
@pytest.mark.parametrize("seed", [1, 2])
def test_periodic_cells_equal_brute_force_over_images(periodic, seed):
    """The wrapped 27-cell stencil with nearest-image distances decides as
    the brute force over every pair and every explicit period shift."""
    L = 40 * LAM
    centre, quat, parts = _cloud(seed, L)
    o = _orc((L,) * 3, periodic, box_exit=0)
    o.load_state(centre, quat, parts, _EMPTY, np.zeros(0, np.int32), 0.0, 0)
    cells, brute = o.contain_decisions(0), o.contain_decisions(1)
    np.testing.assert_array_equal(cells, brute)
    flat = _orc((L,) * 3, 0, box_exit=0)
    flat.load_state(centre, quat, parts, _EMPTY, np.zeros(0, np.int32), 0.0, 0)
    assert cells.sum() > flat.contain_decisions(0).sum()   # images matter
    # One grain alone meets only its own images.
    c1, q1, one = _cloud(seed + 10, L, n_grains=1, per=3000)
    o1 = _orc((L,) * 3, periodic, box_exit=0)
    o1.load_state(c1, q1, one, _EMPTY, np.zeros(0, np.int32), 0.0, 0)
    own = o1.contain_decisions(0)
    np.testing.assert_array_equal(own, o1.contain_decisions(1))
    assert own.sum() > 0


def test_period_that_does_not_divide_exactly_in_fp64():
    """A period of 50 cells of 4 um: (0.2 mm) / (4 um) is 50.00000000000001 in
    FP64, and the grid must still have exactly 50 cells along the periodic
    axis (the last cell borders the first), else contacts across the face
    are missed."""
    lam = 4e-6
    L = 0.2e-3
    assert (L / lam) != 50.0 and round(L / lam) == 50
    g = W.rng(3)
    centre = g.random((3, 3)) * L
    quat = W.shoemake_quaternions(g, 3)
    grain = np.repeat(np.arange(3, dtype=np.int32), 1500)
    site = g.integers(-30, 31, size=(grain.size, 3)).astype(np.int32)
    parts = dict(grain=grain, site=site, dir=g.integers(0, 6, grain.size).astype(np.int32),
                 s=g.random(grain.size) * lam, state=np.zeros(grain.size, np.int32))
    o = Oracle((0, 0, 0), (L,) * 3, lam, lam, lam, W.KIN_A, W.KIN_B, box_exit=0, periodic=7)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=0.0))
    o.load_state(centre, quat, parts, _EMPTY, np.zeros(0, np.int32), 0.0, 0)
    cells = o.contain_decisions(0)
    np.testing.assert_array_equal(cells, o.contain_decisions(1))
    assert cells.sum() > 0


def _first_step(gap0, rate, rc):
    """First step n with gap0 - rate * s_n < rc, s_n the FP64 running sum of
    v dt; also the margin to the threshold at the steps around it."""
    s, n = 0.0, 0
    while True:
        n += 1
        s += VDT
        if gap0 - rate * s < rc:
            before = gap0 - rate * (s - VDT) - rc
            after = rc - (gap0 - rate * s)
            return n, min(before, after)


def _stop_steps(o, n_max):
    """Step at which each particle first stopped (0: never), by dir."""
    n = len(o.particles()["state"])
    stop = np.zeros(n, np.int64)
    for k in range(1, n_max + 1):
        o.step(1e-4, 1)
        st = o.particles()["state"]
        stop[(stop == 0) & (st == 1)] = k
    return stop


def test_grain_meets_its_own_image_at_the_closed_form_step():
    """A nucleus with branching off in a box periodic in x (period 20
    lambda0) and y (26 lambda0): the +x and -x particles close the gap
    L - 2 s through the period and stop when it drops below rc; likewise
    +-y; +-z (not periodic, centre 30 lambda0 from the faces) never stop
    before they exit.  Without periodic axes nothing stops."""
    Lx, Ly, Lz = 20 * LAM, 26 * LAM, 60 * LAM
    nx, mx = _first_step(Lx, 2.0, LAM)
    ny, my = _first_step(Ly, 2.0, LAM)
    assert min(mx, my) > 0.2 * VDT          # no near-tie at the threshold
    c = np.array([[0.3 * LAM, 25.6 * LAM, 30 * LAM]])   # near the faces: crosses them
    o = _orc((Lx, Ly, Lz), 3)
    o.set_branching(0)
    o.init_grains(c, Q0, np.array([0], np.int32))
    stop = _stop_steps(o, ny + 3)
    d = o.particles()["dir"]
    assert stop[d == 0].tolist() == [nx] and stop[d == 1].tolist() == [nx]
    assert stop[d == 2].tolist() == [ny] and stop[d == 3].tolist() == [ny]
    assert stop[d >= 4].tolist() == [0, 0]
    flat = _orc((100 * LAM,) * 3, 0, box_exit=0)
    flat.set_branching(0)
    flat.init_grains(c + 40 * LAM, Q0, np.array([0], np.int32))
    assert not _stop_steps(flat, ny + 3).any()


def test_two_grains_meet_across_a_face():
    """Grains at x = 2 and x = L - 3 lambda0: the -x particle of the first and
    the +x particle of the second are 5 lambda0 apart through the face and
    meet when 5 lambda0 - 2 s < rc, well before the facing pair inside the
    box (15 lambda0 - 2 s < rc).  Without periodic axes the -x particle exits
    the box instead."""
    L = 20 * LAM
    n, m = _first_step(5 * LAM, 2.0, LAM)
    assert m > 0.2 * VDT
    c = np.array([[2 * LAM, 13 * LAM, 30 * LAM], [L - 3 * LAM, 13 * LAM, 30 * LAM]])
    for periodic in (1, 0):
        o = _orc((L, 26 * LAM, 60 * LAM), periodic)
        o.set_branching(0)
        o.init_grains(c, np.repeat(Q0, 2, 0), np.array([0, 0], np.int32))
        o.step(1e-4, n - 1)
        assert (o.particles()["state"] == 0).all()
        o.step(1e-4, 1)
        st, p = o.last_stats(), o.particles()
        if periodic:
            assert st["contained"] == 2 and st["exited"] == 0
            stopped = {(int(g), int(d)) for g, d, s in zip(p["grain"], p["dir"], p["state"]) if s == 1}
            assert stopped == {(0, 1), (1, 0)}
        else:
            assert st["contained"] == 0 and st["exited"] == 1


def test_site_inside_a_grain_through_the_face_does_not_fire():
    """A lattice ball of radius 10 centred 3 lambda0 below the face x = L
    covers the image x + L of a site at x = 2 lambda0: with x periodic the
    site is inside the grain and never fires; without, it fires."""
    L = 20 * LAM
    c = np.array([[L - 3 * LAM, 13 * LAM, 30 * LAM]])
    site = np.array([[2 * LAM, 13 * LAM, 30 * LAM]])
    for periodic, fired in ((1, 0), (0, 1)):
        o = _orc((L, 26 * LAM, 60 * LAM), periodic)
        o.init_grains(c, Q0, np.array([10], np.int32))
        o.nucleate(site, np.array([1.0]), Q0)
        o.step(1e-9, 1)
        assert list(o.site_states()) == [fired]


def test_grain_map_and_deposition_through_the_face():
    """A reached ball of radius 6 whose lattice sites sit on voxel centres,
    centred 1.5 lambda0 below the face x = L: with x periodic its grain map
    is the map of the same ball centred mid-box, rolled by the shift, and its
    deposition counts sum to ball(6) (only part of it without)."""
    L = 20 * LAM
    hi = (L, 26 * LAM, 60 * LAM)
    n = (20, 26, 60)
    vox = (LAM,) * 3
    face = np.array([[18.5 * LAM, 10.5 * LAM, 30.5 * LAM]])
    mid = face - np.array([[10 * LAM, 0, 0]])
    maps = []
    for c in (face, mid):
        o = _orc(hi, 1)
        o.init_grains(c, Q0, np.array([6], np.int32))
        maps.append(o.grain_map(np.array(n, np.int32), np.zeros(3), np.array(vox)))
    ball = (2 * 6 + 1) * (2 * 36 + 12 + 3) // 3
    assert (maps[1] > 0).sum() == ball
    np.testing.assert_array_equal(maps[0], np.roll(maps[1], 10, axis=2))
    flat = _orc(hi, 0)
    flat.init_grains(face, Q0, np.array([6], np.int32))
    fm = flat.grain_map(np.array(n, np.int32), np.zeros(3), np.array(vox))
    assert (fm[:, :, :5] == 0).all() and 0 < (fm > 0).sum() < ball
    # Deposition on node-centred cells of 2 lambda0 tiling the box.
    sp = np.array([2 * LAM] * 3)
    cells = (10, 13, 30)
    o = _orc(hi, 1)
    o.init_grains(face, Q0, np.array([6], np.int32))
    assert o.deposit_counts(cells, sp / 2, sp).sum() == ball
    assert 0 < flat.deposit_counts(cells, sp / 2, sp).sum() < ball
