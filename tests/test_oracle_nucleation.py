"""Pins of the oracle's nucleation (Sec. 2.1.1: a pre-drawn site fires when
its local undercooling reaches its nucleation undercooling) and of the grain
map (Sec. 2.3: each voxel takes the grain of its nearest lattice site)."""
import math

import numpy as np

from oracle import Oracle
from paper_2504_12858_amd import workloads as W


def test_fire_step_in_uniform_cooling():
    """dT(t) = dT0 + rate t everywhere: site i fires in the first step n with
    dT0 + rate n dt >= dTn_i."""
    dT0, rate, dt = 0.5, 10.0, 1e-3
    g = W.rng(8)
    n_sites = 12
    xyz = np.array([[1e-4 + 6e-5 * i, 2e-4 + 5e-5 * (i % 4), 3e-4 + 4e-5 * (i % 3)] for i in range(n_sites)])
    dTn = 0.5 + g.random(n_sites) * 4.0
    # Negligible kinetics: grains stay point-like, so no site gets engulfed.
    o = Oracle((0, 0, 0), (1e-3,) * 3, 5e-6, 5e-6, 5e-6, (1e-12, 0.0), W.KIN_B)
    o.set_field(W.Field(W.FIELD_LINEAR, dT0=dT0, rate=rate))
    o.nucleate(xyz, dTn, W.shoemake_quaternions(g, n_sites))
    expect = np.array([math.ceil((d - dT0) / (rate * dt)) for d in dTn])
    fired_at = np.full(n_sites, -1)
    for n in range(0, int(expect.max()) + 2):
        o.step(dt, 1)
        st = o.site_states()
        fired_at[(st == 1) & (fired_at < 0)] = n
    np.testing.assert_array_equal(fired_at, expect)
    # Grain ids follow firing order, then site index.
    c, _ = o.grains()
    order = np.lexsort((np.arange(n_sites), expect))
    np.testing.assert_allclose(c, xyz[order])
    assert o.count(1) == 6 * n_sites


def test_site_inside_grain_claims_never_fires():
    o = Oracle((0, 0, 0), (1e-3,) * 3, 5e-6, 5e-6, 5e-6, W.KIN_A, W.KIN_B)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=5.0))
    c = np.array([[5e-4, 5e-4, 5e-4]])
    o.init_grains(c, np.array([[1.0, 0, 0, 0]]), np.array([8], np.int32))
    # Inside the claimed ball (L1 < 8 lambda0) but far from every particle.
    o.nucleate(c + [[1.2e-6, 0.9e-6, 0.0]], np.array([0.0]), np.array([[1.0, 0, 0, 0]]))
    o.step(1e-4, 20)
    assert o.site_states()[0] == 0
    assert o.count(4) == 1


def test_site_near_particle_waits():
    """A site within rc of a particle stays dormant; once the particle has
    moved away (and the site is not claimed) it fires."""
    lam = 5e-6
    o = Oracle((0, 0, 0), (1e-3,) * 3, lam, lam, lam, W.KIN_A, W.KIN_B, branching=0)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=5.0))
    c = np.array([[5e-4, 5e-4, 5e-4]])
    q = W.bunge_quaternion(0, 0, 45)   # crystal x axis along world (1,1,0)/sqrt2
    o.init_grains(c, q[None, :], np.array([0], np.int32))
    # Site on the world x axis at 0.8 rc from the centre: its rounded lattice
    # position in the rotated grain is a neighbour of the origin, which is
    # never claimed without branching.  The six particles start at the centre.
    y = c + [[0.8 * lam, 0.0, 0.0]]
    o.nucleate(y, np.array([1.0]), np.array([[1.0, 0, 0, 0]]))
    o.step(1e-4, 1)
    assert o.site_states()[0] == 0
    v = 1e-5 * 25 + 1e-6 * 125
    # The site is at distance |y - x_p| from the particles on the +-x crystal
    # axes; after enough steps every particle is > rc away.
    o.step(1e-4, int(2 * lam / (v * 1e-4)) + 2)
    assert o.site_states()[0] == 1


def test_same_step_sites_resolved_in_index_order():
    lam = 5e-6
    o = Oracle((0, 0, 0), (1e-3,) * 3, lam, lam, lam, W.KIN_A, W.KIN_B)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=5.0))
    y0 = np.array([5e-4, 5e-4, 5e-4])
    xyz = np.stack([y0 + [0.1 * lam, 0.1 * lam, 0.1 * lam], y0, y0 + [2e-4, 0, 0]])
    o.nucleate(xyz, np.array([1.0, 0.5, 1.0]), np.array([[1.0, 0, 0, 0]] * 3))
    o.step(1e-4, 1)
    # Site 0 fires first; site 1 (within rc and inside site 0's claimed cell)
    # is blocked; site 2 is far away and fires.
    np.testing.assert_array_equal(o.site_states(), [1, 0, 1])
    c, _ = o.grains()
    np.testing.assert_allclose(c, xyz[[0, 2]])


def test_grain_map_counts_voronoi_cells_of_reached_ball():
    """After k generations in a uniform melt the reached set is the lattice
    ball k; with voxels of edge lambda0/4 aligned to the lattice, every reached
    site's Voronoi cube holds exactly 64 voxel centres."""
    lam, dT, dt = 5e-6, 4.7, 1e-3
    c0 = 5e-4
    o = Oracle((0, 0, 0), (1e-3,) * 3, lam, lam, lam, W.KIN_A, W.KIN_B)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=dT))
    o.init_grains(np.array([[c0] * 3]), np.array([[1.0, 0, 0, 0]]), np.zeros(1, np.int32))
    o.step(dt, 48)      # 3 generations at v dt = 3.247e-7 (15.4 steps each)
    ball3 = 7 * (18 + 6 + 3) // 3
    assert o.count(8) == ball3
    m = 10
    n = np.array([8 * m] * 3, np.int32)
    origin = np.array([c0 - m * lam - lam / 2] * 3) + 0.0
    spacing = np.array([lam / 4] * 3)
    gm = o.grain_map(n, origin, spacing)
    assert (gm == 1).sum() == 64 * ball3
    assert set(np.unique(gm)) == {0, 1}


def test_grain_map_nearest_site_wins():
    lam = 5e-6
    cA = np.array([5e-4, 5e-4, 5e-4])
    cB = cA + [0.3 * lam, 0.0, 0.0]
    o = Oracle((0, 0, 0), (1e-3,) * 3, lam, lam, lam, W.KIN_A, W.KIN_B)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=0.0))
    parts = dict(grain=np.zeros(0, np.int32), site=np.zeros((0, 3), np.int32),
                 dir=np.zeros(0, np.int32), s=np.zeros(0), state=np.zeros(0, np.int32))
    claims = dict(grain=np.array([0, 1], np.int32), site=np.zeros((2, 3), np.int32),
                  flags=np.array([3, 3], np.uint8))
    o.load_state(np.stack([cA, cB]), np.array([[1.0, 0, 0, 0]] * 2), parts, claims,
                 np.zeros(0, np.int32), 0.0, 0)
    # Voxel centres at cA + 0.2 lam (B nearer: 0.1 lam) and cA - 0.1 lam (A nearer).
    for off, label in ((0.2, 2), (-0.1, 1), (0.18, 2), (0.12, 1)):
        y = cA + [off * lam, 0, 0]
        spacing = np.array([1e-9] * 3)
        gm = o.grain_map(np.array([1, 1, 1], np.int32), y - spacing / 2, spacing)
        assert gm.ravel()[0] == label, off
