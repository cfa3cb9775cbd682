"""Pins of the oracle's rebin, containment (grain-boundary formation, Sec.
2.1.2: particles of two grains stop when they meet) and box exit, and of the
FP32 checker against single-rounded numpy float32 arithmetic."""
import numpy as np
import pytest

from oracle import Oracle, f32_cells, f32_contain
from paper_2504_12858_amd import workloads as W


def _cloud(seed, n_grains=5, per_grain=300, lam=5e-6, m=4, stopped_frac=0.3):
    """Grains centred within a few lambda0 of each other so that their
    particle clouds interpenetrate."""
    g = W.rng(seed)
    box = 1e-3
    centre = box / 2 + (g.random((n_grains, 3)) - 0.5) * 6 * lam
    quat = W.shoemake_quaternions(g, n_grains)
    grain = np.repeat(np.arange(n_grains, dtype=np.int32), per_grain)
    site = g.integers(-m, m + 1, size=(grain.size, 3)).astype(np.int32)
    d = g.integers(0, 6, size=grain.size).astype(np.int32)
    s = g.random(grain.size) * lam
    state = np.where(g.random(grain.size) < stopped_frac, 1, 0).astype(np.int32)
    state[g.random(grain.size) < 0.1] = 2   # some retired: never obstacles
    return centre, quat, dict(grain=grain, site=site, dir=d, s=s, state=state)


def _load(centre, quat, parts, lam=5e-6, rc=None):
    rc = lam if rc is None else rc
    o = Oracle((0, 0, 0), (1e-3,) * 3, lam, lam, rc, W.KIN_A, W.KIN_B)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=0.0))
    empty = dict(grain=np.zeros(0, np.int32), site=np.zeros((0, 3), np.int32),
                 flags=np.zeros(0, np.uint8))
    o.load_state(centre, quat, parts, empty, np.zeros(0, np.int32), 0.0, 0)
    return o


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_cell_stencil_equals_brute_force(seed):
    centre, quat, parts = _cloud(seed)
    o = _load(centre, quat, parts)
    cells = o.contain_decisions(0)
    brute = o.contain_decisions(1)
    np.testing.assert_array_equal(cells, brute)
    assert 0 < cells.sum() < (parts["state"] == 0).sum()   # non-trivial case
    # Only active particles can be stopped.
    assert not cells[parts["state"] != 0].any()


@pytest.mark.parametrize("rc_over_h", [0.5, 0.999, 1.0])
def test_cell_stencil_complete_for_rc_up_to_h(rc_over_h):
    lam = 5e-6
    centre, quat, parts = _cloud(7, per_grain=400)
    o = _load(centre, quat, parts, lam=lam, rc=rc_over_h * lam)
    np.testing.assert_array_equal(o.contain_decisions(0), o.contain_decisions(1))


def test_pair_distance_threshold_by_hand():
    """Two single-particle grains on the x axis: they meet iff d < rc."""
    lam = 5e-6
    for gap, expect in ((0.9 * lam, 1), (1.1 * lam, 0)):
        c = np.array([[5e-4, 5e-4, 5e-4], [5e-4 + gap, 5e-4, 5e-4]])
        q = np.array([[1.0, 0, 0, 0]] * 2)
        parts = dict(grain=np.array([0, 1], np.int32), site=np.zeros((2, 3), np.int32),
                     dir=np.array([0, 1], np.int32), s=np.zeros(2), state=np.zeros(2, np.int32))
        o = _load(c, q, parts)
        np.testing.assert_array_equal(o.contain_decisions(0), [expect, expect])
        # Same grain never stops itself.
        parts["grain"][:] = 0
        o = _load(c[:1].repeat(2, 0) + [[0, 0, 0], [gap, 0, 0]], q[:1], dict(parts, grain=np.zeros(2, np.int32)))
        np.testing.assert_array_equal(o.contain_decisions(0), [0, 0])


def test_head_on_grains_stop_each_other():
    """Two nuclei on the x axis in a uniform melt grow towards each other; the
    facing vertices stop when their gap drops below rc, the others keep going."""
    lam, dT, dt = 5e-6, 5.0, 1e-4
    gap0 = 30e-6
    o = Oracle((0, 0, 0), (1e-3,) * 3, lam, lam, lam, W.KIN_A, W.KIN_B, branching=0)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=dT))
    c = np.array([[5e-4, 5e-4, 5e-4], [5e-4 + gap0, 5e-4, 5e-4]])
    o.init_grains(c, np.array([[1.0, 0, 0, 0]] * 2), np.zeros(2, np.int32))
    v = 1e-5 * dT ** 2 + 1e-6 * dT ** 3
    # Gap after n steps: gap0 - 2 n v dt; first n with gap < lam.
    n_meet = int(np.floor((gap0 - lam) / (2 * v * dt))) + 1
    o.step(dt, n_meet - 1)
    assert o.count(2) == 0
    o.step(dt, 1)
    p = o.particles()
    stopped = np.flatnonzero(p["state"] == 1)
    assert sorted(zip(p["grain"][stopped], p["dir"][stopped])) == [(0, 0), (1, 1)]


def test_box_exit_stops_particle():
    lam, dT, dt = 5e-6, 5.0, 1e-4
    o = Oracle((0, 0, 0), (1e-3,) * 3, lam, lam, lam, W.KIN_A, W.KIN_B, branching=0)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=dT))
    v = 1e-5 * dT ** 2 + 1e-6 * dT ** 3
    x0 = 1e-3 - 2.5 * v * dt          # +x vertex leaves during step 3
    o.init_grains(np.array([[x0, 5e-4, 5e-4]]), np.array([[1.0, 0, 0, 0]]), np.zeros(1, np.int32))
    o.step(dt, 2)
    assert o.count(2) == 0
    o.step(dt, 1)
    p = o.particles()
    assert o.last_stats()["exited"] == 1
    assert p["state"][p["dir"] == 0][0] == 1
    # The stopped particle is frozen.
    x = p["x"][p["dir"] == 0][0].copy()
    o.step(dt, 2)
    np.testing.assert_array_equal(o.particles()["x"][p["dir"] == 0][0], x)


def test_f32_cells_single_rounded():
    g = W.rng(5)
    xyz = (g.random((20000, 3)) * 1e-3).astype(np.float32)
    lo = np.zeros(3, np.float32)
    inv_h = np.float32(1.0 / 5e-6)
    ncell = np.array([200, 200, 200], np.int32)
    got = f32_cells(xyz, lo, inv_h, ncell)
    want = np.clip(np.floor((xyz - lo) * inv_h), 0, ncell - 1).astype(np.int32)
    np.testing.assert_array_equal(got, want)


def test_f32_contain_matches_float32_brute_force():
    g = W.rng(6)
    n = 1500
    xyz = (5e-4 + (g.random((n, 3)) - 0.5) * 60e-6).astype(np.float32)
    grain = g.integers(0, 4, n).astype(np.int32)
    role = g.choice(np.array([0, 1, 2], np.uint8), n, p=[0.1, 0.6, 0.3])
    rc2 = np.float32(5e-6 * 5e-6)
    got = f32_contain(xyz, grain, role, rc2)
    d = xyz[:, None, :] - xyz[None, :, :]          # float32
    d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    hit = (d2 < rc2) & (grain[:, None] != grain[None, :]) & (role[None, :] > 0)
    want = (hit.any(axis=1) & (role == 1)).astype(np.uint8)
    np.testing.assert_array_equal(got, want)
    assert want.sum() > 50
