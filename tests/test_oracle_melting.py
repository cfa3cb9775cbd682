"""Melting by walk-back in the oracle (Sec. 2.1.3; reading R15): reached
sites with negative undercooling melt, particles of melted departure sites
go, the solid sites next to the melt are re-activated towards it, and a grain
that melts entirely returns its nucleation site to the dormant pool.  Pinned
by integer brute force on a cube-aligned lattice ball cut by a plane, by the
uniform-superheat closed form, and by a site that fires, melts and fires
again."""
import numpy as np

from oracle import Oracle
from paper_2504_12858_amd import workloads as W

LAM = 5e-6
C = np.array([5e-4, 5e-4, 5e-4])


def _ball(r):
    s = np.arange(-r, r + 1)
    X, Y, Z = np.meshgrid(s, s, s, indexing="ij")
    keep = np.abs(X) + np.abs(Y) + np.abs(Z) <= r
    return {tuple(v) for v in np.stack([X[keep], Y[keep], Z[keep]], axis=1).tolist()}


def _grain(r, field):
    o = Oracle((0, 0, 0), (1e-3, 1e-3, 1e-3), LAM, LAM, LAM, W.KIN_A, W.KIN_B)
    o.set_field(field)
    o.init_grains(C[None, :], np.array([[1.0, 0, 0, 0]]), np.array([r], np.int32))
    o.set_melting(True)
    return o


def _claims(o):
    c = o.claims()
    return {tuple(s): int(f) for s, f in zip(c["site"].tolist(), c["flags"].tolist())}


def test_plane_cut_by_integer_brute_force():
    """dT = -G (x - x_cut) with the zero plane half-way between lattice planes
    cut and cut + 1: sites with S_x > cut melt; each melted site of the first
    melted layer gets a walk-back particle from S = T - e_x (direction +x);
    deeper melted sites have no solid neighbour."""
    r, cut, G = 8, 3, 1e4
    x_cut = C[0] + (cut + 0.5) * LAM
    f = W.Field(W.FIELD_LINEAR, dT0=G * x_cut, grad=(-G, 0.0, 0.0), rate=0.0)
    o = _grain(r, f)
    before = o.particles()
    o.phase(6)                                   # the melting phase alone
    ball = _ball(r)
    melted = {s for s in ball if s[0] > cut}
    survive = ball - melted
    layer = {s for s in melted if s[0] == cut + 1}
    st = o.melt_stats()
    assert st["melted"] == len(melted)
    assert st["reactivated"] == len(layer)
    assert st["grains_melted"] == 0
    # Shell particles (L1 radius r) whose departure site melted are removed.
    dep_melted = sum(1 for s in before["site"].tolist() if s[0] > cut)
    assert st["removed"] == dep_melted
    # Claims: the surviving ball reached, the first melted layer claimed again
    # as targets, everything else gone.  (Shell particles' targets beyond the
    # ball are released with removed particles and kept otherwise.)
    cl = _claims(o)
    reached = {s for s, fl in cl.items() if fl & 2}
    assert reached == survive
    targets = {s for s, fl in cl.items() if fl == 1}
    assert layer <= targets
    assert not any(s[0] > cut + 1 for s in targets)
    # New particles: at T - e_x, direction +x (0), travel 0, active.
    p = o.particles()
    old = set(zip(map(tuple, before["site"].tolist()), before["dir"].tolist()))
    now = [(tuple(s), d) for s, d, st in zip(p["site"].tolist(), p["dir"].tolist(),
                                            p["state"].tolist()) if st == 0]
    got = {k for k in now if k not in old}
    assert got == {((t[0] - 1, t[1], t[2]), 0) for t in layer}
    assert all(p["s"][i] == 0.0 for i in range(len(p["s"])) if p["state"][i] == 0
               and (tuple(p["site"][i]), p["dir"][i]) in got)


def test_uniform_superheat_melts_the_grain():
    o = _grain(5, W.Field(W.FIELD_UNIFORM, dT=-1.0))
    n = len(o.particles()["s"])
    o.step(1e-4, 1)
    st = o.melt_stats()
    assert st["melted"] == len(_ball(5))
    assert st["removed"] == n and st["reactivated"] == 0 and st["grains_melted"] == 1
    assert len(_claims(o)) == 0
    assert (o.particles()["state"] == 2).all() if len(o.particles()["state"]) else True


def test_melted_site_fires_again():
    """A site fires (dT = 5 K >= 1 K), its grain melts entirely at dT = -1 K,
    and the site fires again as a new grain when the undercooling returns."""
    o = Oracle((0, 0, 0), (1e-3, 1e-3, 1e-3), LAM, LAM, LAM, W.KIN_A, W.KIN_B)
    o.set_melting(True)
    o.nucleate(C[None, :], np.array([1.0]), np.array([[1.0, 0, 0, 0]]))
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=5.0))
    o.step(1e-4, 1)
    assert list(o.site_states()) == [1]
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=-1.0))
    o.step(1e-4, 1)
    assert o.melt_stats()["grains_melted"] == 1
    assert list(o.site_states()) == [0]
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=5.0))
    o.step(1e-4, 1)
    assert list(o.site_states()) == [1]
    centres, _ = o.grains()
    assert len(centres) == 2
    cl = o.claims()
    assert set(cl["grain"].tolist()) == {1}


def test_regrowth_after_walk_back():
    """After the plane cut, a uniform undercooling makes the walk-back
    particles reach the first melted layer again."""
    r, cut, G = 8, 3, 1e4
    x_cut = C[0] + (cut + 0.5) * LAM
    o = _grain(r, W.Field(W.FIELD_LINEAR, dT0=G * x_cut, grad=(-G, 0.0, 0.0), rate=0.0))
    o.phase(6)
    layer = {s for s in _ball(r) if s[0] == cut + 1}
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=5.0))
    vdt = (W.KIN_A[0] * 25 + W.KIN_A[1] * 125) * 1e-4
    o.step(1e-4, int(np.ceil(LAM / vdt)))
    assert o.melt_stats()["melted"] == 0
    reached = {s for s, fl in _claims(o).items() if fl & 2}
    assert layer <= reached
