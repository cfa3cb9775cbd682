"""GPU binning and containment: bit-exact against the FP32 checker on the
GPU's own positions, and equal to the FP64 oracle's decisions except for pairs
whose distance is within 1e-4 rc of the contact radius.

The 1e-4 band: FP32 coordinates near 0.5 mm carry an ulp of 6e-11 m, i.e.
1.2e-5 rc at rc = 5 um; a distance built from three coordinate differences of
positions reconstructed with a few roundings each can move by several ulps."""
import numpy as np
import pytest

from oracle import Oracle, f32_cells, f32_contain
from paper_2504_12858_amd import binding as B
from paper_2504_12858_amd import workloads as W
from tests.gpu_helpers import gpu_parts, ident, orc_parts, require_gpu

pytestmark = pytest.mark.gpu


def _cloud(seed, n_grains, per_grain, lam, m, stopped_frac, spread):
    g = W.rng(seed)
    box = 1e-3
    centre = box / 2 + (g.random((n_grains, 3)) - 0.5) * spread
    quat = W.shoemake_quaternions(g, n_grains)
    grain = np.repeat(np.arange(n_grains, dtype=np.int32), per_grain)
    site = g.integers(-m, m + 1, size=(grain.size, 3)).astype(np.int32)
    d = g.integers(0, 6, size=grain.size).astype(np.int32)
    s = (g.random(grain.size) * lam).astype(np.float32).astype(np.float64)
    state = np.where(g.random(grain.size) < stopped_frac, 1, 0).astype(np.int32)
    # Unique identities (grain, site, dir).
    key = (grain.astype(np.int64) << 40) ^ ((site[:, 0] + 64) << 16) ^ ((site[:, 1] + 64) << 8) ^ (site[:, 2] + 64)
    key = key * 8 + d
    _, first = np.unique(key, return_index=True)
    keep = np.sort(first)
    parts = dict(grain=grain[keep], site=site[keep], dir=d[keep], s=s[keep], state=state[keep])
    return centre, quat, parts


EMPTY_CLAIMS = dict(grain=np.zeros(0, np.int32), site=np.zeros((0, 3), np.int32),
                    flags=np.zeros(0, np.uint8))


@pytest.mark.parametrize("seed,n_grains,per_grain,m,spread,h_factor", [
    (1, 6, 400, 4, 30e-6, 1.0),
    (2, 12, 1500, 8, 60e-6, 1.0),
    (3, 40, 3000, 12, 150e-6, 1.0),   # many 4^3-cell bricks, ragged fill
    (4, 12, 1500, 8, 60e-6, 2.0),     # cells of 2 rc: 2x2x2 stencil
    (5, 40, 3000, 12, 150e-6, 2.0),
])
def test_single_step_contact_parity(seed, n_grains, per_grain, m, spread, h_factor):
    require_gpu()
    lam = 5e-6
    h = h_factor * lam
    dT, dt = 3.0, 1e-4
    centre, quat, parts = _cloud(seed, n_grains, per_grain, lam, m, 0.3, spread)
    print(f"contact parity seed={seed} n={len(parts['grain'])}", flush=True)
    p = B.make_params((0, 0, 0), (1e-3,) * 3, lam, h, lam, W.KIN_A, W.KIN_B, branching=0,
                      cap_particles=1 << 18, cap_stopped=1 << 18, cap_grains=64,
                      cap_claim_bricks=1 << 12)
    ctx = B.Context(p)
    ctx.set_thermal_field(W.Field(W.FIELD_UNIFORM, dT=dT))
    ctx.load_state(centre, quat, parts, EMPTY_CLAIMS, np.zeros(0, np.int32), 0.0, 0)
    ctx.step(dt, 1)
    g, key = gpu_parts(ctx)
    xyz = np.stack([g["x"], g["y"], g["z"]], 1)
    # Binning: exported cells equal single-rounded FP32 binning of the
    # exported positions.
    ncell = int(np.ceil(1e-3 / h))
    cells = f32_cells(xyz, np.zeros(3, np.float32), np.float32(1.0 / h), np.array([ncell] * 3, np.int32))
    np.testing.assert_array_equal(cells, g["cell"])
    # Roles before the step: active particles are tested, stopped ones are obstacles.
    pk = ident(parts["grain"], parts["site"], parts["dir"])
    order = np.argsort(pk)
    np.testing.assert_array_equal(pk[order], key)
    pre_state = parts["state"][order]
    role = np.where(pre_state == 0, 1, 2).astype(np.uint8)
    rc2 = np.float32(lam * lam)
    dec = f32_contain(xyz, g["grain"].astype(np.int32), role, rc2)
    gpu_dec = ((pre_state == 0) & (g["state"] == 1)).astype(np.uint8)
    np.testing.assert_array_equal(gpu_dec, dec)
    assert dec.sum() > 0
    # FP64 oracle: same decisions except pairs within 1e-5 of rc.
    o = Oracle((0, 0, 0), (1e-3,) * 3, lam, h, lam, W.KIN_A, W.KIN_B, branching=0)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=dT))
    o.load_state(centre, quat, parts, EMPTY_CLAIMS, np.zeros(0, np.int32), 0.0, 0)
    o.step(dt, 1)
    q, okey = orc_parts(o)
    np.testing.assert_array_equal(okey, key)
    assert np.abs(xyz.astype(np.float64) - q["x"]).max() <= 1e-5 * 1e-3
    mism = np.flatnonzero(q["state"] != g["state"])
    for i in mism:
        d = np.sqrt(((q["x"] - q["x"][i]) ** 2).sum(1))
        other = q["grain"] != q["grain"][i]
        near = np.abs(d[other] - lam).min() / lam
        assert near < 1e-4, (i, near)
    assert len(mism) <= 2


def test_stopped_particles_block_and_survive_steps():
    """A stopped wall of grain 0 stops grain 1's particles arriving later."""
    require_gpu()
    lam = 5e-6
    p = B.make_params((0, 0, 0), (1e-3,) * 3, lam, lam, lam, W.KIN_A, W.KIN_B, branching=0,
                      cap_particles=1024, cap_stopped=1024, cap_grains=4, cap_claim_bricks=1024)
    ctx = B.Context(p)
    ctx.set_thermal_field(W.Field(W.FIELD_UNIFORM, dT=5.0))
    gap0 = 20.3e-6   # (gap0 - rc) / (v dt) is not an integer: no tie at the meeting step
    c = np.array([[5e-4, 5e-4, 5e-4], [5e-4 - gap0, 5e-4, 5e-4]])
    q = np.array([[1.0, 0, 0, 0]] * 2)
    parts = dict(grain=np.array([0, 1], np.int32), site=np.zeros((2, 3), np.int32),
                 dir=np.array([1, 0], np.int32), s=np.zeros(2), state=np.array([1, 0], np.int32))
    ctx.load_state(c, q, parts, EMPTY_CLAIMS, np.zeros(0, np.int32), 0.0, 0)
    v = 1e-5 * 25 + 1e-6 * 125
    n_meet = int(np.floor((gap0 - lam) / (v * 1e-4))) + 1
    ctx.step(1e-4, n_meet - 1)
    assert ctx.counts()["n_active"] == 1
    ctx.step(1e-4, 1)
    st = ctx.counts()
    assert st["n_active"] == 0 and st["n_stopped"] == 2
