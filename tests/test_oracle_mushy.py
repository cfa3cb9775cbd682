"""Mushy-zone deposition in the oracle (reading R14: the inside of a grain's
envelope is the set of lattice sites it has reached, each standing for its
crystal-frame cube of edge lambda0; a reached site counts in the node-centred
cell holding its centre).  Pinned by integer brute force on a cube-aligned
lattice ball and by the nucleus generation counts (reached = ball(k))."""
import numpy as np

from oracle import Oracle
from oracle.oracle import f32_deposit
from paper_2504_12858_amd import workloads as W

LAM = 5e-6


def _ball_sites(r):
    s = np.arange(-r, r + 1)
    X, Y, Z = np.meshgrid(s, s, s, indexing="ij")
    keep = np.abs(X) + np.abs(Y) + np.abs(Z) <= r
    return np.stack([X[keep], Y[keep], Z[keep]], axis=1)


def test_cube_aligned_ball_counts_by_integer_brute_force():
    """Identity orientation, centre on node (i0, j0, k0), cells of 3 lambda0:
    site S counts in cell i0 + floor(S / 3 + 1/2) = i0 + (2 S + 3) // 6 per
    axis (never on a face, since 2 S + 3 is odd)."""
    r, m = 9, 3
    c = np.array([5e-4, 5e-4, 5e-4])
    n = (13, 11, 12)
    i0 = np.array([6, 5, 6])
    spacing = np.full(3, m * LAM)
    origin = c - i0 * spacing
    o = Oracle((0, 0, 0), (1e-3, 1e-3, 1e-3), LAM, LAM, LAM, W.KIN_A, W.KIN_B)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=5.0))
    o.init_grains(c[None, :], np.array([[1.0, 0, 0, 0]]), np.array([r], np.int32))
    got = o.deposit_counts(n, origin, spacing)
    want = np.zeros((n[2], n[1], n[0]), np.uint32)
    S = _ball_sites(r)
    idx = i0 + (2 * S + 3) // 6
    for ix, iy, iz in idx:
        want[iz, iy, ix] += 1
    np.testing.assert_array_equal(got, want)
    assert got.sum() == len(S) == (2 * r + 1) * (2 * r * r + 2 * r + 3) // 3
    # Cells wholly inside the ball hold m^3 sites: g^m = 1 there.
    assert got.max() == m ** 3
    # The FP32 checker bins the same sites the same way (cube-aligned rows).
    gtab = np.zeros((1, 24), np.float32)
    gtab[0, :3] = c
    gtab[0, 13:22] = (LAM * np.eye(3)).reshape(-1)
    chk = f32_deposit(np.zeros(len(S), np.int32), S, gtab, n, origin, 1.0 / spacing)
    np.testing.assert_array_equal(chk, want)


def test_nucleus_generations_reach_ball_k():
    """From a 6-point nucleus in uniform undercooling, after k generations the
    reached sites are ball(k) = 1, 7, 25, 63, ...: the counts sum to it."""
    w = W.nucleus_uniform(lambda0=LAM, dT=5.0, quat=W.shoemake_quaternions(W.rng(8), 1)[0])
    o = Oracle.from_workload(w)
    vdt = (W.KIN_A[0] * 25 + W.KIN_A[1] * 125) * 1e-4
    steps_per_gen = int(np.ceil(LAM / vdt))
    n = (40, 40, 40)
    origin = np.array(w.grain_centre[0]) - 20 * 2e-6
    for k in range(1, 4):
        o.step(1e-4, steps_per_gen)
        got = o.deposit_counts(n, origin, (2e-6,) * 3)
        ball = (2 * k + 1) * (2 * k * k + 2 * k + 3) // 3
        assert got.sum() == ball, (k, got.sum(), ball)
