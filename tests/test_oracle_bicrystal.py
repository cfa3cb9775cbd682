"""Behavioural pin: competitive growth in a constant gradient (Sec. 3.3 and
Sec. 4.2 discuss that grains whose <100> axis is aligned with the gradient
overgrow misoriented ones).  Grain A (cube-aligned) and grain B (rotated 30
degrees about y) start side by side on the cold face; A's share of the growth
front rises and ends above one half."""
import numpy as np

from oracle import Oracle
from paper_2504_12858_amd import workloads as W


def _front_share(o, n, vox):
    gm = o.grain_map(n, np.zeros(3), np.array([vox] * 3))
    top = []
    for i in range(n[0]):
        for j in range(n[1]):
            nz = np.flatnonzero(gm[:, j, i])
            if len(nz):
                top.append(gm[nz[-1], j, i])
    return (np.array(top) == 1).mean()


def test_aligned_grain_overgrows_misoriented_grain():
    w = W.bicrystal(dt=2e-3)
    o = Oracle.from_workload(w)
    n = np.array([50, 10, 100], np.int32)
    shares = []
    for k in range(10):
        o.step(w.dt, 100)
        assert o.error == 0
        shares.append(_front_share(o, n, 20e-6))
    late = shares[4:]
    assert all(b >= a for a, b in zip(late, late[1:])), shares
    assert shares[-1] > 0.6
