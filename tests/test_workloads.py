"""Statistical checks of the seeded input generators."""
import math

import numpy as np
from scipy import stats

from paper_2504_12858_amd import workloads as W


def test_truncated_normal_bounds_and_moments():
    x = W.truncated_normal(W.rng(1), 200000, 5.0, 1.0, 0.0, 10.0)
    assert x.min() >= 0 and x.max() <= 10
    # Truncation at +-5 sigma changes the moments by < 1e-5.
    assert abs(x.mean() - 5.0) < 4 / math.sqrt(x.size)
    assert abs(x.std() - 1.0) < 0.01


def test_shoemake_rotation_angle_density():
    """Uniform rotations have angle density (1 - cos w)/pi on [0, pi]."""
    q = W.shoemake_quaternions(W.rng(2), 100000)
    np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, rtol=1e-12)
    w = 2 * np.arccos(np.clip(np.abs(q[:, 0]), 0, 1))
    res = stats.kstest(w, lambda t: (t - np.sin(t)) / np.pi)
    assert res.pvalue > 1e-3


def test_bunge_identity_and_axis():
    np.testing.assert_allclose(W.bunge_quaternion(0, 0, 0), [1, 0, 0, 0])
    q = W.bunge_quaternion(90, 0, 0)
    np.testing.assert_allclose(q, [math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)], atol=1e-15)


def test_cet_workload_counts():
    w = W.cet()
    n_face = int(round(1e8 * 4e-3 * 2e-3))
    n_bulk = int(round(1e11 * 8e-9))
    assert len(w.site_dTn) == n_face + n_bulk == 1600
    assert (w.site_dTn[:n_face] == 0).all()
    assert (w.site_xyz[:n_face, 2] == 0).all()
    b = w.site_dTn[n_face:]
    assert b.min() >= 0 and b.max() <= 10
    # Same seed, same draws.
    w2 = W.cet()
    np.testing.assert_array_equal(w.site_xyz, w2.site_xyz)
