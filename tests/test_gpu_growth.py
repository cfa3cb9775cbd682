"""GPU (HIP, FP32) growth and branching against the closed forms and the FP64
oracle: single-grain octahedron, nucleus generations, tilted-grain parity."""
import math

import numpy as np
import pytest

from oracle import Oracle
from paper_2504_12858_amd import workloads as W
from tests.gpu_helpers import context_for, gpu_claims, gpu_parts, orc_claims, orc_parts, require_gpu

pytestmark = pytest.mark.gpu


def shell(r):
    return 4 * r * r + 2 if r > 0 else 1


def ball(r):
    return (2 * r + 1) * (2 * r * r + 2 * r + 3) // 3


def test_single_grain_closed_form_on_gpu():
    require_gpu()
    w = W.single_grain()
    ctx = context_for(w)
    print("single grain: 10002 particles, 200 steps", flush=True)
    v = 1e-5 * 25 + 1e-6 * 125
    for n in range(1, w.n_steps + 1):
        st = ctx.step(w.dt, 1)
        if n == 133:
            assert st["n_active"] == 10002 and st["spawners"] == 0
        if n == 134:
            assert st["spawners"] == 10002
            assert st["n_active"] == 10810
    assert st["n_active"] == 10810 and st["n_stopped"] == 0
    p, key = gpu_parts(ctx)
    c = np.array(w.grain_centre[0])
    l1 = np.abs(np.stack([p["x"], p["y"], p["z"]], 1).astype(np.float64) - c).sum(1)
    expect = 50 * w.lambda0 + 200 * v * w.dt
    # FP32 positions near 0.5 mm: a few ulps (6e-11 m) per coordinate.
    np.testing.assert_allclose(l1, expect, rtol=0, atol=1e-9)
    cl, _ = gpu_claims(ctx)
    assert len(cl) == ball(50) + 10002 + 10810
    # Same identities as the oracle, positions within 1e-5 of the box.
    o = Oracle.from_workload(w)
    o.step(w.dt, w.n_steps)
    q, okey = orc_parts(o)
    np.testing.assert_array_equal(key, okey)
    xyz = np.stack([p["x"], p["y"], p["z"]], 1).astype(np.float64)
    assert np.abs(xyz - q["x"]).max() <= 1e-5 * w.box_size
    oc, ockey = orc_claims(o)
    _, gckey = gpu_claims(ctx)
    np.testing.assert_array_equal(gckey, ockey)


@pytest.mark.parametrize("seed", [0, 11])
def test_nucleus_generations_on_gpu(seed):
    require_gpu()
    quat = (1, 0, 0, 0) if seed == 0 else W.shoemake_quaternions(W.rng(seed), 1)[0]
    w = W.nucleus_uniform(lambda0=5e-6, dT=4.7, quat=quat)
    ctx = context_for(w)
    v = 1e-5 * 4.7 ** 2 + 1e-6 * 4.7 ** 3
    dt = 1e-3
    k_done = 0
    for n in range(1, 96):
        st = ctx.step(dt, 1)
        k = int(math.floor(n * v * dt / w.lambda0))
        if k > k_done:
            k_done = k
            assert st["n_active"] == shell(k + 1), (n, k)
            reached = (gpu_claims(ctx)[0]["flags"] & 2).astype(bool).sum()
            assert reached == ball(k)
    assert k_done >= 6


def test_tilted_grain_in_gradient_matches_oracle():
    """Sec. 3.1 setting on the GPU: every particle identity and position agrees
    with the oracle after 300 steps of 0.01 s."""
    require_gpu()
    lam = 200e-6
    L = 0.04
    c = np.array([L / 2] * 3)
    G, rate, dT0 = 250.0, 0.1, 2.0
    q = W.bunge_quaternion(20, 20, 20)
    fld = W.Field(W.FIELD_LINEAR, dT0=dT0 + G * c[2], grad=(0, 0, -G), rate=rate)
    w = W.Workload(name="tilted", lo=(0, 0, 0), hi=(L, L, L), lambda0=lam, h=lam, rc=lam,
                   a=(1e-4, 0.0), b=(2.0, 3.0), theta=0.0, dt=0.01, n_steps=300, field=fld,
                   grain_centre=c[None, :], grain_quat=q[None, :], grain_shell=np.zeros(1, np.int32))
    ctx = context_for(w)
    ctx.step(w.dt, w.n_steps)
    o = Oracle.from_workload(w)
    o.step(w.dt, w.n_steps)
    p, key = gpu_parts(ctx)
    r, okey = orc_parts(o)
    np.testing.assert_array_equal(key, okey)
    xyz = np.stack([p["x"], p["y"], p["z"]], 1).astype(np.float64)
    assert np.abs(xyz - r["x"]).max() <= 1e-5 * L
    np.testing.assert_array_equal(p["state"], r["state"])
