"""Parity at full size: the CET moving-source workload at its 20M-active
snapshot (4 x 2 x 1 mm, lambda0 = 1 um, 256^3 resampled field, 55M stopped
particles), in the launch schedule the bench times (autotuned at the
snapshot).  One step is checked on a sample the oracle computes particle by
particle: every particle active before the step inside a 0.23 x 0.23 x 0.98
mm column (about 150k) advances by v(dT(x) - theta) dt with the FP64
oracle's field and kinetics (Eq. (2)), and its containment decision equals
the FP32 checker's over every particle of the column after the step (the
particles of grains nucleated in the step excepted, which appear after the
containment)."""
import numpy as np
import pytest

import bench
from oracle import Oracle, f32_contain
from tests.gpu_helpers import ident, require_gpu

pytestmark = pytest.mark.gpu

LO = np.array([1.875e-3, 0.875e-3, 0.0])
HI = np.array([2.125e-3, 1.125e-3, 1.0e-3])
INNER = 10e-6   # sample margin: 5 cells of 2 um, far beyond the contact stencil


def _velocity(w, dT):
    v = np.zeros_like(dT)
    pos = dT > 0
    for a, b in zip(w.a, w.b):
        v[pos] += a * dT[pos] ** b
    return v


def test_one_step_at_the_20m_snapshot():
    require_gpu()
    w = bench.cet_workload()
    ctx = bench.make_context(w)
    _, st = bench.advance_to_snapshot(ctx, w, bench.TARGET_ACTIVE)
    assert st["n_active"] >= bench.TARGET_ACTIVE
    ctx.autotune(w.dt, 3)
    c0 = ctx.counts()
    t_n, ng0 = c0["t"], c0["n_grains"]
    p0 = ctx.particles(window=(LO, HI))
    x0 = np.stack([p0["x"], p0["y"], p0["z"]], axis=1).astype(np.float64)
    inner = np.all((x0 > LO + INNER) & (x0 < HI - INNER), axis=1) & (p0["state"] == 0)
    print(f"snapshot: active {c0['n_active']} stopped {c0['n_stopped']}; column "
          f"{len(p0)} particles, {inner.sum()} sampled", flush=True)
    assert inner.sum() > 50000

    ctx.step(w.dt, 1)
    p1 = ctx.particles(window=(LO, HI))
    k0 = ident(p0["grain"], p0["site"], p0["dir"])
    k1 = ident(p1["grain"], p1["site"], p1["dir"])
    assert len(np.unique(k1)) == len(k1)
    order = np.argsort(k1)
    pos = np.searchsorted(k1[order], k0)
    pos = np.minimum(pos, len(k1) - 1)
    found = k1[order][pos] == k0
    same = inner & found          # still there with the same identity (not spawned)
    j = order[pos[same]]
    print(f"sampled {inner.sum()}: {same.sum()} kept their identity", flush=True)
    assert same.sum() > 0.8 * inner.sum()

    # Advance: s += v(dT(x) - theta) dt, dT from the oracle's FP64 sampling
    # of the moving source at t_n.
    o = Oracle.from_workload(w, init=False)
    dT, _ = o.field_value(x0[same], t_n)
    want = _velocity(w, dT - w.theta) * w.dt
    got = p1["s"][j].astype(np.float64) - p0["s"][same].astype(np.float64)
    err = np.abs(got - want)
    tol = 1e-3 * np.abs(want) + 2e-6 * w.lambda0
    print(f"travel: max step {want.max():.3e} m, max error {err.max():.3e} m, "
          f"worst ratio {(err / tol).max():.3f}", flush=True)
    assert np.all(err <= tol)

    # Containment: FP32 distances with the kernel's operation order; the
    # obstacles are every particle of the column after the step except those
    # of grains nucleated in it.
    role = np.where(p1["grain"] < ng0, 2, 0).astype(np.uint8)
    role[j] = 1
    xyz = np.stack([p1["x"], p1["y"], p1["z"]], axis=1)
    dec = f32_contain(xyz, p1["grain"].astype(np.int32), role, np.float32(w.rc * w.rc))
    stopped = p1["state"][j] == 1
    print(f"contained in the sample: gpu {stopped.sum()} checker {dec[j].sum()}", flush=True)
    assert dec[j].sum() > 100
    np.testing.assert_array_equal(stopped.astype(np.uint8), dec[j])
    ctx.close()
