"""Checkpoint and resume through the C ABI: a state saved, loaded into a new
context with twice the capacities and stepped on equals, bit for bit, the
state of the context that was never interrupted (order-independent digests
of particles and claims, grain rows, site states, counts)."""
import numpy as np
import pytest

from paper_2504_12858_amd import binding as B
from paper_2504_12858_amd import workloads as W
from tests.gpu_helpers import context_for, gpu_claims, gpu_parts, ident, require_gpu

pytestmark = pytest.mark.gpu

CAPS = dict(cap_particles=1 << 19, cap_stopped=1 << 19, cap_claim_bricks=1 << 15)
BIG = {k: 2 * v for k, v in CAPS.items()}


def _scaled_cet():
    return W.cet(seed=3, size=(0.4e-3, 0.2e-3, 0.1e-3), lambda0=4e-6, grid_n=24, dT0=6.0,
                 rate=2.0, bulk_density=2e12, face_density=2e8, dt=1.5e-3, n_steps=300,
                 U=0.005, q=0.004)


def _scaled_directional():
    return W.directional(seed=2, n_grains=8, size=(0.3e-3, 0.3e-3, 0.6e-3), dT0=10.0, dt=5e-4)


def _summary(ctx):
    st = ctx.counts()
    return (ctx.digest(), ctx.grains().tobytes(), ctx.site_states().tobytes(),
            {k: st[k] for k in ("n_active", "n_stopped", "n_grains", "n_claim_bricks", "step")},
            st["t"])


@pytest.mark.parametrize("make,n1,n2", [(_scaled_cet, 70, 90), (_scaled_directional, 96, 61)])
def test_save_restore_resume_equals_uninterrupted(make, n1, n2):
    require_gpu()
    w = make()
    print(f"{w.name}: save after {n1} steps, resume for {n2}", flush=True)
    ref = context_for(w, **CAPS)
    ref.step(w.dt, n1 + n2)
    a = context_for(w, **CAPS)
    a.step(w.dt, n1)
    blob = a.save_state()
    hdr = B.state_check(blob)
    assert hdr["step"] == n1 and hdr["bytes"] == blob.nbytes
    assert hdr["n_grains"] == a.counts()["n_grains"]
    a.close()
    # A new context, twice the capacities, no grains and no sites of its own.
    b = B.Context(B.params_from_workload(w, **BIG))
    b.set_thermal_field(w.field)
    b.restore_state(blob)
    assert b.n_sites == len(w.site_dTn)
    b.step(w.dt, n2)
    got, want = _summary(b), _summary(ref)
    assert got[3] == want[3]
    assert got[4] == want[4]
    assert got[1] == want[1], "grain rows"
    assert got[2] == want[2], "site states"
    pb, kb = gpu_parts(b)
    pr, kr = gpu_parts(ref)
    if pb.tobytes() != pr.tobytes():
        for st in (0, 1):
            sb, sr = pb[pb["state"] == st], pr[pr["state"] == st]
            tb = {(int(k), r.tobytes()) for k, r in zip(ident(sb["grain"], sb["site"], sb["dir"]), sb)}
            tr = {(int(k), r.tobytes()) for k, r in zip(ident(sr["grain"], sr["site"], sr["dir"]), sr)}
            only_b = sorted(tb - tr)[:5]
            only_r = sorted(tr - tb)[:5]
            print(f"state {st}: {len(sb)} vs {len(sr)}; only restored {len(tb - tr)}, only "
                  f"uninterrupted {len(tr - tb)}", flush=True)
            for k, raw in only_b:
                print("  restored     ", np.frombuffer(raw, B.PARTICLE_DTYPE), flush=True)
            for k, raw in only_r:
                print("  uninterrupted", np.frombuffer(raw, B.PARTICLE_DTYPE), flush=True)
    np.testing.assert_array_equal(kb, kr)
    assert pb.tobytes() == pr.tobytes()
    cb, _ = gpu_claims(b)
    cr, _ = gpu_claims(ref)
    assert cb.tobytes() == cr.tobytes()
    assert got[0] == want[0], "particle and claim digests"
    # Restoring into a context that already holds the same sites works too.
    c = context_for(w, **CAPS)
    c.restore_state(blob)
    c.step(w.dt, n2)
    assert c.digest() == want[0]
    for x in (b, c, ref):
        x.close()


def test_restore_rejects_other_geometry_sites_and_small_capacities():
    require_gpu()
    w = _scaled_cet()
    a = context_for(w, **CAPS)
    a.step(w.dt, 60)
    blob = a.save_state()
    n_parts = B.state_check(blob)["n_particles"]
    # Another lambda0.
    w2 = _scaled_cet()
    w2.lambda0 = w.lambda0 * 2
    w2.rc = w2.lambda0
    w2.h = w2.lambda0
    b = B.Context(B.params_from_workload(w2, **CAPS))
    with pytest.raises(B.GrainEnvError) as e:
        b.restore_state(blob)
    assert e.value.status == B.GE_EINVAL
    # Other registered sites.
    c = B.Context(B.params_from_workload(w, **CAPS))
    c.set_thermal_field(w.field)
    c.nucleate(w.site_xyz[:3] * 0.5, w.site_dTn[:3], w.site_quat[:3])
    with pytest.raises(B.GrainEnvError) as e:
        c.restore_state(blob)
    assert e.value.status == B.GE_EINVAL
    # Too few particle slots for the saved particles.
    d = B.Context(B.params_from_workload(w, cap_particles=max(64, n_parts // 4),
                                         cap_stopped=1 << 19, cap_claim_bricks=1 << 15))
    with pytest.raises(B.GrainEnvError) as e:
        d.restore_state(blob)
    assert e.value.status == B.GE_ECAPACITY
    # A corrupted blob never reaches the device.
    bad = blob.copy()
    bad[200] ^= 1
    with pytest.raises(B.GrainEnvError) as e:
        a.restore_state(bad)
    assert e.value.status == B.GE_EINVAL
    for x in (a, b, c, d):
        x.close()
