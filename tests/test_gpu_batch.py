"""Batched launches: contexts of different sizes and kinds advanced together
give, call after call, bitwise the states and counters of the same contexts
stepped alone."""
import numpy as np
import pytest

from paper_2504_12858_amd import binding as B
from paper_2504_12858_amd import workloads as W
from tests.gpu_helpers import context_for, gpu_claims, gpu_parts, require_gpu

pytestmark = pytest.mark.gpu

CAPS = dict(cap_particles=1 << 20, cap_stopped=1 << 20, cap_claim_bricks=1 << 16)
DT = 5e-4


def _workloads():
    return [
        W.directional(seed=11, n_grains=8, size=(0.3e-3, 0.3e-3, 0.6e-3), dT0=10.0, h=10e-6),
        W.directional(seed=12, n_grains=3, size=(0.2e-3, 0.2e-3, 0.3e-3), dT0=9.0),
        W.cet(seed=5, size=(0.4e-3, 0.2e-3, 0.1e-3), lambda0=4e-6, grid_n=24, dT0=6.0, rate=2.0,
              bulk_density=2e12, face_density=2e8, U=0.005, q=0.004),
        W.single_grain(shell_r=6),
        W.directional(seed=13, n_grains=16, size=(0.4e-3, 0.4e-3, 0.4e-3), dT0=10.0),
    ]


def _state(ctx):
    p, _ = gpu_parts(ctx)
    c, _ = gpu_claims(ctx)
    return p.tobytes(), c.tobytes()


def _stats(st):
    st = dict(st)
    st.pop("pair_tests")  # depends on the order within a cell
    return st


def test_batch_equals_plain_contexts():
    require_gpu()
    ws = _workloads()
    batch = B.Batch([B.params_from_workload(w, **CAPS) for w in ws])
    for m, w in zip(batch.members, ws):
        m.init_from_workload(w)
    refs = [context_for(w, **CAPS) for w in ws]
    for n in (40, 7, 33, 48):
        print(f"batch step {n}", flush=True)
        got = batch.step(DT, n)
        for i, (r, w) in enumerate(zip(refs, ws)):
            want = r.step(DT, n)
            assert _stats(got[i]) == _stats(want), (i, n)
            assert _state(batch.members[i]) == _state(r), (i, n)
    # A member stepped alone between batched steps, then the batch again.
    batch.members[2].step(DT, 5)
    refs[2].step(DT, 5)
    batch.step(DT, 16)
    for r in refs:
        r.step(DT, 16)
    for i, r in enumerate(refs):
        assert _state(batch.members[i]) == _state(r), i
        r.close()
    batch.close()


def test_batch_with_periodic_members_equals_plain_contexts():
    """Members with periodic lateral boundaries and members without share the
    batched launches (which then decide per member); each equals its plain
    context bit for bit."""
    require_gpu()
    ws = _workloads()[:2]
    per = W.directional(seed=11, n_grains=8, size=(0.3e-3, 0.3e-3, 0.6e-3), dT0=10.0, h=10e-6)
    per.periodic = 3
    ws = [per] + ws
    batch = B.Batch([B.params_from_workload(w, **CAPS) for w in ws])
    for m, w in zip(batch.members, ws):
        m.init_from_workload(w)
    refs = [context_for(w, **CAPS) for w in ws]
    for n in (40, 33, 64):
        got = batch.step(DT, n)
        for i, r in enumerate(refs):
            want = r.step(DT, n)
            assert _stats(got[i]) == _stats(want), (i, n)
            assert _state(batch.members[i]) == _state(r), (i, n)
    p = batch.members[0].particles()
    assert ((p["x"] < 0) | (p["x"] >= 0.3e-3) | (p["y"] < 0) | (p["y"] >= 0.3e-3)).any()
    for r in refs:
        r.close()
    batch.close()


def test_batch_schedule_and_graphs_keep_results():
    """Odd block totals, the autotuner and graphs off change only speed."""
    require_gpu()
    ws = _workloads()[:3]
    outs = []
    for mode in range(3):
        batch = B.Batch([B.params_from_workload(w, **CAPS) for w in ws])
        for m, w in zip(batch.members, ws):
            m.init_from_workload(w)
        if mode == 1:
            batch.set_blocks({"advance": 24, "branch": 8, "contain": 4096, "dirty": 40,
                              "scatter": 16, "children": 64, "stoplink": 8,
                              "cellscan": 512})
            batch.use_graphs(False)
        if mode == 2:
            batch.step(DT, 3)
            before = [_state(m) for m in batch.members]
            best = batch.autotune(DT, 2)
            assert all(v > 0 for v in best.values())
            assert [_state(m) for m in batch.members] == before
            best = batch.autotune(DT, 1, restore=False)
        steps = [m.counts()["step"] for m in batch.members]
        assert len(set(steps)) == 1 and steps[0] < 160
        batch.step(DT, 160 - steps[0])
        outs.append([_state(m) for m in batch.members])
        batch.close()
    assert outs[0] == outs[1] == outs[2]


def test_hold_and_digest():
    """A held context does not change (digest, step count); released, it
    continues exactly like a context that was never held.  Equal states have
    equal digests, different states different ones."""
    require_gpu()
    ws = _workloads()[:2]
    batch = B.Batch([B.params_from_workload(w, **CAPS) for w in ws])
    for m, w in zip(batch.members, ws):
        m.init_from_workload(w)
    refs = [context_for(w, **CAPS) for w in ws]
    batch.step(DT, 20)
    for r in refs:
        r.step(DT, 20)
    d0 = batch.members[0].digest()
    assert d0 == refs[0].digest() and d0 != refs[1].digest()
    batch.members[0].hold(True)
    st = batch.step(DT, 40)
    assert st[0]["advanced"] == 0 and st[0]["step"] == 20
    assert batch.members[0].digest() == d0
    refs[1].step(DT, 40)
    assert batch.members[1].digest() == refs[1].digest()
    batch.members[0].hold(False)
    batch.step(DT, 33)
    refs[0].step(DT, 33)
    refs[1].step(DT, 33)
    for m, r in zip(batch.members, refs):
        assert m.digest() == r.digest()
        assert _state(m) == _state(r)
        r.close()
    batch.close()


def test_batch_members_against_the_oracle():
    """Batched members against the FP64 oracle, each run as its own oracle
    simulation: two directional realisations (different seeds: positions and
    orientations of the grains) and a scaled CET member (moving source,
    nucleation) agree on >= 99.9 % of grain-map voxels; a single grain keeps
    the oracle's particle identities, with positions within 1e-5 of the box."""
    require_gpu()
    from oracle import Oracle
    from tests.gpu_helpers import orc_parts
    n_steps = 480
    sg = W.single_grain(shell_r=6)
    sg.field = W.Field(W.FIELD_UNIFORM, dT=4.7)  # no travel total on a multiple of lambda0
    ws = [W.directional(seed=2, n_grains=8, size=(0.3e-3, 0.3e-3, 0.6e-3), dT0=10.0),
          W.directional(seed=21, n_grains=8, size=(0.3e-3, 0.3e-3, 0.6e-3), dT0=10.0),
          W.cet(seed=3, size=(0.4e-3, 0.2e-3, 0.1e-3), lambda0=4e-6, grid_n=24, dT0=6.0,
                rate=6.0, bulk_density=2e12, face_density=2e8, U=0.005, q=0.004),
          sg]
    batch = B.Batch([B.params_from_workload(w, **CAPS) for w in ws])
    for m, w in zip(batch.members, ws):
        m.init_from_workload(w)
    print(f"batch of {len(ws)} members: {n_steps} steps", flush=True)
    batch.step(DT, n_steps)
    for i, (m, w) in enumerate(zip(batch.members, ws)):
        o = Oracle.from_workload(w)
        o.step(DT, n_steps)
        assert o.error == 0
        if w.name == "single_grain":
            p, key = gpu_parts(m)
            q, okey = orc_parts(o)
            np.testing.assert_array_equal(key, okey)
            xyz = np.stack([p["x"], p["y"], p["z"]], 1).astype(np.float64)
            err = np.abs(xyz - q["x"]).max()
            print(f"member {i} single grain: {len(p)} particles, max |dx| {err:.3e} m",
                  flush=True)
            assert err <= 1e-5 * w.box_size
            continue
        vox = 5e-6 if w.name == "directional" else 4e-6
        n = [int(round((h - l) / vox)) for l, h in zip(w.lo, w.hi)]
        gm = m.grain_map(n, w.lo, [vox] * 3)
        om = o.grain_map(np.array(n, np.int32), np.array(w.lo), np.array([vox] * 3))
        agree, solid = (gm == om).mean(), (om > 0).mean()
        print(f"member {i} {w.name}: map agreement {agree:.6f}, solid {solid:.3f}", flush=True)
        assert solid > 0.02
        assert agree >= 0.999
        if len(w.site_dTn):
            fired_gpu, fired_orc = m.site_states() == 1, o.site_states() == 1
            assert fired_gpu.sum() > 5
            assert (fired_gpu != fired_orc).sum() <= max(1, 0.01 * fired_orc.sum())
    batch.close()
