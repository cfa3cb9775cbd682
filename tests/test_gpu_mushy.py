"""Mushy-zone deposition on the GPU (the volume inside the envelopes per
cell of a deposition grid): counts kept step by step through branching,
nucleation and new grains equal the FP32 checker on the GPU's own reached
sites and grain rows, bit for bit; they equal a recount from the claims and
the counts after a state load; they agree with the FP64 oracle's run; the
fraction query is min(1, count lambda0^3 / V); and the error paths."""
import numpy as np
import pytest

from oracle import Oracle
from oracle.oracle import f32_deposit
from paper_2504_12858_amd import binding as B
from paper_2504_12858_amd import workloads as W
from tests.gpu_helpers import context_for, gpu_state_for_oracle, require_gpu

pytestmark = pytest.mark.gpu


def _cet():
    return W.cet(seed=3, size=(0.4e-3, 0.2e-3, 0.1e-3), lambda0=4e-6, grid_n=24, dT0=6.0,
                 rate=2.0, bulk_density=2e12, face_density=2e8, dt=1.5e-3, n_steps=300,
                 U=0.005, q=0.004)


def _grid(w, cells=(24, 12, 6)):
    spacing = tuple((h - l) / c for l, h, c in zip(w.lo, w.hi, cells))
    origin = tuple(l + 0.5 * s for l, s in zip(w.lo, spacing))
    return cells, origin, spacing


def _checker(ctx, n, origin, spacing):
    c = ctx.claims()
    reached = (c["flags"] & 2) != 0
    gtab = np.zeros((ctx.counts()["n_grains"], 24), np.float32)
    ctx.query_envelope(B.QUERY_GRAINS, gtab)
    inv = (1.0 / np.asarray(spacing, np.float64)).astype(np.float32)
    return f32_deposit(c["grain"][reached].astype(np.int32), c["site"][reached], gtab, n,
                       np.asarray(origin, np.float32), inv)


def test_deposition_counts_match_the_fp32_checker():
    require_gpu()
    w = _cet()
    n, origin, spacing = _grid(w)
    ctx = context_for(w)
    ctx.set_deposition_grid(n, origin, spacing)
    print(f"cet scaled with deposition: {w.n_steps} steps", flush=True)
    st = ctx.step(w.dt, w.n_steps)
    assert st["nucleated"] > 10
    got = ctx.mushy_counts()
    want = _checker(ctx, n, origin, spacing)
    print(f"reached sites counted {got.sum()} checker {want.sum()}", flush=True)
    assert want.sum() > 10000
    np.testing.assert_array_equal(got, want)
    # A recount from the claims gives the same counts.
    ctx.set_deposition_grid(n, origin, spacing)
    np.testing.assert_array_equal(ctx.mushy_counts(), want)
    # g^m = min(1, count lambda0^3 / V).
    gm = ctx.mushy_fraction()
    site_over_cell = w.lambda0 ** 3 / np.prod(spacing)
    np.testing.assert_array_equal(
        gm, np.minimum(1.0, got.astype(np.float64) * site_over_cell).astype(np.float32))
    assert gm.max() == 1.0 and gm.min() == 0.0
    ctx.close()


def test_deposition_agrees_with_the_oracle_run():
    require_gpu()
    w = _cet()
    n, origin, spacing = _grid(w)
    ctx = context_for(w)
    ctx.set_deposition_grid(n, origin, spacing)
    ctx.step(w.dt, w.n_steps)
    o = Oracle.from_workload(w)
    o.step(w.dt, w.n_steps)
    assert o.error == 0
    g = ctx.mushy_counts().astype(np.int64)
    r = o.deposit_counts(n, origin, spacing).astype(np.int64)
    rel = np.abs(g - r).sum() / r.sum()
    print(f"reached gpu {g.sum()} oracle {r.sum()} relative cell difference {rel:.2e}", flush=True)
    assert abs(g.sum() - r.sum()) <= 1e-3 * r.sum()
    assert rel <= 2e-3
    ctx.close()


def _grains(ctx, w):
    """Centres and quaternions of the grains of a CET run: every grain comes
    from a fired site, identified by its FP32 centre."""
    rows = ctx.grains()
    key = {tuple(np.float32(v) for v in xyz): i for i, xyz in enumerate(w.site_xyz)}
    idx = np.array([key[tuple(r[:3])] for r in rows])
    return w.site_xyz[idx], w.site_quat[idx]


def test_deposition_after_state_load():
    """A state loaded into a context with a deposition grid is counted again."""
    require_gpu()
    w = _cet()
    n, origin, spacing = _grid(w)
    a = context_for(w)
    a.set_deposition_grid(n, origin, spacing)
    a.step(w.dt, 120)
    parts, claims = gpu_state_for_oracle(a, None, None)
    centre, quat = _grains(a, w)
    st = a.counts()
    b = context_for(w)
    b.set_deposition_grid(n, origin, spacing)
    b.load_state(centre, quat, parts, claims, a.site_states(), st["t"], st["step"])
    np.testing.assert_array_equal(b.grains(), a.grains())
    np.testing.assert_array_equal(b.mushy_counts(), a.mushy_counts())
    a.close()
    b.close()


def test_deposition_errors():
    require_gpu()
    w = _cet()
    ctx = context_for(w)
    with pytest.raises(B.GrainEnvError):           # no grid set
        ctx.query_envelope(B.QUERY_MUSHY_COUNTS, np.zeros(8, np.uint32))
    with pytest.raises(B.GrainEnvError):           # larger than field_n
        ctx.set_deposition_grid((w.field.n[0] + 1, 4, 4), (0, 0, 0), (1e-5,) * 3)
    with pytest.raises(B.GrainEnvError):           # bad spacing
        ctx.set_deposition_grid((4, 4, 4), (0, 0, 0), (1e-5, 0.0, 1e-5))
    ctx.set_deposition_grid((4, 4, 4), (0, 0, 0), (1e-4,) * 3)
    ctx.set_deposition_grid(None)
    with pytest.raises(B.GrainEnvError):           # turned off
        ctx.query_envelope(B.QUERY_MUSHY_COUNTS, np.zeros(64, np.uint32))
    ctx.close()
