"""The allocation-free particle query (static scratch, no hipMalloc) against
the allocating one, through the C ABI: two calls in a row, the second with a
smaller window, each equal as a set of records to GE_QUERY_PARTICLES on the
same window; device and host outputs agree; an oversized window is refused."""
import numpy as np
import pytest

from paper_2504_12858_amd import binding as B
from paper_2504_12858_amd import workloads as W
from tests.gpu_helpers import context_for, require_gpu

pytestmark = pytest.mark.gpu


def _canon(p):
    p = p.copy()
    p["pad"] = 0
    order = np.lexsort((p["dir"], p["site"][:, 2], p["site"][:, 1], p["site"][:, 0],
                        p["grain"], p["state"]))
    return p[order].tobytes()


def test_noalloc_query_equals_allocating_query():
    torch = require_gpu()
    w = W.cet(seed=3, size=(0.4e-3, 0.2e-3, 0.1e-3), lambda0=4e-6, grid_n=24, dT0=6.0,
              rate=2.0, bulk_density=2e12, face_density=2e8, dt=1.5e-3, U=0.005, q=0.004)
    ctx = context_for(w)
    print("no-alloc query: 200 steps of the scaled CET workload", flush=True)
    ctx.step(w.dt, 200)
    windows = [((0.0, 0.0, 0.0), (0.4e-3, 0.2e-3, 0.1e-3)),
               ((0.1e-3, 0.05e-3, 0.0), (0.25e-3, 0.12e-3, 0.06e-3))]
    sizes = []
    for win in windows:
        want = ctx.particles(window=win)
        got, n = ctx.particles_noalloc(window=win)
        assert n == len(want) > 0
        assert _canon(got) == _canon(want)
        # The same records into device memory.
        dev = torch.zeros(n * B.PARTICLE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        ctx.particles_noalloc(window=win, out=dev)
        back = dev.cpu().numpy().view(B.PARTICLE_DTYPE)
        assert _canon(back) == _canon(want)
        sizes.append(n)
    assert sizes[1] < sizes[0]
    # The whole state (no window) as well.
    allp, n = ctx.particles_noalloc()
    assert _canon(allp) == _canon(ctx.particles())
    ctx.close()


def test_noalloc_query_refuses_more_than_its_staging():
    require_gpu()
    # 1,081,602 particles on the L1 shell of radius 520 lattice steps (2.6 mm),
    # all outside the 1 mm box, so all stopped.
    w = W.single_grain(shell_r=520)
    ctx = context_for(w, cap_particles=1 << 21, cap_stopped=1 << 21, cap_claim_bricks=1 << 20)
    print("no-alloc query: 1,081,602 particles", flush=True)
    with pytest.raises(B.GrainEnvError) as e:
        ctx.particles_noalloc()
    assert e.value.status == B.GE_ECAPACITY
    # A window inside the limit (the cap of the shell around +x, about 1e5
    # particles) still works after the refusal.
    win = ((2.0e-3, -0.6e-3, -0.6e-3), (3.2e-3, 1.6e-3, 1.6e-3))
    got, n = ctx.particles_noalloc(window=win)
    assert 50_000 < n < 1 << 20
    assert _canon(got) == _canon(ctx.particles(window=win))
    ctx.close()
