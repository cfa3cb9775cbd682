"""Oracle scenarios run under AddressSanitizer + UndefinedBehaviorSanitizer
(started by tests/test_sanitizers.py with the sanitizer runtime preloaded):
every entry point of the oracle on small inputs."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import oracle as orc  # noqa: E402

orc.LIB_PATH = sys.argv[1]
from oracle import Oracle, f32_cells, f32_contain  # noqa: E402
from paper_2504_12858_amd import workloads as W  # noqa: E402

# Single grain, branching (closed-form case, shortened).
w = W.single_grain(shell_r=8)
o = Oracle.from_workload(w)
o.step(w.dt, 40)
assert o.error == 0 and o.n_active() > 0
o.grain_map(np.array([20, 20, 20], np.int32), np.array([4e-4] * 3), np.array([1e-5] * 3))
o.deposit_counts(np.array([8, 8, 8], np.int32), np.array([4e-4] * 3), np.array([2.5e-5] * 3))
o.contain_decisions(0)
o.contain_decisions(1)
# CET with the moving source, nucleation and melting; periodic axes.
for per in (0, 3):
    w = W.cet(seed=3, size=(0.2e-3, 0.1e-3, 0.05e-3), lambda0=4e-6, grid_n=12, dT0=6.0, rate=2.0,
              bulk_density=2e12, face_density=2e8, dt=1.5e-3, U=0.005, q=0.004)
    w.periodic = per
    o = Oracle.from_workload(w)
    o.set_melting(1)
    o.step(w.dt, 40)
    assert o.error == 0
    o.melt_stats()
    o.site_states()
    p = o.particles()
    c = o.claims()
    g, R = o.grains()
    # Reload the state into a new oracle.
    o2 = Oracle.from_workload(w, init=False)
    o2.nucleate(w.site_xyz, w.site_dTn, w.site_quat)
    quat = np.tile([1.0, 0.0, 0.0, 0.0], (len(g), 1))
    o2.load_state(g, quat, p, c, o.site_states(), o.time, 40)
    o2.step(w.dt, 3)
# Solute field.
w, spec = W.directional_solute(n_steps=10)
o = Oracle.from_workload(w)
o.step(w.dt, 10)
o.field_value(np.array([[1e-4, 1e-4, 1e-4]]), 0.0)
# Adjoint: record, replay, gradient.
w = W.single_grain(shell_r=4)
o = Oracle(w.lo, w.hi, w.lambda0, w.h, w.rc, w.a, w.b, branching=0)
o.set_field(W.Field(W.FIELD_LINEAR, dT0=5.0, grad=(1e3, 0.0, 0.0), rate=1.0))
o.init_grains(w.grain_centre, w.grain_quat, w.grain_shell)
p = o.particles()
nact = o.adjoint_record(1e-4, 20)
parts = dict(grain=p["grain"], site=p["site"], dir=p["dir"], s=p["s"])
o2 = Oracle(w.lo, w.hi, w.lambda0, w.h, w.rc, w.a, w.b, branching=0)
o2.set_field(W.Field(W.FIELD_LINEAR, dT0=5.0, grad=(1e3, 0.0, 0.0), rate=1.0))
o2.init_grains(w.grain_centre, w.grain_quat, w.grain_shell)
o2.adjoint_replay(np.array(w.a), 0.0, parts, nact, 0.0, 1e-4, 20)
o2.adjoint_grad(parts, nact, 0.0, 1e-4, 20, np.ones((len(nact), 3)))
# FP32 checkers.
rng = np.random.default_rng(1)
xyz = rng.random((500, 3)).astype(np.float32) * 1e-4
f32_cells(xyz, np.zeros(3, np.float32), np.float32(1e5), np.array([10, 10, 10], np.int32))
f32_contain(xyz, rng.integers(0, 3, 500).astype(np.int32), np.ones(500, np.uint8), np.float32(1e-12))
print("oracle scenarios clean", flush=True)
