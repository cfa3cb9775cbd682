#!/usr/bin/env python3
"""Envelope particle-updates/s of the plain grain-envelope step on one MI355X.

Workload: columnar-to-equiaxed transition under a moving Rosenthal source
(4 x 2 x 1 mm box, 256^3 FP32 undercooling grid resampled every step, 800
face and 800 bulk nuclei, lambda0 = rc = 1 um, cells of h = 2 um, dT0 = 12 K), advanced
untimed from t = 0 to the first step with >= 20M active particles.  Then W
warm-up steps (an event between every two phases: the dominant phase) and K
timed steps with two events per step around the dominant phase alone,
bracketed by stream synchronisations; then one re-sort interval of steps with
an event between every two phases gives the phase table.

value     = particle updates (active particles advanced) over the K steps / s
roofline  = the dominant phase's algorithmic bytes per launch / its average
            launch duration (HIP events around it on the context's stream in
            every timed step), against the 8 TB/s HBM peak
step_roofline = value x the method's algorithmic bytes per update of the whole
            step (83 B at this workload) against the same peak
cpu_baseline = the FP64 oracle stepping a spatial window of the same snapshot
            on the host cores

The timed region (and the batched leg's timed steps) is bracketed by
roctxProfilerResume / roctxProfilerPause, so `rocprofv3 --selected-regions`
records exactly the timed launches.
`--copy-probe MB` instead runs a plain device copy of MB megabytes inside such
a region (the calibration of the HBM byte counters) and exits.

Progress goes to stderr; one JSON line goes to stdout.
"""
import argparse
import ctypes
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "envelope particle-updates/s @20M FP32 vs plain; batched & adjoint vs plain"
CET_KNOBS = dict(dT0=12.0, lambda0=1e-6, h=2e-6)
TARGET_ACTIVE = 20_000_000
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per particle update of the whole step at this workload:
# read state 20, write position and travel 16, write the cell-ordered record
# 16, read it in the containment sweep 16, cell key 8, field resample write
# and gather read 2 x 64 MiB per step over ~20M updates 6.7.
STEP_BYTES_PER_UPDATE = 83.0
KERNEL_SOURCES = ("paper_2504_12858_amd/csrc/kernels.hip", "paper_2504_12858_amd/csrc/internal.h")

# Algorithmic bytes per unit of each phase (what the method must move):
#   advance  : read and write the 16-B record of each active particle
#   scatter  : read a record, write it and its 16-B position to their cell slot
#   contain  : read each active position once (neighbours counted in their own cell)
#   branch   : read and write the spawner's record
#   resort   : read and write record and position of each stopped particle
#   resample : write one FP32 node value
PHASE_BYTES = {"advance": 32, "scatter": 48, "contain": 16, "branch": 32, "resample": 4,
               "children": 48, "dirty": 16}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class ProfilerRegion:
    """roctxProfilerResume / Pause when the roctx library is present (a no-op
    without a profiler attached)."""

    def __init__(self):
        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"):
            try:
                self.lib = ctypes.CDLL(name)
                break
            except OSError:
                continue

    def resume(self):
        if self.lib is not None:
            self.lib.roctxProfilerResume(ctypes.c_uint64(0))

    def pause(self):
        if self.lib is not None:
            self.lib.roctxProfilerPause(ctypes.c_uint64(0))


# Loaded before the HIP runtime starts, so that a profiler attached to the
# process intercepts the region calls.
REGION = ProfilerRegion()


def kernel_sources_sha():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _traffic_fields():
    """Machine-read fields of the committed counter summaries
    (profiles/*hbm_traffic*.md) taken on the current kernel sources."""
    sha = kernel_sources_sha()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*hbm_traffic*.md"))):
        text = open(path).read()
        fields = dict(re.findall(r"^- ([\w\[\]]+): `([^`]*)`", text, flags=re.M))
        if fields.get("kernel_sources_sha256") == sha:
            yield fields


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the counters (FETCH_SIZE +
    WRITE_SIZE, calibrated), or None when no summary was taken on the current
    kernel sources."""
    for f in _traffic_fields():
        v = f.get(f"traffic_bytes_per_launch[{kernel}]")
        if v is not None:
            return float(v)
        if f.get("kernel") == kernel:
            return float(f["traffic_bytes_per_launch"])
    return None


def measured_step_traffic():
    """HBM bytes per step of every kernel of the step, from the counters, or
    None (see measured_traffic)."""
    for f in _traffic_fields():
        if "traffic_bytes_per_step" in f:
            return float(f["traffic_bytes_per_step"])
    return None


def copy_probe(mb):
    """A plain device copy (elementwise multiply by one) of `mb` MB, three
    times, inside a profiler region: reads and writes mb MB per launch."""
    import torch
    n = int(mb * 1e6) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    REGION.resume()
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    REGION.pause()
    print(json.dumps({"copy_probe_bytes": 4 * n, "launches": 3}), flush=True)


def cet_workload():
    from paper_2504_12858_amd import workloads as W
    return W.cet(**CET_KNOBS)


# Steps between re-sorts of the stopped store for the CET workload (the
# containment's recent-stop lists grow with it, the re-sort's share falls).
RESORT_EVERY = 24


def make_context(w):
    from paper_2504_12858_amd import binding as B
    # Room for the legs that run on after the timed steps (melting,
    # deposition, solute: about 600 more steps, to about 30M active and more
    # than 130M stopped particles).
    return B.Context.from_workload(w, cap_particles=1 << 26, cap_stopped=1 << 28,
                                   cap_claim_bricks=1 << 25, cap_grains=4096,
                                   resort_every=RESORT_EVERY)


def advance_to_snapshot(ctx, w, target, max_steps=6000, chunk=50):
    steps = 0
    st = None
    while steps < max_steps:
        st = ctx.step(w.dt, chunk)
        steps += chunk
        log(f"[snapshot] step {steps} active {st['n_active']} stopped {st['n_stopped']} "
            f"grains {st['n_grains']}")
        if st["n_active"] >= target:
            break
    return steps, st


def grain_quaternions(ctx, w):
    """Centres and quaternions of the context's grains: every grain of the
    CET workload comes from a fired site, identified by its FP32 centre."""
    import numpy as np
    rows = ctx.grains()
    key = {tuple(np.float32(v) for v in xyz): i for i, xyz in enumerate(w.site_xyz)}
    idx = np.array([key[tuple(r[:3])] for r in rows])
    return w.site_xyz[idx], w.site_quat[idx]


ADJ_STORED = 512_000
ADJ_STEPS = 500
ADJ_CKPT = 50


def adjoint_leg():
    """Recorded forward + adjoint backward against the plain forward over the
    same window: directional growth (2 x 2 x 4 mm, linear field), 16 grains
    (seed 5), branching on until >= 512k stored particles, then a 500-step
    window with branching off; checkpoints every 50 steps; gradients of
    L = sum |x_N - xhat|^2 at (a0, a1, theta = 0), targets from a run with
    a * 1.05 and theta = +2 K."""
    import torch
    from paper_2504_12858_amd import workloads as W
    from paper_2504_12858_amd import binding as B
    from paper_2504_12858_amd.adjoint import AdjointRun
    w = W.directional(seed=5, n_grains=16)
    ctx = B.Context.from_workload(w, cap_particles=1 << 21, cap_stopped=1 << 21,
                                  cap_claim_bricks=1 << 18)
    steps = 0
    while steps < 6000:
        st = ctx.step(w.dt, 50)
        steps += 50
        if st["n_active"] + st["n_stopped"] >= ADJ_STORED:
            break
    log(f"[adjoint] snapshot at step {steps}: {st['n_active']} active, {st['n_stopped']} stopped")
    run = AdjointRun.capture(ctx, w.b, w.dt, ADJ_STEPS, ADJ_CKPT)
    a = tuple(w.a)

    def restore(a0, a1, th):
        run.restore()
        ctx.set_model((a0, a1), w.b, th, 0)
        torch.cuda.synchronize()

    restore(a[0] * 1.05, a[1] * 1.05, 2.0)
    ctx.adjoint_forward(w.dt, ADJ_STEPS, ADJ_CKPT)
    xhat = ctx.adjoint_positions().clone()
    # Warm-up of both paths (first launches load code objects).
    restore(a[0], a[1], 0.0)
    ctx.step(w.dt, 20)
    restore(a[0], a[1], 0.0)
    ctx.adjoint_forward(w.dt, ADJ_STEPS, ADJ_CKPT)
    ctx.adjoint_backward(2.0 * (ctx.adjoint_positions() - xhat))
    restore(a[0], a[1], 0.0)
    t0 = time.perf_counter()
    plain = ctx.step(w.dt, ADJ_STEPS)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    restore(a[0], a[1], 0.0)
    t0 = time.perf_counter()
    n = ctx.adjoint_forward(w.dt, ADJ_STEPS, ADJ_CKPT)
    x = ctx.adjoint_positions()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dLdx = 2.0 * (x - xhat)
    grad = ctx.adjoint_backward(dLdx)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    loss = float(((x.double() - xhat.double()) ** 2).sum())
    acc = adjoint_accuracy(ctx, run, w, a, xhat, dLdx, grad)
    ctx.close()
    return {"workload": "directional-16-grains-512k-500-steps", "tracked": int(n),
            "snapshot_step": steps, "steps": ADJ_STEPS, "ckpt_every": ADJ_CKPT,
            "plain_forward_ms": round(1e3 * t_plain, 3),
            "recorded_forward_ms": round(1e3 * (t1 - t0), 3),
            "backward_ms": round(1e3 * (t2 - t1), 3),
            "ratio_vs_plain": round((t2 - t0) / t_plain, 4),
            "plain_updates": int(plain["advanced"]),
            "active_per_step": round(plain["advanced"] / ADJ_STEPS),
            "loss": loss, "grad_a0_a1_theta": [float(v) for v in grad], "accuracy": acc}


ADJ_SAMPLE = 20_000
ADJ_FD_H = 1e-4


def adjoint_accuracy(ctx, run, w, a, xhat, dLdx, grad):
    """Gradient errors of the adjoint leg.
    (1) Central differences of L = sum |x_N - xhat|^2 on the HIP path: six
        more recorded forwards at a0 (1 +- h), a1 (1 +- h) (h = 1e-4
        relative) and theta = +-1e-4 K (absolute: theta = 0 at the point).
        These runs take their own masks, as the target run does, so a
        particle that stops one step earlier or later in a perturbed run
        adds a jump the frozen-mask gradient does not see.  Hence also the
        same differences over the particles that advance the same number of
        steps in the three runs of each parameter, against the adjoint
        gradient of that part of L.
    (2) The FP64 oracle's adjoint on the GPU's masks for a seeded sample of
        20k tracked particles (dL/dx zero outside the sample), and the
        oracle's FP64 replay of their final positions."""
    import numpy as np
    import torch
    from oracle import Oracle
    from paper_2504_12858_amd import binding as B
    from paper_2504_12858_amd import workloads as W
    t0 = B.state_check(run.blob)["t"]
    base = (a[0], a[1], 0.0)
    steps = (ADJ_FD_H * a[0], ADJ_FD_H * a[1], ADJ_FD_H)
    run.forward(*base)
    nact0 = ctx.adjoint_tracked()["nact"].copy()
    xh = xhat.double()
    fd, fd_same, same = [], [], []
    for k in range(3):
        Ls, Ls_same, nacts = [], [], []
        r2 = []
        for sg in (1.0, -1.0):
            p = list(base)
            p[k] += sg * steps[k]
            xp = run.forward(*p)
            nacts.append(ctx.adjoint_tracked()["nact"].copy())
            r2.append(((xp.double() - xh) ** 2).sum(dim=1))
        keep = (nacts[0] == nact0) & (nacts[1] == nact0)
        m = torch.from_numpy(keep).to(xh.device)
        Ls = [float(v.sum()) for v in r2]
        Ls_same = [float((v * m).sum()) for v in r2]
        fd.append((Ls[0] - Ls[1]) / (2 * steps[k]))
        fd_same.append((Ls_same[0] - Ls_same[1]) / (2 * steps[k]))
        same.append(keep)
    fd, fd_same = np.array(fd), np.array(fd_same)
    g = np.array(grad, np.float64)
    rel_fd = np.abs(g - fd) / np.abs(fd)
    # The base recorded run again (the FD runs replaced the recording).
    run.forward(*base)
    g_same = []
    for k in range(3):
        d_k = dLdx.detach().clone()
        d_k[torch.from_numpy(~same[k]).to(d_k.device)] = 0.0
        g_same.append(float(ctx.adjoint_backward(d_k)[k]))
    g_same = np.array(g_same)
    rel_fd_same = np.abs(g_same - fd_same) / np.abs(fd_same)
    tr = ctx.adjoint_tracked()
    n = len(tr)
    idx = np.sort(W.rng(7).choice(n, size=min(ADJ_SAMPLE, n), replace=False))
    d_all = dLdx.detach().float().cpu().numpy()
    d_s = np.zeros_like(d_all)
    d_s[idx] = d_all[idx]
    g_s = np.array(ctx.adjoint_backward(torch.from_numpy(d_s).cuda()))
    o = Oracle(w.lo, w.hi, w.lambda0, w.h, w.rc, w.a, w.b, w.theta, 0, w.box_exit, w.periodic)
    o.set_field(w.field)
    o.init_grains(w.grain_centre, w.grain_quat, np.zeros(len(w.grain_centre), np.int32))
    parts = dict(grain=tr["grain"][idx].astype(np.int32), site=tr["site"][idx].astype(np.int32),
                 dir=tr["dir"][idx].astype(np.int32), s=tr["s0"][idx].astype(np.float64))
    go = o.adjoint_grad(parts, tr["nact"][idx], t0, w.dt, ADJ_STEPS,
                        d_s[idx].astype(np.float64))
    xo = o.adjoint_replay(np.array(w.a), 0.0, parts, tr["nact"][idx], t0, w.dt, ADJ_STEPS)
    xg = ctx.adjoint_positions().cpu().numpy()[idx].astype(np.float64)
    box = max(h - l for l, h in zip(w.lo, w.hi))
    rel_o = np.abs(g_s - go) / np.abs(go)
    return {"fd_h_relative": ADJ_FD_H, "fd_theta_step_K": ADJ_FD_H,
            "fd_grad": [float(v) for v in fd],
            "rel_err_vs_central_differences": [float(v) for v in rel_fd],
            "same_masks_fraction": [float(v.mean()) for v in same],
            "fd_grad_same_masks": [float(v) for v in fd_same],
            "grad_same_masks": [float(v) for v in g_same],
            "rel_err_vs_central_differences_same_masks": [float(v) for v in rel_fd_same],
            "oracle_sample": int(len(idx)),
            "oracle_grad_sample": [float(v) for v in go],
            "gpu_grad_sample": [float(v) for v in g_s],
            "rel_err_vs_oracle_adjoint": [float(v) for v in rel_o],
            "replay_max_abs_dx_over_box": float(np.abs(xg - xo).max() / box)}


DIRECTIONAL_STEPS = 2000
DIRECTIONAL_TIMED = 100


def directional_leg(steps=DIRECTIONAL_STEPS, timed=DIRECTIONAL_TIMED):
    """The directional-growth workload at its stated size (2 x 2 x 4 mm, 64
    grains on the cold face, linear field, lambda0 = h = rc = 5 um, dt =
    5e-5 s): `steps` steps untimed (about 2M stored particles), then `timed`
    more steps timed with HIP events on the context's stream (recorded
    sequences, default schedule)."""
    import torch
    from paper_2504_12858_amd import workloads as W
    from paper_2504_12858_amd import binding as B
    w = W.directional(seed=2)
    ctx = B.Context.from_workload(w, cap_particles=1 << 22, cap_stopped=1 << 22,
                                  cap_claim_bricks=1 << 20)
    st0 = ctx.step(w.dt, steps)
    ctx.prepare_step(w.dt)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    st = ctx.step(w.dt, timed)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ctx.close()
    return {"workload": "directional-2x2x4mm-64-grains", "steps_before": steps,
            "active_at_start": st0["n_active"], "stored_at_start": st0["n_active"] + st0["n_stopped"],
            "steps": timed, "ms_per_step": round(ms / timed, 4),
            "updates_per_s": st["advanced"] / (ms * 1e-3),
            "active_after": st["n_active"], "stopped_after": st["n_stopped"]}


BATCH_MEMBERS = 128
BATCH_STEPS = 200


def batch_leg(members=BATCH_MEMBERS, steps=BATCH_STEPS):
    """Batched against sequential plain stepping of the same contexts:
    directional growth (2 x 2 x 4 mm, 64 grains, lambda0 = 5 um, cells of
    10 um), member m with seed 1000 + m and a target of N_m ~ U{50k..1M}
    stored particles (seed 4).  Two identical batches are advanced to the
    snapshot (each member held once it reaches its target, checked every 32
    steps); batch A's shared launches are autotuned from the snapshot (which
    is restored), then batch A takes `steps` batched steps and batch B steps
    its members one after the other with plain ge_step calls.  The states must
    agree bit for bit (order-independent digests).  Last, batch A takes the
    same steps again with every member held: the launch floor of the recorded
    per-phase sequence (launch, dispatch and retire of every block, no
    work)."""
    import numpy as np
    import torch
    from paper_2504_12858_amd import workloads as W
    from paper_2504_12858_amd import binding as B
    targets = W.rng(4).integers(50_000, 1_000_001, size=members)
    ws = [W.directional(seed=1000 + m, h=10e-6) for m in range(members)]
    dt = ws[0].dt

    def params(m):
        c = int(1.5 * targets[m]) + (1 << 18)
        return B.params_from_workload(ws[m], cap_particles=c, cap_stopped=c,
                                      cap_claim_bricks=1 << 17)

    def snapshot():
        b = B.Batch([params(m) for m in range(members)])
        for m, w in zip(b.members, ws):
            m.init_from_workload(w)
        held = np.zeros(members, bool)
        k = 0
        while not held.all() and k < 6000:
            st = b.step(dt, 32)
            k += 32
            for m in range(members):
                if not held[m] and st[m]["n_active"] + st[m]["n_stopped"] >= targets[m]:
                    b.members[m].hold(True)
                    held[m] = True
        for m in b.members:
            m.hold(False)
        return b, k

    t0 = time.perf_counter()
    a, ka = snapshot()
    b, kb = snapshot()
    log(f"[batch] snapshots in {time.perf_counter() - t0:.1f} s ({ka} batched steps)")
    stored = sum(m.counts()["n_active"] + m.counts()["n_stopped"] for m in a.members)
    t0 = time.perf_counter()
    blocks = a.autotune(dt, 2)
    t_tune = time.perf_counter() - t0
    log(f"[batch] autotuned {blocks} in {t_tune:.1f} s")
    for m in b.members:
        m.prepare_step(dt)
    torch.cuda.synchronize()
    REGION.resume()
    t0 = time.perf_counter()
    sa = a.step(dt, steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    REGION.pause()
    t0 = time.perf_counter()
    sb = [m.step(dt, steps) for m in b.members]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    equal = all(x.digest() == y.digest() for x, y in zip(a.members, b.members))
    upd_a = sum(s["advanced"] for s in sa)
    upd_b = sum(s["advanced"] for s in sb)
    # Launch floor: the same recorded sequences and block shares with every
    # member held, so every block of every launch returns at once.
    for m in a.members:
        m.hold(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.step(dt, steps)
    torch.cuda.synchronize()
    t_floor = time.perf_counter() - t0
    a.close()
    b.close()
    return {"workload": f"directional-{members}-members-50k-1M", "members": members,
            "stored_at_snapshot": int(stored), "steps": steps,
            "batched_s": round(t_batch, 4), "plain_sequential_s": round(t_plain, 4),
            "speedup": round(t_plain / t_batch, 3), "blocks": blocks,
            "autotune_s": round(t_tune, 2),
            "launch_floor_s": round(t_floor, 4), "launch_floor_frac": round(t_floor / t_batch, 4),
            "batched_updates_per_s": upd_a / t_batch, "plain_updates_per_s": upd_b / t_plain,
            "bitwise_equal": bool(equal and upd_a == upd_b)}


MUSHY_STEPS = 32


def mushy_leg(ctx, w, steps=MUSHY_STEPS):
    """Mushy-zone deposition at the 20M snapshot on the 256^3 node grid of
    the field: the full count of every reached site when the grid is set,
    then blocks of `steps` steps (recorded sequences) with the deposition
    off, on, on, off (the state grows between blocks: the order cancels the
    trend), each after 16 untimed steps, timed with HIP events; the branch
    phase (where reached sites are deposited) with the deposition on and
    off; the g^m query."""
    import numpy as np
    import torch
    fd = w.field
    n = tuple(fd.n)
    s = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    on_ms, off_ms = [], []
    recount_ms = 0.0
    branch_ms = {}
    for on in (False, True, True, False):
        if on:
            recount_ms = timed(lambda: ctx.set_deposition_grid(n, fd.origin, fd.spacing))
        else:
            ctx.set_deposition_grid(None)
        ctx.step(w.dt, 16, stats=False)
        ctx.prepare_step(w.dt)
        (on_ms if on else off_ms).append(timed(lambda: ctx.step(w.dt, steps, stats=False)) / steps)
        if on not in branch_ms:
            ctx.profile(1)
            ctx.step(w.dt, 4, stats=False)
            ph, k = ctx.profile_read()
            ctx.profile(0)
            branch_ms[on] = ph["branch"] / max(k, 1)
    ctx.set_deposition_grid(n, fd.origin, fd.spacing)
    t = time.perf_counter()
    gm = ctx.mushy_fraction()
    query_ms = 1e3 * (time.perf_counter() - t)
    cnt = ctx.mushy_counts()
    ctx.set_deposition_grid(None)
    on, off = sum(on_ms) / len(on_ms), sum(off_ms) / len(off_ms)
    return {"workload": f"cet-moving-source-20M snapshot, deposition on the {n[0]}x{n[1]}x{n[2]} "
                        "node grid of the field",
            "steps_per_block": steps, "recount_ms": round(recount_ms, 3),
            "step_ms_deposition_on": round(on, 4), "step_ms_deposition_off": round(off, 4),
            "overhead_ms_per_step": round(on - off, 4),
            "branch_ms_deposition_on": round(branch_ms[True], 4),
            "branch_ms_deposition_off": round(branch_ms[False], 4),
            "reached_sites": int(cnt.sum(dtype=np.int64)),
            "cells_mushy_full": int((gm >= 1.0).sum()), "cells_mushy_partial": int(((gm > 0) & (gm < 1)).sum()),
            "fraction_query_to_host_ms": round(query_ms, 2)}


MELT_STEPS = 32


def melt_leg(ctx, w, steps=MELT_STEPS):
    """Melting by walk-back at the 20M snapshot under the moving source (its
    melt pool): after a pre-roll with melting on until three blocks of 16
    steps in a row melt solid sites, blocks of `steps` steps with melting on,
    off, off, on, each after 16 untimed steps, timed with HIP events, and the
    melting counts of the timed blocks."""
    import torch
    s = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        out = fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), out

    # Advance with melting on until the source melts solid sites step after
    # step (the melt pool has to reach grown solid; the first block after
    # melting is turned on only melts what the field had already melted), so
    # that the timed blocks melt.
    ctx.set_melting(True)
    pre, melted_pre, streak = 0, 0, 0
    while pre < 2400 and streak < 3:
        melted_pre = int(ctx.step(w.dt, 16)["melted"])
        pre += 16
        streak = streak + 1 if (melted_pre > 0 and pre > 16) else 0
    on_ms, off_ms, counts = [], [], {}
    # Melting stays on from the pre-roll into the first block (steady melting);
    # on, off, off, on cancels the growth of the state between blocks.
    for on in (True, False, False, True):
        ctx.set_melting(on)
        ctx.step(w.dt, 16, stats=False)
        ctx.prepare_step(w.dt)
        ms, st = timed(lambda: ctx.step(w.dt, steps))
        (on_ms if on else off_ms).append(ms / steps)
        if on:
            for k in ("melted", "removed", "reactivated", "grains_melted"):
                counts[k] = counts.get(k, 0) + int(st[k])
    ctx.set_melting(False)
    on, off = sum(on_ms) / len(on_ms), sum(off_ms) / len(off_ms)
    return {"workload": "cet-moving-source-20M snapshot, melting under the moving source",
            "steps_per_block": steps, "step_ms_melting_on": round(on, 4),
            "step_ms_melting_off": round(off, 4), "overhead_ms_per_step": round(on - off, 4),
            "preroll_steps_until_melting": pre,
            "melted_per_step_last_preroll_block": round(melted_pre / 16, 1),
            "timed_from_step": int(ctx.counts()["step"]) - 4 * (16 + steps),
            "per_step_on": {k: round(v / (2 * steps), 1) for k, v in counts.items()}}


PERIODIC_STEPS = 100


def periodic_leg(schedule, plain_value, steps=PERIODIC_STEPS):
    """Periodic lateral boundaries (Sec. 3.4 imposes periodic conditions on
    the faces normal to x and y) at the bench's scale: the CET workload with
    x and y periodic (periods of 2000 and 1000 cells; the moving-source field
    wraps with the positions), advanced to the same 20M-active snapshot
    target, then `steps` steps timed with HIP events on the context's stream
    (recorded sequences) in the launch schedule of the plain run."""
    import torch
    s = torch.cuda.current_stream()
    w = cet_workload()
    w.periodic = 3
    ctx = make_context(w)
    snap, st0 = advance_to_snapshot(ctx, w, TARGET_ACTIVE)
    ctx.set_schedule(schedule)
    ctx.step(w.dt, 5, stats=False)
    ctx.prepare_step(w.dt)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    st = ctx.step(w.dt, steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    value = st["advanced"] / (ms * 1e-3)
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return {"workload": "cet-moving-source-20M with x and y periodic", "snapshot_step": snap,
            "active_at_snapshot": st0["n_active"], "steps": steps,
            "ms_per_step": round(ms / steps, 4), "updates_per_s": value,
            "vs_walls_updates_per_s": round(value / plain_value, 4),
            "active_after": st["n_active"], "stopped_after": st["n_stopped"]}


SOLUTE_STEPS = 20


def solute_leg(ctx, w, steps=SOLUTE_STEPS):
    """Coupled stepping at the 20M snapshot: a temperature-and-solute field on
    the 256^3 node grid of the box, handed over from device arrays (FP64)
    before a step, as a coupled solver would (the undercooling is taken with
    respect to the liquidus of the local concentration, Sec. 3.4).  A
    stand-in solver (torch, outside the timed spans) gives the node
    temperatures T = T_L(w0) - dT_R(x, t), dT_R being the moving-source
    undercooling of the workload, and a static segregation pattern w around
    w0, so the undercooling is the workload's plus liq_m (w - w0).  Steps
    alternate between a hand-over before the step and the field kept; HIP
    events time the hand-over (node conversion included) and the step."""
    import torch
    from paper_2504_12858_amd import workloads as W
    fd = w.field
    n = tuple(fd.n)
    dev = torch.device("cuda")
    k, j, i = torch.meshgrid(*(torch.arange(m, dtype=torch.float64, device=dev)
                               for m in (n[2], n[1], n[0])), indexing="ij")
    X = fd.origin[0] + i * fd.spacing[0]
    Y = fd.origin[1] + j * fd.spacing[1]
    Z = fd.origin[2] + k * fd.spacing[2]
    del i, j, k
    w0, amp, period = 3.0, 0.3, 1e-4
    wn = (w0 + amp * torch.sin(2 * math.pi * X / period) *
          torch.sin(2 * math.pi * Y / period)).contiguous()
    T_L0 = W.LIQ_T + W.LIQ_M * w0

    def temperature(t):
        L = fd.x_end - fd.x_start
        phase = math.fmod(fd.U * t, 2 * L)
        xs, sg = (fd.x_start + phase, 1.0) if phase < L else (fd.x_start + 2 * L - phase, -1.0)
        xi = sg * (X - xs)
        r = torch.sqrt(xi * xi + (Y - fd.ys) ** 2 + (Z - fd.zs) ** 2).clamp_min(fd.r_min)
        rise = fd.q / (2 * math.pi) / r * torch.exp(-fd.U / (2 * fd.alpha) * (xi + r))
        dT = (fd.dT0 + fd.rate * t + fd.grad[0] * X + fd.grad[1] * Y + fd.grad[2] * Z - rise)
        return (T_L0 - dT.clamp_min(fd.dT_min)).contiguous()

    def field(t):
        return W.Field(W.FIELD_SOLUTE, n=n, origin=tuple(fd.origin), spacing=tuple(fd.spacing),
                       T=temperature(t), w=wn, liq_T=W.LIQ_T, liq_m=W.LIQ_M)

    ctx.set_thermal_field(field(float(ctx.counts()["t"])))
    ctx.step(w.dt, 2, stats=False)
    s = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for it in range(steps):
        coupled = it % 2 == 0
        f = field(float(ctx.counts()["t"])) if coupled else None
        e = ev[it]
        e[0].record(s)
        if coupled:
            ctx.set_thermal_field(f)
        e[1].record(s)
        ctx.step(w.dt, 1, stats=False)
        e[2].record(s)
    torch.cuda.synchronize()
    hand = [ev[i][0].elapsed_time(ev[i][1]) for i in range(0, steps, 2)]
    step_c = [ev[i][1].elapsed_time(ev[i][2]) for i in range(0, steps, 2)]
    step_p = [ev[i][1].elapsed_time(ev[i][2]) for i in range(1, steps, 2)]
    st = ctx.counts()
    mean = lambda v: sum(v) / len(v)  # noqa: E731
    return {"workload": "cet-moving-source-20M snapshot, temperature-and-solute field "
                        f"{n[0]}x{n[1]}x{n[2]} nodes (FP64 T and w on the device)",
            "steps": steps, "n_active": int(st["n_active"]),
            "handover_ms": round(mean(hand), 4),
            "step_after_handover_ms": round(mean(step_c), 4),
            "step_field_kept_ms": round(mean(step_p), 4),
            "coupled_updates_per_s": st["n_active"] / ((mean(hand) + mean(step_c)) * 1e-3)}


def cell_change(ctx, w):
    """Of the particles active before and after one step (neither branched
    nor stopped in it), the fraction whose cell changed: particle queries
    before and after the step, matched by identity (grain, departure site,
    direction)."""
    import numpy as np

    def active():
        p = ctx.particles()
        p = p[p["state"] == 0]
        s = p["site"].astype(np.int64) + (1 << 15)
        key = ((p["grain"].astype(np.int64) << 51) | (s[:, 0] << 35) | (s[:, 1] << 19)
               | (s[:, 2] << 3) | p["dir"].astype(np.int64))
        cell = ((p["cell"][:, 2].astype(np.int64) << 42) | (p["cell"][:, 1].astype(np.int64) << 21)
                | p["cell"][:, 0].astype(np.int64))
        o = np.argsort(key)
        return key[o], cell[o]

    k0, c0 = active()
    ctx.step(w.dt, 1)
    k1, c1 = active()
    both, i0, i1 = np.intersect1d(k0, k1, assume_unique=True, return_indices=True)
    moved = int(np.count_nonzero(c0[i0] != c1[i1]))
    return {"active_before": int(len(k0)), "active_after": int(len(k1)), "kept": int(len(both)),
            "changed_cell": moved, "fraction": round(moved / max(len(both), 1), 4),
            "fraction_of_active": round(moved / max(len(k0), 1), 4)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(ctx, w, budget_s=15.0, max_steps=400, one_thread_s=5.0):
    """The FP64 oracle steps a 0.25 x 0.25 x 1 mm column of the snapshot on
    every host core, then a few more steps of the same column on one thread."""
    import numpy as np
    from oracle import Oracle
    from oracle import oracle as orc
    lo = np.array([1.875e-3, 0.875e-3, 0.0])
    hi = np.array([2.125e-3, 1.125e-3, 1.0e-3])
    margin = 4 * w.lambda0
    parts = ctx.particles(window=(lo, hi))
    claims = ctx.claims(window=(lo - margin, hi + margin))
    centre, quat = grain_quaternions(ctx, w)
    o = Oracle.from_workload(w, init=False)
    o.nucleate(w.site_xyz, w.site_dTn, w.site_quat)
    st = ctx.counts()
    o.load_state(centre, quat,
                 dict(grain=parts["grain"], site=parts["site"], dir=parts["dir"],
                      s=parts["s"].astype(np.float64), state=parts["state"]),
                 dict(grain=claims["grain"], site=claims["site"], flags=claims["flags"]),
                 ctx.site_states(), st["t"], st["step"])
    n_act = int((parts["state"] == 0).sum())
    log(f"[cpu] window {n_act} active, {len(parts) - n_act} stopped, {len(claims)} claims")
    updates = 0
    t0 = time.perf_counter()
    k = 0
    while k < max_steps:
        o.step(w.dt, 1)
        updates += o.last_stats()["advanced"]
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    cores = orc.threads()
    log(f"[cpu] {k} oracle steps in {dt:.2f} s on {cores} threads")
    # The same column, continued, on one thread.
    orc.set_threads(1)
    u1, k1 = 0, 0
    t1 = time.perf_counter()
    while k1 < max_steps:
        o.step(w.dt, 1)
        u1 += o.last_stats()["advanced"]
        k1 += 1
        if time.perf_counter() - t1 > one_thread_s:
            break
    d1 = time.perf_counter() - t1
    orc.set_threads(cores)
    log(f"[cpu] {k1} oracle steps in {d1:.2f} s on one thread")
    return {"value": updates / dt, "unit": "particle-updates/s", "cores": cores,
            "kind": "oracle", "value_one_thread": u1 / d1, "steps_one_thread": k1,
            "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": f"FP64 oracle, {k} steps of the 0.25x0.25x1 mm column "
                      f"x in [1.875,2.125] mm, y in [0.875,1.125] mm of the same snapshot "
                      f"({n_act} active particles, {len(parts) - n_act} stopped, "
                      f"{len(claims)} claimed sites)"}


def main():
    global RESORT_EVERY
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--target", type=int, default=TARGET_ACTIVE)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-solute", action="store_true")
    ap.add_argument("--no-mushy", action="store_true")
    ap.add_argument("--no-melt", action="store_true")
    ap.add_argument("--no-periodic", action="store_true")
    ap.add_argument("--no-directional", action="store_true")
    ap.add_argument("--cell-change", action="store_true",
                    help="after the timed steps, measure the fraction of the kept particles "
                         "that change cell in one step (particle queries; slow)")
    ap.add_argument("--resort-every", type=int, default=RESORT_EVERY, metavar="STEPS",
                    help="steps between re-sorts of the stopped store of the 20M contexts")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="MB")
    ap.add_argument("--autotune", type=int, default=6, metavar="STEPS",
                    help="autotune the launch schedule at the snapshot with STEPS steps per "
                         "trial before the warm-up; every trial starts from the snapshot, "
                         "which is restored (0: the default schedule)")
    ap.add_argument("--schedule", default="", metavar="KERNEL=BLOCKS,...",
                    help="blocks per launch of the named tunable kernels (others keep the "
                         "default from the occupancy of the kernel)")
    args = ap.parse_args()
    RESORT_EVERY = args.resort_every
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "slab decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    w = cet_workload()
    t_build = time.perf_counter()
    ctx = make_context(w)
    snap_steps, st = advance_to_snapshot(ctx, w, args.target)
    log(f"[snapshot] reached in {time.perf_counter() - t_build:.1f} s")
    if args.schedule:
        ctx.set_schedule({k: int(v) for k, v in
                          (item.split("=") for item in args.schedule.split(","))})
    if args.autotune:
        t_tune = time.perf_counter()
        best = ctx.autotune(w.dt, args.autotune)
        log(f"[autotune] {best} in {time.perf_counter() - t_tune:.1f} s")
    # The warm-up steps run with an event between every two phases (plain
    # launches): the phase table, and the phase that takes longest.
    phases, n_prof = {}, 0
    if args.warmup:
        ctx.profile(1)
        ctx.step(w.dt, args.warmup)
        phases, n_prof = ctx.profile_read()
        ctx.profile(0)
    dom = (max((k for k in phases if k in PHASE_BYTES), key=lambda k: phases[k])
           if n_prof else "contain")
    # The timed steps carry two events per step around that phase alone (an
    # event between every two phases costs the step about 1 %).
    ctx.profile_phase(dom)
    torch.cuda.synchronize()
    REGION.resume()
    t0 = time.perf_counter()
    stats = ctx.step(w.dt, args.steps)           # synchronises at the end
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    REGION.pause()
    dom_ms, n_dom = ctx.profile_read()
    ctx.profile(0)
    if n_dom != args.steps or not dom_ms[dom] > 0:
        raise RuntimeError(f"phase timer: {n_dom} steps, {dom_ms[dom]} ms for {dom}")
    # The phase table: one re-sort interval after the timed steps, an event
    # between every two phases.
    if args.steps:
        ctx.profile(1)
        ctx.step(w.dt, RESORT_EVERY)
        phases, n_prof = ctx.profile_read()
        ctx.profile(0)
    elapsed = t1 - t0
    value = stats["advanced"] / elapsed
    ms_step = 1e3 * elapsed / args.steps
    log(f"[timed] {args.steps} steps {elapsed:.3f} s, {stats['advanced']} updates, "
        f"active {stats['n_active']} stopped {stats['n_stopped']} spawners "
        f"{stats['spawners']} children {stats['children']} contained {stats['contained']} "
        f"pair tests {stats['pair_tests']} dirty {stats['dirty_tests']}")
    for k, v in sorted(phases.items(), key=lambda kv: -kv[1]):
        log(f"[phase] {k:9s} {v / max(n_prof, 1):8.3f} ms/step (after the timed steps)")
    avg_ms = dom_ms[dom] / n_dom
    log(f"[timed phase] {dom} {avg_ms:.4f} ms/step over the timed steps")
    units = stats["advanced"] / args.steps
    if dom == "resample":
        units = float(w.field.n[0] * w.field.n[1] * w.field.n[2])
    elif dom == "branch":
        units = stats["spawners"] / args.steps
    achieved = PHASE_BYTES[dom] * units / (avg_ms * 1e-3) / 1e9
    kname = "k_" + dom
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kname),
                "kernel": kname, "bytes_per_unit": PHASE_BYTES[dom],
                "units_per_launch": round(units), "avg_launch_ms": round(avg_ms, 4)}
    step_gbs = value * STEP_BYTES_PER_UPDATE / 1e9
    step_roofline = {"bound": "hbm", "bytes_per_update": STEP_BYTES_PER_UPDATE,
                     "achieved": round(step_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4)}
    step_bytes = measured_step_traffic()
    step_traffic = None
    if step_bytes is not None:
        tb = step_bytes / (ms_step * 1e-3) / 1e9
        step_traffic = {"bytes_per_step": step_bytes, "achieved": round(tb, 2),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(tb / HBM_PEAK_GBS, 4),
                        "vs_algorithmic": round(step_bytes / (STEP_BYTES_PER_UPDATE * stats["advanced"]
                                                              / args.steps), 3)}
    out = {
        "metric": METRIC, "value": value, "unit": "particle-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cet-moving-source-20M", "box_mm": [4, 2, 1],
                   "lambda0_um": 1.0, "h_um": 2.0, "dT0_K": CET_KNOBS["dT0"], "grid": 256,
                   "sites": 1600,
                   "dt_s": w.dt, "snapshot_step": snap_steps,
                   "active_at_snapshot": st["n_active"], "stopped_at_snapshot": st["n_stopped"],
                   "active_after": stats["n_active"], "stopped_after": stats["n_stopped"],
                   "timed_from_step": int(stats["step"]) - args.steps,
                   "schedule": ctx.schedule(), "autotuned": bool(args.autotune),
                   "schedule_set": args.schedule or None},
        "phases_ms_per_step": {k: round(v / max(n_prof, 1), 4) for k, v in phases.items()},
        "phases_window": f"{n_prof} steps after the timed ones, an event between every two phases",
        "roofline": roofline,
        "step_roofline": step_roofline,
        "step_traffic": step_traffic,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ctx, w)
    if args.cell_change:
        out["cell_change"] = cell_change(ctx, w)
        log(f"[cell change] {out['cell_change']}")
    if not args.no_melt:
        log(f"[melt] start: {ctx.counts()}")
        out["melting"] = melt_leg(ctx, w)
        log(f"[melt] {out['melting']}")
    if not args.no_mushy:
        log(f"[mushy] start: {ctx.counts()}")
        out["mushy"] = mushy_leg(ctx, w)
        log(f"[mushy] {out['mushy']}")
    if not args.no_solute:
        log(f"[solute] start: {ctx.counts()}")
        out["solute"] = solute_leg(ctx, w)
        log(f"[solute] {out['solute']}")
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    if not args.no_periodic:
        out["periodic"] = periodic_leg(out["config"]["schedule"], value)
        log(f"[periodic] {out['periodic']}")
    if not args.no_directional:
        out["directional"] = directional_leg()
        log(f"[directional] {out['directional']}")
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg()
        log(f"[adjoint] {out['adjoint']}")
    if not args.no_batch:
        out["batched"] = batch_leg()
        log(f"[batch] {out['batched']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
