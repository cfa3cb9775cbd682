"""Helpers shared by the GPU parity tests: build contexts, export states in a
canonical order, move a state between the HIP path and the oracle."""
import numpy as np

from paper_2504_12858_amd import binding as B


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X; run them with -m gpu on a GPU box"
    return torch


def ident(grain, site, d):
    """Canonical identity of a particle: (grain, departure site, direction)."""
    site = np.asarray(site).reshape(-1, 3).astype(np.int64)
    return ((np.asarray(grain, np.int64) << 40) ^ ((site[:, 0] + 32768) << 24) ^
            ((site[:, 1] + 32768) << 8) ^ (site[:, 2] + 32768)) * 8 + np.asarray(d, np.int64)


def gpu_parts(ctx):
    p = ctx.particles()
    key = ident(p["grain"], p["site"], p["dir"])
    order = np.argsort(key, kind="stable")
    return p[order], key[order]


def orc_parts(o, include_retired=False):
    p = o.particles()
    keep = np.ones(len(p["grain"]), bool) if include_retired else p["state"] != 2
    q = {k: v[keep] for k, v in p.items()}
    key = ident(q["grain"], q["site"], q["dir"])
    order = np.argsort(key, kind="stable")
    return {k: v[order] for k, v in q.items()}, key[order]


def gpu_claims(ctx):
    c = ctx.claims()
    key = ident(c["grain"], c["site"], np.zeros(len(c), np.int64))
    order = np.argsort(key)
    return c[order], key[order]


def orc_claims(o):
    c = o.claims()
    key = ident(c["grain"], c["site"], np.zeros(len(c["grain"]), np.int64))
    order = np.argsort(key)
    return {k: v[order] for k, v in c.items()}, key[order]


def gpu_state_for_oracle(ctx, grain_centre, grain_quat):
    """Exports the GPU state in the oracle's load_state format (FP32 travel
    values are exact in FP64)."""
    p = ctx.particles()
    c = ctx.claims()
    parts = dict(grain=p["grain"].astype(np.int32), site=p["site"].astype(np.int32),
                 dir=p["dir"].astype(np.int32), s=p["s"].astype(np.float64),
                 state=p["state"].astype(np.int32))
    claims = dict(grain=c["grain"].astype(np.int32), site=c["site"].astype(np.int32),
                  flags=c["flags"].astype(np.uint8))
    return parts, claims


def context_for(w, **caps):
    caps.setdefault("cap_particles", 1 << 20)
    caps.setdefault("cap_stopped", 1 << 20)
    caps.setdefault("cap_claim_bricks", 1 << 16)
    return B.Context.from_workload(w, **caps)
