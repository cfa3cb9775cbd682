"""Differentiation of the envelope step with respect to the kinetic law and
the undercooling offset, behind torch.autograd.

EnvelopeRun.apply(params, run) returns the final positions x_N (float32
[n, 3] on the device) of the particles tracked over a recorded run of the
hand-written HIP step; params = (a0, a1, theta) as a float64 tensor.  Its
backward calls the hand-written adjoint kernel (ge_adjoint_backward): the
deactivation masks are those of the forward run, the travel is checkpointed
every `ckpt_every` steps and recomputed segment by segment.

Every call of the forward restarts from the same saved state (AdjointRun),
so the tracked particles keep their order from call to call.
"""
from dataclasses import dataclass

import numpy as np

from . import binding as B


@dataclass
class AdjointRun:
    """A saved state of a context plus the recorded-run settings."""
    ctx: "B.Context"
    grain_centre: np.ndarray
    grain_quat: np.ndarray
    parts: dict
    claims: dict
    site_state: np.ndarray
    t0: float
    step0: int
    b: tuple
    dt: float
    n_steps: int
    ckpt_every: int = 50

    @classmethod
    def capture(cls, ctx, grain_centre, grain_quat, b, dt, n_steps, ckpt_every=50):
        """Saves the context's current state (particles, claims, sites, time)."""
        p = ctx.particles()
        c = ctx.claims()
        st = ctx.counts()
        parts = dict(grain=p["grain"].astype(np.int32), site=p["site"].astype(np.int32),
                     dir=p["dir"].astype(np.int32), s=p["s"].astype(np.float64),
                     state=p["state"].astype(np.int32))
        claims = dict(grain=c["grain"].astype(np.int32), site=c["site"].astype(np.int32),
                      flags=c["flags"].astype(np.uint8))
        return cls(ctx, np.asarray(grain_centre, np.float64), np.asarray(grain_quat, np.float64),
                   parts, claims, ctx.site_states(), float(st["t"]), int(st["step"]), tuple(b),
                   float(dt), int(n_steps), int(ckpt_every))

    def restore(self):
        self.ctx.load_state(self.grain_centre, self.grain_quat, self.parts, self.claims,
                            self.site_state, self.t0, self.step0)

    def forward(self, a0, a1, theta):
        """Recorded run from the saved state; returns x_N (torch, device)."""
        self.restore()
        self.ctx.set_model((a0, a1), self.b, theta, 0)
        self.ctx.adjoint_forward(self.dt, self.n_steps, self.ckpt_every)
        return self.ctx.adjoint_positions()


def _function():
    import torch

    class EnvelopeRun(torch.autograd.Function):
        @staticmethod
        def forward(fctx, params, run):
            a0, a1, th = (float(v) for v in params.detach().cpu().tolist())
            x = run.forward(a0, a1, th)
            fctx.run = run
            fctx.device = params.device
            return x

        @staticmethod
        def backward(fctx, gx):
            g = fctx.run.ctx.adjoint_backward(gx.contiguous())
            return torch.tensor(g, dtype=torch.float64, device=fctx.device), None

    return EnvelopeRun


_ENVELOPE_RUN = None


def envelope_run(params, run):
    """x_N(params) for params = (a0, a1, theta), differentiable."""
    global _ENVELOPE_RUN
    if _ENVELOPE_RUN is None:
        _ENVELOPE_RUN = _function()
    return _ENVELOPE_RUN.apply(params, run)
