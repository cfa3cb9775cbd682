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
    """A saved state of a context (ge_save_state blob) plus the recorded-run
    settings."""
    ctx: "B.Context"
    blob: np.ndarray
    b: tuple
    dt: float
    n_steps: int
    ckpt_every: int = 50

    @classmethod
    def capture(cls, ctx, b, dt, n_steps, ckpt_every=50):
        """Saves the context's current state (grains, particles, claims, sites, time)."""
        return cls(ctx, ctx.save_state(), tuple(b), float(dt), int(n_steps), int(ckpt_every))

    def restore(self):
        self.ctx.restore_state(self.blob)

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
