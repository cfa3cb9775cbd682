"""The hand-written adjoint of the HIP step: a closed form in a uniform melt,
the FP64 oracle's frozen-mask gradient and replay on the GPU's own masks,
the torch.autograd wrapper, and the error paths."""
import ctypes

import numpy as np
import pytest

from oracle import Oracle
from paper_2504_12858_amd import binding as B
from paper_2504_12858_amd import workloads as W
from tests.gpu_helpers import ident, require_gpu

pytestmark = pytest.mark.gpu

LAM = 5e-6
BOX = (0.0, 0.0, 0.0), (1e-3, 1e-3, 1e-3)


def _ctx(field, centre, quat, shells, branching=0):
    p = B.make_params(BOX[0], BOX[1], LAM, LAM, LAM, W.KIN_A, W.KIN_B, branching=branching,
                      cap_particles=1 << 16, cap_stopped=1 << 16, cap_claim_bricks=1 << 12)
    ctx = B.Context(p)
    ctx.set_thermal_field(field)
    ctx.init_grains(centre, quat, shells)
    return ctx


def _oracle(field, centre, quat, shells):
    o = Oracle(BOX[0], BOX[1], LAM, LAM, LAM, W.KIN_A, W.KIN_B, branching=0)
    o.set_field(field)
    o.init_grains(centre, quat, shells)
    return o


def _tracked_parts(tr):
    return dict(grain=tr["grain"].astype(np.int32), site=tr["site"].astype(np.int32),
                dir=tr["dir"].astype(np.int32), s=tr["s0"].astype(np.float64))


def _directions(quat, tr):
    out = []
    for g, d in zip(tr["grain"], tr["dir"]):
        w, x, y, z = quat[g]
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        out.append((1 if d % 2 == 0 else -1) * R[:, d // 2])
    return np.array(out)


def test_uniform_melt_closed_form_on_gpu():
    """Uniform dT: x_N = x_0 + N dt v(dT - theta) u, so the gradient of
    L = sum <c_i, x_N,i> is sum <c_i, u_i> N dt (dT^b0, dT^b1, -v'(dT))."""
    require_gpu()
    dT, dt, N = 5.0, 1e-4, 40
    q = W.shoemake_quaternions(W.rng(3), 2)
    ctx = _ctx(W.Field(W.FIELD_UNIFORM, dT=dT), np.array([[3e-4] * 3, [7e-4] * 3]), q,
               np.array([3, 2], np.int32))
    n = ctx.adjoint_forward(dt, N, ckpt_every=7)
    tr = ctx.adjoint_tracked()
    assert n == len(tr) and (tr["nact"] == N).all()
    c = W.rng(9).normal(size=(n, 3)).astype(np.float32)
    g = np.array(ctx.adjoint_backward(c))
    u = _directions(q, tr)
    cu = (c.astype(np.float64) * u).sum(1)
    a, b = W.KIN_A, W.KIN_B
    vp = a[0] * b[0] * dT ** (b[0] - 1) + a[1] * b[1] * dT ** (b[1] - 1)
    want = np.array([(cu * N * dt * dT ** b[0]).sum(), (cu * N * dt * dT ** b[1]).sum(),
                     -(cu * N * dt * vp).sum()])
    np.testing.assert_allclose(g, want, rtol=1e-5)
    ctx.close()


CASE = dict(
    field=W.Field(W.FIELD_LINEAR, dT0=7.0, grad=(-2e3, 1e3, -4e3), rate=3.0),
    centre=np.array([[5e-4, 5e-4, 5e-4], [5.2e-4, 5.05e-4, 4.95e-4], [4.9e-4, 5.15e-4, 5.1e-4]]),
    shells=np.array([2, 2, 1], np.int32), dt=1e-3, N=60)


@pytest.mark.parametrize("ckpt_every", [50, 7, 1, 60])
def test_gradient_matches_oracle_on_gpu_masks(ckpt_every):
    """Three grains grow into each other in a linear field (particles stop
    on the way).  On the GPU's own masks: final positions match the
    oracle's FP64 replay and the gradient matches the oracle's FP64 adjoint."""
    require_gpu()
    q = W.shoemake_quaternions(W.rng(5), 3)
    f, dt, N = CASE["field"], CASE["dt"], CASE["N"]
    ctx = _ctx(f, CASE["centre"], q, CASE["shells"])
    n = ctx.adjoint_forward(dt, N, ckpt_every=ckpt_every)
    tr = ctx.adjoint_tracked()
    assert (tr["nact"] < N).any() and (tr["nact"] == N).any()
    x = ctx.adjoint_positions().cpu().numpy().astype(np.float64)
    # The GPU masks agree with the oracle's own masks (matched by identity).
    o = _oracle(f, CASE["centre"], q, CASE["shells"])
    op = o.particles()
    onact = o.adjoint_record(dt, N)
    okey = ident(op["grain"], op["site"], op["dir"])[: len(onact)]
    gkey = ident(tr["grain"], tr["site"], tr["dir"])
    m = dict(zip(okey.tolist(), onact.tolist()))
    same = np.array([m.get(k) == v for k, v in zip(gkey.tolist(), tr["nact"].tolist())])
    assert same.mean() >= 0.99, same.mean()
    parts = _tracked_parts(tr)
    xo = o.adjoint_replay(np.array(W.KIN_A), 0.0, parts, tr["nact"], 0.0, dt, N)
    np.testing.assert_allclose(x, xo, rtol=0, atol=1e-5 * 1e-3)
    xhat = xo + W.rng(2).normal(scale=1e-6, size=xo.shape)
    dLdx = 2.0 * (x - xhat)
    g = np.array(ctx.adjoint_backward(dLdx.astype(np.float32)))
    go = o.adjoint_grad(parts, tr["nact"], 0.0, dt, N, dLdx.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(g, go, rtol=2e-4)
    # Bitwise reproducible.
    assert np.array_equal(g, np.array(ctx.adjoint_backward(dLdx.astype(np.float32))))
    ctx.close()


def test_gradient_through_a_periodic_face():
    """x periodic, a node field periodic in x (dT = 5 + 2 sin(2 pi x / L)),
    two grains whose particles cross the face x = L during the run and meet
    across it: on the GPU's masks the replay and the gradient match the
    oracle's, which take the field at the wrapped positions."""
    require_gpu()
    L = BOX[1][0]
    n = (41, 5, 5)
    x = np.arange(n[0]) * (L / 40)
    data = np.broadcast_to((5.0 + 2.0 * np.sin(2 * np.pi * x / L)).astype(np.float32),
                           (n[2], n[1], n[0]))
    f = W.Field(W.FIELD_GRID, n=n, origin=(0.0, 0.0, 0.0), spacing=(L / 40, 0.25e-3, 0.25e-3),
                data=np.ascontiguousarray(data))
    centre = np.array([[L - 2 * LAM, 5e-4, 5e-4], [3 * LAM, 5.01e-4, 4.99e-4]])
    q = W.shoemake_quaternions(W.rng(9), 2)
    shells = np.array([3, 2], np.int32)
    dt, N = 1e-3, 60
    p = B.make_params(BOX[0], BOX[1], LAM, LAM, LAM, W.KIN_A, W.KIN_B, branching=0, periodic=1,
                      cap_particles=1 << 16, cap_stopped=1 << 16, cap_claim_bricks=1 << 12,
                      field_n=n)
    ctx = B.Context(p)
    ctx.set_thermal_field(f)
    ctx.init_grains(centre, q, shells)
    ctx.adjoint_forward(dt, N, ckpt_every=7)
    tr = ctx.adjoint_tracked()
    assert (tr["nact"] < N).any() and (tr["nact"] == N).any()
    xg = ctx.adjoint_positions().cpu().numpy().astype(np.float64)
    assert ((xg[:, 0] >= L) | (xg[:, 0] < 0)).any()   # some crossed the face
    o = Oracle(BOX[0], BOX[1], LAM, LAM, LAM, W.KIN_A, W.KIN_B, branching=0, periodic=1)
    o.set_field(f)
    o.init_grains(centre, q, shells)
    op = o.particles()
    onact = o.adjoint_record(dt, N)
    okey = ident(op["grain"], op["site"], op["dir"])[: len(onact)]
    m = dict(zip(okey.tolist(), onact.tolist()))
    same = np.array([m.get(k) == v for k, v in zip(ident(tr["grain"], tr["site"], tr["dir"]).tolist(),
                                                   tr["nact"].tolist())])
    assert same.mean() >= 0.99, same.mean()
    parts = _tracked_parts(tr)
    xo = o.adjoint_replay(np.array(W.KIN_A), 0.0, parts, tr["nact"], 0.0, dt, N)
    np.testing.assert_allclose(xg, xo, rtol=0, atol=1e-5 * 1e-3)
    dLdx = 2.0 * (xg - (xo + W.rng(4).normal(scale=1e-6, size=xo.shape)))
    g = np.array(ctx.adjoint_backward(dLdx.astype(np.float32)))
    go = o.adjoint_grad(parts, tr["nact"], 0.0, dt, N, dLdx.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(g, go, rtol=2e-4)
    ctx.close()


def test_envelope_run_autograd():
    """torch.autograd through EnvelopeRun: loss = sum |x_N - xhat|^2; the
    parameter gradient equals the adjoint call on dL/dx = 2 (x_N - xhat)
    and the oracle's FP64 gradient."""
    torch = require_gpu()
    from paper_2504_12858_amd.adjoint import AdjointRun, envelope_run
    q = W.shoemake_quaternions(W.rng(5), 3)
    f, dt, N = CASE["field"], CASE["dt"], CASE["N"]
    ctx = _ctx(f, CASE["centre"], q, CASE["shells"])
    run = AdjointRun.capture(ctx, W.KIN_B, dt, N, ckpt_every=50)
    # Targets: a run with a +5 % and theta = +2 K (its own masks).
    with torch.no_grad():
        xhat = envelope_run(torch.tensor([W.KIN_A[0] * 1.05, W.KIN_A[1] * 1.05, 2.0],
                                         dtype=torch.float64, device="cuda"), run).clone()
    params = torch.tensor([W.KIN_A[0], W.KIN_A[1], 0.0], dtype=torch.float64, device="cuda",
                          requires_grad=True)
    x = envelope_run(params, run)
    loss = ((x.double() - xhat.double()) ** 2).sum()
    loss.backward()
    g = params.grad.cpu().numpy()
    dLdx = (2.0 * (x.detach().double() - xhat.double())).float()
    direct = np.array(ctx.adjoint_backward(dLdx))
    assert np.array_equal(g, direct)
    tr = ctx.adjoint_tracked()
    o = _oracle(f, CASE["centre"], q, CASE["shells"])
    go = o.adjoint_grad(_tracked_parts(tr), tr["nact"], 0.0, dt, N,
                        dLdx.cpu().numpy().astype(np.float64))
    np.testing.assert_allclose(g, go, rtol=2e-4)
    assert np.all(np.isfinite(g)) and np.all(g != 0)
    ctx.close()


def test_adjoint_error_paths():
    require_gpu()
    q = W.shoemake_quaternions(W.rng(5), 3)
    f, dt, N = CASE["field"], CASE["dt"], CASE["N"]
    ctx = _ctx(f, CASE["centre"], q, CASE["shells"], branching=1)
    with pytest.raises(B.GrainEnvError):        # branching on
        ctx.adjoint_forward(dt, N)
    ctx.close()
    ctx = _ctx(f, CASE["centre"], q, CASE["shells"])
    g = (ctypes.c_double * 3)()
    dummy = np.zeros(3, np.float32)
    assert ctx.lib.ge_adjoint_backward(ctx.ctx, dummy.ctypes.data_as(ctypes.c_void_p), 0, g) == -6
    with pytest.raises(B.GrainEnvError):        # branching back on
        ctx.set_model(W.KIN_A, W.KIN_B, 0.0, 1)
        ctx.adjoint_forward(dt, N)
    ctx.set_model(W.KIN_A, W.KIN_B, 0.0, 0)
    n = ctx.adjoint_forward(dt, N, ckpt_every=10)
    dLdx = np.ones((n, 3), np.float32)
    ctx.adjoint_backward(dLdx)
    ctx.set_model((W.KIN_A[0] * 2, W.KIN_A[1]), W.KIN_B, 0.0, 0)
    with pytest.raises(B.GrainEnvError):        # model changed since the recorded run
        ctx.adjoint_backward(dLdx)
    ctx.close()
