"""Pins of the oracle's frozen-mask adjoint: a closed form in a uniform melt
and central finite differences of frozen-mask replays in a gradient."""
import numpy as np

from oracle import Oracle
from paper_2504_12858_amd import workloads as W


def _parts_of(o):
    p = o.particles()
    return dict(grain=p["grain"], site=p["site"], dir=p["dir"], s=p["s"], state=p["state"]), p


def test_uniform_melt_closed_form():
    """dT uniform: s_N = s_0 + n_act dt v(dT - theta), so
    d<c, x_N>/da_j = <c, u> n_act dt (dT - theta)^b_j and
    d<c, x_N>/dtheta = -<c, u> n_act dt v'(dT - theta)."""
    dT, dt, N = 5.0, 1e-4, 40
    o = Oracle((0, 0, 0), (1e-3,) * 3, 5e-6, 5e-6, 5e-6, W.KIN_A, W.KIN_B, branching=0)
    o.set_field(W.Field(W.FIELD_UNIFORM, dT=dT))
    q = W.shoemake_quaternions(W.rng(3), 2)
    o.init_grains(np.array([[3e-4] * 3, [7e-4] * 3]), q, np.zeros(2, np.int32))
    parts, p0 = _parts_of(o)
    t0 = o.time
    nact = o.adjoint_record(dt, N)
    assert (nact == N).all()
    c = W.rng(9).normal(size=(len(nact), 3))
    g = o.adjoint_grad(parts, nact, t0, dt, N, c)
    _, R = o.grains()
    u = np.array([(1 if d % 2 == 0 else -1) * R[gi][:, d // 2] for gi, d in zip(parts["grain"], parts["dir"])])
    cu = (c * u).sum(1)
    a, b = W.KIN_A, W.KIN_B
    vp = a[0] * b[0] * dT ** (b[0] - 1) + a[1] * b[1] * dT ** (b[1] - 1)
    want = np.array([(cu * N * dt * dT ** b[0]).sum(), (cu * N * dt * dT ** b[1]).sum(),
                     -(cu * N * dt * vp).sum()])
    np.testing.assert_allclose(g, want, rtol=1e-12)


def test_gradient_matches_central_differences_with_frozen_masks():
    """Two grains in a linear field grow into each other (some particles stop);
    the adjoint gradient of L = sum |x_N - xhat|^2 equals central differences
    of frozen-mask replays."""
    lam, dt, N = 5e-6, 1e-3, 60
    o = Oracle((0, 0, 0), (1e-3,) * 3, lam, lam, lam, W.KIN_A, W.KIN_B, branching=0)
    fld = W.Field(W.FIELD_LINEAR, dT0=7.0, grad=(-2e3, 1e3, -4e3), rate=3.0)
    o.set_field(fld)
    q = W.shoemake_quaternions(W.rng(5), 3)
    c = np.array([[5e-4, 5e-4, 5e-4], [5.2e-4, 5.05e-4, 4.95e-4], [4.9e-4, 5.15e-4, 5.1e-4]])
    o.init_grains(c, q, np.array([2, 2, 1], np.int32))
    parts, _ = _parts_of(o)
    t0 = o.time
    nact = o.adjoint_record(dt, N)
    assert (nact < N).any() and (nact == N).any()      # masks matter
    x_fwd = o.particles()["x"][: len(nact)]
    a0 = np.array(W.KIN_A)
    x0 = o.adjoint_replay(a0, 0.0, parts, nact, t0, dt, N)
    np.testing.assert_allclose(x0, x_fwd, rtol=0, atol=1e-15)
    xhat = x0 + W.rng(2).normal(scale=1e-6, size=x0.shape)

    def loss(a, th):
        x = o.adjoint_replay(a, th, parts, nact, t0, dt, N)
        return ((x - xhat) ** 2).sum()

    g = o.adjoint_grad(parts, nact, t0, dt, N, 2 * (x0 - xhat))
    fd = []
    for j in range(2):
        h = 1e-4 * a0[j]
        ap, am = a0.copy(), a0.copy()
        ap[j] += h
        am[j] -= h
        fd.append((loss(ap, 0.0) - loss(am, 0.0)) / (2 * h))
    h = 1e-4
    fd.append((loss(a0, h) - loss(a0, -h)) / (2 * h))
    np.testing.assert_allclose(g, fd, rtol=1e-5)
