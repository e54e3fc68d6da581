"""Pins of the oracle's adjoint and velocity synthesis (no GPU).

The adjoint has no printed form in the paper; its plain definition is the transpose of the
step's Jacobian. It is pinned against (a) reverse-mode autodiff of an independent torch
statement of the flux form and (b) central finite differences of the oracle's own forward.
The velocity synthesis is pinned against closed forms of single modes, the exact discrete
RMS of a random field, zero discrete divergence and a dot-product test of its transpose.
"""
import numpy as np
import pytest
import torch

import oracle
import pf_fixtures as fx


def torch_rhs(phi, U, V, W, dx, eps, gamma, delta, s):
    """Eq. 1 flux form in torch FP64 (value at c + d e_a is roll(., -d) along that axis)."""
    dims = {0: 2, 1: 1, 2: 0}  # x -> last array axis

    def sh(a, d, ax):
        return torch.roll(a, shifts=-d, dims=dims[ax])

    g = [(sh(phi, 1, a) - sh(phi, -1, a)) / (2 * dx) for a in range(3)]
    mag = torch.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2 + delta ** 2)
    w = phi * (1 - phi)
    vel = (U, V, W)
    f = torch.zeros_like(phi)
    for a in range(3):
        q = w * g[a] / mag
        F = (-s * vel[a] * 0.5 * (sh(phi, -1, a) + phi) + gamma * eps * (phi - sh(phi, -1, a)) / dx
             - gamma * 0.5 * (sh(q, -1, a) + q))
        f = f + (sh(F, 1, a) - F) / dx
    return f


def setup(seed, shape=(6, 7, 8), delta=0.3):
    rng = np.random.default_rng(seed)
    dx = 1.0 / shape[2]
    phi = fx.drops_ic(shape, dx, [(0.5, 0.5, 0.5)], [0.3], dx) * 0.8 + 0.2 * rng.uniform(size=shape)
    U, V, W = fx.random_edge_faces(rng, shape, dx)
    kw = dict(dx=dx, eps=dx, gamma=1.3, delta=delta / dx)
    return rng, phi, (U, V, W), kw


def test_torch_statement_matches_oracle_forward():
    rng, phi, vel, kw = setup(0)
    f = oracle.rhs(phi, *vel, s=0.7, **kw)
    t = torch_rhs(*(torch.tensor(a) for a in (phi, *vel)), kw["dx"], kw["eps"], kw["gamma"],
                  kw["delta"], 0.7)
    np.testing.assert_allclose(t.numpy(), f, rtol=0, atol=1e-11 * np.abs(f).max())


@pytest.mark.parametrize("delta", [0.0, 0.3])
def test_rhs_vjp_matches_autodiff(delta):
    rng, phi, vel, kw = setup(1, delta=delta)
    lam = rng.standard_normal(phi.shape)
    pb, ub, vb, wb = oracle.rhs_vjp(phi, *vel, lam, s=0.6, **kw)
    ts = [torch.tensor(a, requires_grad=True) for a in (phi, *vel)]
    f = torch_rhs(*ts, kw["dx"], kw["eps"], kw["gamma"], kw["delta"], 0.6)
    f.backward(torch.tensor(lam))
    for mine, t in zip((pb, ub, vb, wb), ts):
        ref = t.grad.numpy()
        np.testing.assert_allclose(mine, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def _fd_check(fun, x, v, lam, h):
    return np.sum(lam * (fun(x + h * v) - fun(x - h * v))) / (2 * h)


@pytest.mark.parametrize("scheme", [1, 2, 3, 4])
def test_adjoint_step_matches_finite_differences(scheme):
    """<lam, (step(phi + h v) - step(phi - h v)) / 2h> == <adjoint(lam), v>, and likewise for
    each face-velocity array, over 16 random directions (FP64)."""
    rng, phi, vel, kw = setup(2)
    U, V, W = vel
    step_kw = dict(dt=0.05 * kw["dx"], scheme=scheme, vel_mode=1, vel_T=0.9, t0=0.2, **kw)
    adj_kw = dict(dt=step_kw["dt"], scheme=scheme, vel_mode=1, vel_T=0.9, t=0.2, **kw)
    lam = rng.standard_normal(phi.shape)
    lam_n, ub, vb, wb = oracle.adjoint_step(phi, U, V, W, lam, **adj_kw)
    for d in range(16):
        v = rng.standard_normal(phi.shape)
        fd = _fd_check(lambda p: oracle.step(p, U, V, W, **step_kw), phi, v, lam, 1e-6)
        assert np.sum(lam_n * v) == pytest.approx(fd, rel=2e-7, abs=1e-9)
        a = d % 3
        grads = (ub, vb, wb)

        def with_vel(x, a=a):
            vv = [U, V, W]
            vv[a] = x
            return oracle.step(phi, *vv, **step_kw)

        fd = _fd_check(with_vel, (U, V, W)[a], v, lam, 1e-6)
        assert np.sum(grads[a] * v) == pytest.approx(fd, rel=2e-7, abs=1e-9)


@pytest.mark.parametrize("scheme,walls", [(4, (True, False, False)), (4, (False, True, True)),
                                          (1, (True, True, True)), (2, (False, False, True)),
                                          (3, (True, True, False))])
def test_adjoint_step_with_walls_matches_finite_differences(scheme, walls):
    """The adjoint on walled axes against central differences of the walled forward (16
    directions in phi, and in each face array: the wall faces' velocity has no effect, so its
    gradient is zero there)."""
    rng, phi, vel, kw = setup(9, delta=0.2)
    U, V, W = vel
    step_kw = dict(dt=0.05 * kw["dx"], scheme=scheme, vel_mode=1, vel_T=0.9, t0=0.2,
                   walls=walls, **kw)
    adj_kw = dict(dt=step_kw["dt"], scheme=scheme, vel_mode=1, vel_T=0.9, t=0.2, walls=walls,
                  **kw)
    lam = rng.standard_normal(phi.shape)
    lam_n, ub, vb, wb = oracle.adjoint_step(phi, U, V, W, lam, **adj_kw)
    grads = (ub, vb, wb)
    for a, w in enumerate(walls):  # no gradient on the wall faces (index 0 of a walled axis)
        if w:
            sl = [slice(None)] * 3
            sl[2 - a] = 0
            assert not grads[a][tuple(sl)].any()
    for d in range(16):
        v = rng.standard_normal(phi.shape)
        fd = _fd_check(lambda p: oracle.step(p, U, V, W, **step_kw), phi, v, lam, 1e-6)
        assert np.sum(lam_n * v) == pytest.approx(fd, rel=2e-7, abs=1e-9)
        a = d % 3

        def with_vel(x, a=a):
            vv = [U, V, W]
            vv[a] = x
            return oracle.step(phi, *vv, **step_kw)

        fd = _fd_check(with_vel, (U, V, W)[a], v, lam, 1e-6)
        assert np.sum(grads[a] * v) == pytest.approx(fd, rel=2e-7, abs=1e-9)


def test_adjoint_two_steps_chain():
    """Two adjoint steps in sequence equal the adjoint of the two-step map (by FD)."""
    rng, phi, vel, kw = setup(3)
    dt = 0.05 * kw["dx"]
    lam = rng.standard_normal(phi.shape)
    phi1 = oracle.step(phi, *vel, dt=dt, **kw)
    l1, *_ = oracle.adjoint_step(phi1, *vel, lam, dt=dt, t=dt, **kw)
    l0, *_ = oracle.adjoint_step(phi, *vel, l1, dt=dt, t=0.0, **kw)
    v = rng.standard_normal(phi.shape)
    fd = _fd_check(lambda p: oracle.step(p, *vel, dt=dt, nsteps=2, **kw), phi, v, lam, 1e-6)
    assert np.sum(l0 * v) == pytest.approx(fd, rel=2e-7)


# --------------------------------------------------------------------- velocity synthesis


def _single_mode(M, m, comp, val=1.0):
    c = np.zeros((M, M, M, 3))
    c[m[2] - 1, m[1] - 1, m[0] - 1, comp] = val
    return c


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_single_mode_closed_form(comp):
    """Discrete curl of one separable mode. A one-cell difference of sin(2 pi m x + t) is
    (2/dx) sin(pi m dx) cos(2 pi m (x + dx/2) + t); positions follow the edge layout."""
    n = (10, 12, 14)  # nx, ny, nz
    shape = (n[2], n[1], n[0])
    dx = 1.0 / n[0]  # box lengths are n*dx; modes use x / L
    M = 3
    rng = np.random.default_rng(5)
    th = rng.uniform(0, 2 * np.pi, size=(3, M))
    m = (2, 3, 1)
    U, V, W = oracle.velocity_from_coeffs(shape, dx=dx, phases=th, coeffs=_single_mode(M, m, comp, 1.7))
    L = [nn * dx for nn in n]
    node = [np.arange(nn) * dx for nn in n]
    mid = [(np.arange(nn) + 0.5) * dx for nn in n]
    S = lambda a, x: np.sin(2 * np.pi * m[a] * x / L[a] + th[a, m[a] - 1])  # noqa: E731
    D = lambda a, x: (2 / dx) * np.sin(np.pi * m[a] * dx / L[a]) * np.cos(  # noqa: E731
        2 * np.pi * m[a] * x / L[a] + th[a, m[a] - 1])
    outer = lambda fx_, fy, fz: fz[:, None, None] * fy[None, :, None] * fx_[None, None, :]  # noqa: E731
    Z = np.zeros(shape)
    if comp == 2:   # Az at (node, node, mid): U = +d/dy Az, V = -d/dx Az
        eU = outer(S(0, node[0]), D(1, mid[1]), S(2, mid[2]))
        eV = -outer(D(0, mid[0]), S(1, node[1]), S(2, mid[2]))
        eW = Z
    elif comp == 1:  # Ay at (node, mid, node): U = -d/dz Ay, W = +d/dx Ay
        eU = -outer(S(0, node[0]), S(1, mid[1]), D(2, mid[2]))
        eV = Z
        eW = outer(D(0, mid[0]), S(1, mid[1]), S(2, node[2]))
    else:            # Ax at (mid, node, node): V = +d/dz Ax, W = -d/dy Ax
        eU = Z
        eV = outer(S(0, mid[0]), S(1, node[1]), D(2, mid[2]))
        eW = -outer(S(0, mid[0]), D(1, mid[1]), S(2, node[2]))
    for got, exp in ((U, eU), (V, eV), (W, eW)):
        np.testing.assert_allclose(got, 1.7 * exp, rtol=0, atol=1e-12)


def test_random_field_unit_rms_and_divergence_free():
    """The fixture's exact discrete-RMS scaling gives RMS 1 of the oracle's field; the
    discrete divergence vanishes to round-off."""
    n, M = 16, 4
    rng = np.random.default_rng(6)
    th, c = fx.random_modes(rng, M, n)
    U, V, W = oracle.velocity_from_coeffs((n, n, n), dx=1.0 / n, phases=th, coeffs=c)
    rms = np.sqrt((np.mean(U ** 2) + np.mean(V ** 2) + np.mean(W ** 2)) / 3)
    assert rms == pytest.approx(1.0, rel=1e-12)
    div = (np.roll(U, -1, 2) - U + np.roll(V, -1, 1) - V + np.roll(W, -1, 0) - W) * n
    assert np.abs(div).max() < 1e-11 * np.abs(U).max() * n


def test_velocity_transpose_dot_product():
    shape, M = (6, 8, 10), 3
    dx = 0.1
    rng = np.random.default_rng(7)
    th = rng.uniform(0, 2 * np.pi, size=(3, M))
    c = rng.standard_normal((M, M, M, 3))
    U, V, W = oracle.velocity_from_coeffs(shape, dx=dx, phases=th, coeffs=c)
    ub, vb, wb = (rng.standard_normal(shape) for _ in range(3))
    cb = oracle.velocity_from_coeffs_T(shape, dx=dx, phases=th, Ubar=ub, Vbar=vb, Wbar=wb)
    lhs = np.sum(U * ub) + np.sum(V * vb) + np.sum(W * wb)
    assert lhs == pytest.approx(np.sum(c * cb), rel=1e-12)
