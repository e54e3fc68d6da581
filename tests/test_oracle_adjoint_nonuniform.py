"""Pins of the oracle's adjoint on non-uniform rectilinear meshes (no GPU).

The transpose of the non-uniform step's Jacobian is pinned against (a) reverse-mode autodiff of
an independent torch statement of the non-uniform flux form (periodic axes, both eps modes),
(b) central finite differences of the oracle's own non-uniform forward (walled axes, every
scheme, time-varying velocity, one-plane grids) and (c) the uniform adjoint, which equal widths
must reproduce.
"""
import numpy as np
import pytest
import torch

import oracle
import pf_fixtures as fx


def torch_rhs_nu(phi, U, V, W, h, dx, eps, gamma, delta, s, eps_mode):
    """Flux form on a periodic non-uniform mesh in torch FP64: gradient over the distance
    between the two neighbours' centres, diffusion over the distance between the face's two
    cell centres, divergence over the cell width; eps per cell (mode 1: eps * largest width of
    the axes longer than one cell / dx), averaged onto the face."""
    dims = {0: 2, 1: 1, 2: 0}  # x -> last array axis

    def sh(a, d, ax):
        return torch.roll(a, shifts=-d, dims=dims[ax])

    def along(v, ax):
        shape = [1, 1, 1]
        shape[dims[ax]] = -1
        return v.reshape(shape)

    dist = [0.5 * (torch.roll(h[a], 1) + h[a]) for a in range(3)]  # centres of cells i-1 and i
    span = [dist[a] + torch.roll(dist[a], -1) for a in range(3)]    # centres of cells i-1 and i+1
    g = [(sh(phi, 1, a) - sh(phi, -1, a)) / along(span[a], a) for a in range(3)]
    mag = torch.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2 + delta ** 2)
    w = phi * (1 - phi)
    if eps_mode:
        widths = [along(h[a], a).expand_as(phi) for a in range(3) if phi.shape[dims[a]] > 1]
        ec = eps * torch.stack(widths).amax(0) / dx
    else:
        ec = torch.full_like(phi, eps)
    vel = (U, V, W)
    f = torch.zeros_like(phi)
    for a in range(3):
        q = w * g[a] / mag
        eps_f = 0.5 * (sh(ec, -1, a) + ec)
        F = (-s * vel[a] * 0.5 * (sh(phi, -1, a) + phi)
             + gamma * eps_f * (phi - sh(phi, -1, a)) / along(dist[a], a)
             - gamma * 0.5 * (sh(q, -1, a) + q))
        f = f + (sh(F, 1, a) - F) / along(h[a], a)
    return f


def setup(seed, shape=(6, 7, 9), delta=0.3, ratio=2.5):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    dx = 1.0 / nx
    h = [fx.random_widths(rng, n, 1.0, ratio) for n in (nx, ny, nz)]
    phi = (fx.drops_ic(shape, dx, [(0.5 * nx * dx, 0.5 * ny * dx, 0.5 * nz * dx)], [0.3], dx) * 0.8
           + 0.2 * rng.uniform(size=shape))
    U, V, W = (rng.standard_normal(shape) for _ in range(3))
    kw = dict(hx=h[0], hy=h[1], hz=h[2], dx=dx, eps=1.1 * dx, gamma=1.3, delta=delta / dx)
    return rng, phi, (U, V, W), h, kw


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("eps_mode", [0, 1])
def test_torch_statement_matches_oracle_forward_nu(eps_mode):
    rng, phi, vel, h, kw = setup(0)
    f = oracle.rhs_nu(phi, *vel, s=0.7, eps_mode=eps_mode, **kw)
    t = torch_rhs_nu(*(torch.tensor(a) for a in (phi, *vel)), [torch.tensor(x) for x in h],
                     kw["dx"], kw["eps"], kw["gamma"], kw["delta"], 0.7, eps_mode)
    np.testing.assert_allclose(t.numpy(), f, rtol=0, atol=1e-12 * np.abs(f).max())


@pytest.mark.parametrize("eps_mode,delta,shape", [(0, 0.3, (6, 7, 9)), (1, 0.3, (6, 7, 9)),
                                                  (1, 0.0, (5, 8, 6)), (1, 0.3, (1, 9, 10))])
def test_rhs_vjp_nu_matches_autodiff(eps_mode, delta, shape):
    rng, phi, vel, h, kw = setup(1, shape=shape, delta=delta)
    lam = rng.standard_normal(phi.shape)
    pb, ub, vb, wb = oracle.rhs_vjp_nu(phi, *vel, lam, s=0.6, eps_mode=eps_mode, **kw)
    ts = [torch.tensor(a, requires_grad=True) for a in (phi, *vel)]
    f = torch_rhs_nu(*ts, [torch.tensor(x) for x in h], kw["dx"], kw["eps"], kw["gamma"],
                     kw["delta"], 0.6, eps_mode)
    f.backward(torch.tensor(lam))
    for mine, ref in zip((pb, ub, vb, wb), ts):
        r = ref.grad.numpy()
        np.testing.assert_allclose(mine, r, rtol=0, atol=1e-12 * np.abs(r).max())


@pytest.mark.parametrize("walls", [(True, False, False), (False, True, True), (True, True, True)])
def test_rhs_vjp_nu_matches_finite_differences_with_walls(walls):
    rng, phi, vel, h, kw = setup(2, shape=(7, 6, 8))
    lam = rng.standard_normal(phi.shape)
    pb, ub, vb, wb = oracle.rhs_vjp_nu(phi, *vel, lam, s=0.8, eps_mode=1, walls=walls, **kw)
    eps = 1e-6
    for k in range(4):
        d = rng.standard_normal(phi.shape)
        if k == 0:
            fp = oracle.rhs_nu(phi + eps * d, *vel, s=0.8, eps_mode=1, walls=walls, **kw)
            fm = oracle.rhs_nu(phi - eps * d, *vel, s=0.8, eps_mode=1, walls=walls, **kw)
            mine = float((d * pb).sum())
        else:
            vp = [v.copy() for v in vel]
            vm = [v.copy() for v in vel]
            vp[k - 1] += eps * d
            vm[k - 1] -= eps * d
            fp = oracle.rhs_nu(phi, *vp, s=0.8, eps_mode=1, walls=walls, **kw)
            fm = oracle.rhs_nu(phi, *vm, s=0.8, eps_mode=1, walls=walls, **kw)
            mine = float((d * (ub, vb, wb)[k - 1]).sum())
        fd = float((lam * (fp - fm)).sum() / (2 * eps))
        assert rel(mine, fd) <= 2e-7, (k, mine, fd)


@pytest.mark.parametrize("scheme,walls,shape", [(4, (False, False, False), (6, 7, 8)),
                                                (3, (True, False, False), (6, 7, 8)),
                                                (2, (False, True, True), (6, 7, 8)),
                                                (1, (True, True, False), (6, 7, 8)),
                                                (4, (False, False, False), (1, 8, 9))])
def test_adjoint_step_nu_matches_finite_differences(scheme, walls, shape):
    rng, phi, vel, h, kw = setup(3, shape=shape)
    kw.update(dt=0.05 * min(map(min, h)) ** 2 / (kw["gamma"] * kw["eps"]) * 10.0, eps_mode=1,
              walls=walls)
    step_kw = dict(kw)
    lam = rng.standard_normal(phi.shape)
    adj = oracle.adjoint_step_nu(phi, *vel, lam, t=0.2, scheme=scheme, vel_mode=1, vel_T=0.9, **kw)
    eps = 1e-6
    for k in range(4):
        d = rng.standard_normal(phi.shape)
        args_p, args_m = [phi, *vel], [phi, *vel]
        args_p = [a + (eps * d if i == k else 0.0) for i, a in enumerate(args_p)]
        args_m = [a - (eps * d if i == k else 0.0) for i, a in enumerate(args_m)]
        fp = oracle.step_nu(*args_p, t0=0.2, scheme=scheme, vel_mode=1, vel_T=0.9, **step_kw)
        fm = oracle.step_nu(*args_m, t0=0.2, scheme=scheme, vel_mode=1, vel_T=0.9, **step_kw)
        fd = float((lam * (fp - fm)).sum() / (2 * eps))
        mine = float((d * adj[k]).sum())
        assert rel(mine, fd) <= 2e-7, (k, mine, fd)


@pytest.mark.parametrize("scheme", [1, 2, 3, 4])
def test_equal_widths_reduce_to_the_uniform_adjoint(scheme):
    rng, phi, vel, h, kw = setup(4, shape=(6, 7, 8))
    dx = kw["dx"]
    uni = dict(dx=dx, eps=kw["eps"], gamma=kw["gamma"], delta=kw["delta"], dt=0.1 * dx)
    lam = rng.standard_normal(phi.shape)
    walls = (True, False, True)
    a = oracle.adjoint_step(phi, *vel, lam, t=0.1, scheme=scheme, vel_mode=1, vel_T=0.7,
                            walls=walls, **uni)
    b = oracle.adjoint_step_nu(phi, *vel, lam, hx=np.full(8, dx), hy=np.full(7, dx),
                               hz=np.full(6, dx), t=0.1, scheme=scheme, vel_mode=1, vel_T=0.7,
                               eps_mode=1, walls=walls, **uni)
    for x, y in zip(a, b):
        np.testing.assert_allclose(y, x, rtol=0, atol=1e-13 * np.abs(x).max())
