"""Stage inputs kept for the adjoint: phasefield_step_stages stores the Runge-Kutta stage values
of one step (Sec. 2.3: RK4 y2, y3, y4; RK3 its first two low-storage stages; RK2 the midpoint
value) and phasefield_adjoint_step_stages takes them instead of recomputing them.

Checked for RK4, RK3, RK2 and Euler, FP64 and FP32, per-stage and fused variants, periodic and
walled grids, one-plane grids, steady and time-varying velocity: the new phi, in place and into
a separate buffer (phi then untouched), bitwise equal to phasefield_step's; lam and the velocity
gradients bitwise equal to phasefield_adjoint_step's (which the adjoint tests hold to the
oracle); every stage buffer written completely; in FP64 each stored stage against its definition
evaluated with the oracle's right-hand side from the previously stored stage (1e-12 relative
L-inf); the Rollout with stage caching, without it and keeping every step bitwise equal; the
argument refusals.
"""
import numpy as np
import pytest
import torch

import oracle
import pf_fixtures as fx

pytestmark = pytest.mark.gpu

F, T = False, True


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_linf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def case(seed, shape):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    dx = 1.0 / max(shape)
    phi = fx.drops_ic(shape, dx, [(0.5 * nx * dx, 0.5 * ny * dx, 0.5 * nz * dx)],
                      [0.3 * max(shape) * dx], 1.5 * dx) * 0.8 + 0.2 * rng.uniform(size=shape)
    U, V, W = fx.random_edge_faces(rng, shape, dx)
    s = 1.0 / fx.max_face_speed(U, V, W)
    lam = rng.standard_normal(shape)
    return phi, U * s, V * s, W * s, lam, dx


CASES = [
    # scheme, dtype, shape (nz, ny, nx), variant (None: the default), walls (x, y, z), vel_mode
    ("rk4", "f64", (20, 18, 40), "fused_32x16", (F, F, F), 1),
    ("rk4", "f64", (20, 18, 40), "tiled_64x8", (F, F, F), 0),
    ("rk4", "f32", (20, 18, 70), "fused_64x8", (F, F, F), 1),
    ("rk4", "f32", (12, 10, 14), "tiled_32x4", (F, F, F), 0),
    ("rk4", "f64", (14, 18, 40), "fused_32x16", (T, F, T), 0),
    ("rk4", "f32", (14, 18, 40), "fused_32x16x32", (F, T, F), 1),
    ("rk4", "f64", (1, 20, 18), None, (F, F, F), 0),
    ("rk4", "f64", (176, 176, 176), "fused_32x16", (F, F, F), 1),  # FP64 fused from 176^3
    ("rk3", "f64", (12, 10, 14), None, (F, F, F), 1),
    ("rk3", "f32", (20, 18, 40), "fused_32x16", (F, F, F), 0),
    ("rk2", "f64", (12, 10, 14), None, (F, F, F), 1),
    ("rk2", "f32", (20, 18, 40), "fused_32x16", (F, T, F), 0),
    ("rk2", "f64", (20, 18, 40), "fused_64x8", (F, F, F), 0),
    ("euler", "f64", (9, 11, 7), None, (F, F, F), 0),
]


@pytest.mark.parametrize("scheme,dtype,shape,vname,walls,vel_mode", CASES)
def test_stages_match_step_and_adjoint_bitwise(lib, scheme, dtype, shape, vname, walls, vel_mode):
    pf = lib
    phi, U, V, W, lam, dx = case(3, shape)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    kd = pf.PF_F64 if dtype == "f64" else pf.PF_F32
    names = [pf.phasefield_variant_name(kd, k) for k in range(pf.phasefield_variant_count(kd))]
    nz, ny, nx = shape
    dt, delta, t, vel_T = 0.12 * dx, 0.05 / dx, 0.1, 0.8
    s = pf.Solver((nx, ny, nz), dx, dx, 1.2, dt, dtype=dtype, scheme=scheme, delta=delta,
                  walls=walls, vel_mode=vel_mode, vel_T=vel_T,
                  variant=-1 if vname is None else names.index(vname))
    print("case", scheme, dtype, shape, s.variant_name, walls, vel_mode, flush=True)
    g = [dev(a, tdt) for a in (phi, U, V, W)]
    ref_phi = g[0].clone()
    s.step(ref_phi, *g[1:], t0=t, nsteps=1)
    lam_ref = dev(lam, tdt)
    grad_ref = [torch.zeros_like(g[0]) for _ in range(3)]
    s.adjoint_step(g[0], *g[1:], t, lam_ref, *grad_ref)

    ns = s.stage_count
    assert ns == {"rk4": 3, "rk3": 2, "rk2": 1, "euler": 0}[scheme]
    ys = [torch.full_like(g[0], float("nan")) for _ in range(ns)]
    phi1 = g[0].clone()
    s.step_stages(phi1, *g[1:], t, *ys)
    # out of place: phi untouched, the same new phi and stages
    ys2 = [torch.full_like(g[0], float("nan")) for _ in range(ns)]
    phi_in = g[0].clone()
    phi2 = torch.full_like(g[0], float("nan"))
    s.step_stages(phi_in, *g[1:], t, *ys2, phi_next=phi2)
    lam1 = dev(lam, tdt)
    grad1 = [torch.zeros_like(g[0]) for _ in range(3)]
    s.adjoint_step_stages(g[0], ys, *g[1:], t, lam1, *grad1)
    torch.cuda.synchronize()
    s.close()
    assert torch.equal(phi1, ref_phi)
    assert torch.equal(phi2, ref_phi) and torch.equal(phi_in, g[0])
    for a, b in zip(ys, ys2):
        assert torch.equal(a, b)
    assert torch.equal(lam1, lam_ref)
    for a, b in zip(grad1, grad_ref):
        assert torch.equal(a, b)
    for y in ys:
        assert bool(torch.isfinite(y).all())
    if dtype != "f64" or ns == 0:
        return
    # each stage from its definition, the oracle's f evaluated at the previous stored stage
    sf = (lambda tt: float(np.cos(np.pi * tt / vel_T))) if vel_mode else (lambda tt: 1.0)

    def f(y, tt):
        return oracle.rhs(y, U, V, W, dx=dx, eps=dx, gamma=1.2, delta=delta, s=sf(tt), walls=walls)

    Y = [host(y) for y in ys]
    if scheme == "rk4":
        refs = [phi + 0.5 * dt * f(phi, t), phi + 0.5 * dt * f(Y[0], t + 0.5 * dt),
                phi + dt * f(Y[1], t + 0.5 * dt)]
    elif scheme == "rk3":
        g1, g2, z2 = 8.0 / 15.0, 5.0 / 12.0, -17.0 / 60.0
        k1 = f(phi, t)
        refs = [phi + dt * g1 * k1, phi + dt * (g1 + z2) * k1 + dt * g2 * f(Y[0], t + g1 * dt)]
    else:
        refs = [phi + 0.5 * dt * f(phi, t)]
    for k, (y, r) in enumerate(zip(Y, refs)):
        err = rel_linf(y, r)
        print("stage", k + 2, "error", err, flush=True)
        assert err <= 1e-12, (k, err)


@pytest.mark.parametrize("dtype,vel_mode", [("f64", 0), ("f32", 1)])
def test_rollout_with_and_without_stage_caching_bitwise(lib, dtype, vel_mode):
    """The checkpointed Rollout (24 steps of 24^3, checkpoint 10: segments 10, 10, 4) gives the
    same gradients and final state bit for bit whether the re-run segments keep their stage
    inputs, each adjoint step recomputes them, or the forward keeps every state and stage input
    (keep_all)."""
    pf = lib
    n = 24
    c = fx.adjoint_case(n)
    th, co = (dev(a) for a in c.modes)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    p0 = pf.make_params(c.shape, c.dx, c.eps, 1.0, 1.0)
    u, v, w = pf.velocity_from_coeffs(p0, th, co)
    torch.cuda.synchronize()
    fx.set_speed(c, max(float(x.abs().max()) for x in (u, v, w)))
    s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, c.dt, dtype=dtype, delta=c.delta,
                  vel_mode=vel_mode, vel_T=40 * c.dt)
    out = []
    for cache, keep_all in ((True, False), (False, False), (None, True)):
        phi0 = dev(c.phi0, tdt).requires_grad_(True)
        cc = dev(c.modes[1]).requires_grad_(True)
        phiT = pf.Rollout.apply(phi0, cc, s, th, 24, 10, 0.0, cache, keep_all)
        L = 0.5 * ((phiT - dev(c.extra["target"], tdt)) ** 2).sum()
        L.backward()
        torch.cuda.synchronize()
        out.append((phi0.grad.clone(), cc.grad.clone(), phiT.detach().clone()))
    s.close()
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert torch.equal(a, b)
    assert float(out[0][0].abs().max()) > 0.0 and float(out[0][1].abs().max()) > 0.0


def test_stage_argument_refusals(lib):
    pf = lib
    phi, U, V, W, lam, dx = case(5, (8, 8, 8))
    s = pf.Solver((8, 8, 8), dx, dx, 1.0, 0.1 * dx)
    g = [dev(a) for a in (phi, U, V, W)]
    y = [torch.zeros_like(g[0]) for _ in range(3)]
    with pytest.raises(pf.PhaseFieldError) as ei:  # RK4 needs y4
        pf.phasefield_step_stages(s.handle, s.params, g[0], *g[1:], 0.0, y[0], y[1], None)
    assert ei.value.status == pf.PF_ERR_INVALID
    with pytest.raises(pf.PhaseFieldError) as ei:  # coinciding stage buffers
        s.step_stages(g[0], *g[1:], 0.0, y[0], y[1], y[1])
    assert ei.value.status == pf.PF_ERR_INVALID
    with pytest.raises(pf.PhaseFieldError) as ei:  # a stage buffer is phi
        s.step_stages(g[0], *g[1:], 0.0, g[0], y[1], y[2])
    assert ei.value.status == pf.PF_ERR_INVALID
    with pytest.raises(pf.PhaseFieldError) as ei:  # a stage buffer is phi_next
        s.step_stages(g[0], *g[1:], 0.0, *y, phi_next=y[2])
    assert ei.value.status == pf.PF_ERR_INVALID
    with pytest.raises(pf.PhaseFieldError) as ei:
        s.step_stages(g[0], *g[1:], float("nan"), *y)
    assert ei.value.status == pf.PF_ERR_INVALID
    lam_t = dev(lam)
    with pytest.raises(pf.PhaseFieldError) as ei:  # the adjoint needs y3
        pf.phasefield_adjoint_step_stages(s.handle, s.params, g[0], y[0], None, y[2], *g[1:], 0.0,
                                          lam_t)
    assert ei.value.status == pf.PF_ERR_INVALID
    s.close()
