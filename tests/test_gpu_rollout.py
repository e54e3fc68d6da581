"""The differentiable rollout (Rollout: forward steps with checkpoints, discrete adjoint
backward) on the adjoint workload at its stated size: 128^3, a seeded 8-mode solenoidal field
(8^3 x 3 potential coefficients), a drop of R = 0.2 carried for 400 RK4 steps, loss
L = 0.5 |phi_T - target|^2 against a centred drop of R = 0.2, checkpoint every 20 steps,
delta = 1e-3/dx. Gradients with respect to phi_0 and the coefficients.

FP64 is checked three ways: bitwise invariance under the checkpoint interval (1, 20, 400); the
oracle's adjoint chain on a 24-step horizon (checkpoint 10: segments 10, 10, 4) at 1e-11 (the
oracle runs on the host; the full 400-step chain would take it tens of minutes); and central
finite differences of the GPU forward on 16 seeded directions (8 in phi_0, 8 in the
coefficients), h = 1e-6 |x| / |d|, fourth-order formula, at 1e-6 relative. FP32 storage is
checked against the FP64 gradient at 1e-3 (relative L-inf of each gradient, and each
directional derivative), and for bitwise checkpoint invariance.
"""
import numpy as np
import pytest
import torch

import oracle
import pf_fixtures as fx

pytestmark = pytest.mark.gpu

NSTEPS, CKPT = 400, 20


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_linf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def workload(lib):
    pf = lib
    c = fx.adjoint_case(128)
    th, co = (dev(a) for a in c.modes)
    p0 = pf.make_params(c.shape, c.dx, c.eps, 1.0, 1.0)
    u, v, w = pf.velocity_from_coeffs(p0, th, co)
    torch.cuda.synchronize()
    fx.set_speed(c, max(float(t.abs().max()) for t in (u, v, w)))
    return c


def solver(pf, c, dtype):
    n = c.shape[0]
    return pf.Solver((n, n, n), c.dx, c.eps, c.gamma, c.dt, dtype=dtype, delta=c.delta)


def loss(pf, s, th, coeffs, phi0, target, nsteps, ckpt):
    phiT = pf.Rollout.apply(phi0, coeffs, s, th, nsteps, ckpt, 0.0)
    return 0.5 * ((phiT - target) ** 2).sum()


def grads(pf, s, c, dtype, nsteps, ckpt):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    th = dev(c.modes[0])
    p0 = dev(c.phi0, tdt).requires_grad_(True)
    cc = dev(c.modes[1]).requires_grad_(True)
    L = loss(pf, s, th, cc, p0, dev(c.extra["target"], tdt), nsteps, ckpt)
    L.backward()
    torch.cuda.synchronize()
    return host(p0.grad), host(cc.grad)


@pytest.fixture(scope="module")
def fp64_grads(lib, workload):
    s = solver(lib, workload, "f64")
    g = grads(lib, s, workload, "f64", NSTEPS, CKPT)
    s.close()
    return g


def directions(c, count=16, seed=0):
    """Seeded directions: the first half in phi_0 only, the second in the coefficients only."""
    out = []
    for k in range(count):
        rng = np.random.default_rng(seed + k)
        if k < count // 2:
            out.append((rng.standard_normal(c.shape), np.zeros(c.modes[1].shape)))
        else:
            out.append((np.zeros(c.shape), rng.standard_normal(c.modes[1].shape)))
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rollout_checkpoint_invariance(lib, workload, dtype):
    s = solver(lib, workload, dtype)
    ref = grads(lib, s, workload, dtype, NSTEPS, CKPT)
    for ck in (1, NSTEPS):
        got = grads(lib, s, workload, dtype, NSTEPS, ck)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), ck
    s.close()


def test_rollout_fp64_matches_oracle_chain(lib, workload):
    """24 steps with checkpoints every 10 (a ragged last segment) against the oracle's FP64
    adjoint chain: forward states, reverse sweep of adjoint steps, projection of the face
    gradients onto the coefficients."""
    pf = lib
    c = workload
    nsteps, ckpt = 24, 10
    s = solver(pf, c, "f64")
    gphi, gco = grads(pf, s, c, "f64", nsteps, ckpt)
    s.close()
    U, V, W = oracle.velocity_from_coeffs(c.shape, dx=c.dx, phases=c.modes[0], coeffs=c.modes[1])
    kw = dict(dx=c.dx, eps=c.eps, gamma=c.gamma, dt=c.dt, delta=c.delta)
    print("oracle chain running (128^3, 24 steps)", flush=True)
    states = [c.phi0]
    for n in range(nsteps):
        states.append(oracle.step(states[-1], U, V, W, **kw))
    lam = states[-1] - c.extra["target"]
    gu, gv, gw = (np.zeros(c.shape) for _ in range(3))
    for n in reversed(range(nsteps)):
        lam, a, b, d = oracle.adjoint_step(states[n], U, V, W, lam, t=n * c.dt, **kw)
        gu += a
        gv += b
        gw += d
    cg = oracle.velocity_from_coeffs_T(c.shape, dx=c.dx, phases=c.modes[0], Ubar=gu, Vbar=gv,
                                       Wbar=gw)
    e_phi, e_co = rel_linf(gphi, lam), rel_linf(gco, cg)
    print("rollout vs oracle chain: dL/dphi0", e_phi, "dL/dcoeffs", e_co, flush=True)
    assert e_phi <= 1e-11 and e_co <= 1e-11


def test_rollout_fp64_matches_finite_differences(lib, workload, fp64_grads):
    pf = lib
    c = workload
    s = solver(pf, c, "f64")
    th, tg = dev(c.modes[0]), dev(c.extra["target"])
    gphi, gco = fp64_grads
    nx, ncf = np.linalg.norm(c.phi0), np.linalg.norm(c.modes[1])
    worst = 0.0
    with torch.no_grad():
        for k, (d0, dc) in enumerate(directions(c)):
            d = d0 if k < 8 else dc
            h = 1e-6 * (nx if k < 8 else ncf) / np.linalg.norm(d)

            def L_at(m):
                return float(loss(pf, s, th, dev(c.modes[1] + m * h * dc),
                                  dev(c.phi0 + m * h * d0), tg, NSTEPS, CKPT))

            fd = (8.0 * (L_at(1) - L_at(-1)) - (L_at(2) - L_at(-2))) / (12.0 * h)
            an = float(np.sum(gphi * d0) + np.sum(gco * dc))
            rel = abs(an - fd) / abs(fd)
            worst = max(worst, rel)
            print(f"direction {k}: adjoint {an:.12e} FD {fd:.12e} rel {rel:.2e}", flush=True)
            assert rel <= 1e-6, (k, an, fd)
    print("worst relative FD mismatch", worst, flush=True)
    s.close()


def test_rollout_fp32_close_to_fp64(lib, workload, fp64_grads):
    pf = lib
    c = workload
    s = solver(pf, c, "f32")
    g32 = grads(pf, s, c, "f32", NSTEPS, CKPT)
    s.close()
    e_phi, e_co = rel_linf(g32[0], fp64_grads[0]), rel_linf(g32[1], fp64_grads[1])
    print("FP32 rollout gradient vs FP64: dL/dphi0", e_phi, "dL/dcoeffs", e_co, flush=True)
    assert e_phi <= 1e-3 and e_co <= 1e-3
    for k, (d0, dc) in enumerate(directions(c)):
        a32 = float(np.sum(g32[0] * d0) + np.sum(g32[1] * dc))
        a64 = float(np.sum(fp64_grads[0] * d0) + np.sum(fp64_grads[1] * dc))
        assert abs(a32 - a64) <= 1e-3 * abs(a64), (k, a32, a64)
