"""Parity at the full benchmark size (512^3), on sampled cells.

Inputs are built on the host (seeded drops; the Fourier face field contracted with numpy), so
no oracle input comes from the GPU path. The GPU advances the whole grid in the benchmark's
configuration (tuned tile variant, FP32 storage). The oracle cannot step 134M cells in a test,
but a cell's value after m RK4 steps depends only on the input within 8m cells of it (four
stages, each reaching two cells along an axis; 4m for RK2's two stages), so the oracle runs on a
periodic patch of that radius plus 2 around each sampled cell and its centre value is exact.
The non-uniform mesh at the same size is sampled the same way (its widths sliced with the patch),
for a step and for an adjoint step. The adjoint workload (128^3) is compared on every cell.
"""
import numpy as np
import pytest
import torch

import oracle
import pf_fixtures as fx

pytestmark = pytest.mark.gpu


def patch(a, k, j, i, R):
    n = a.shape
    kk = (k + np.arange(-R, R + 1)) % n[0]
    jj = (j + np.arange(-R, R + 1)) % n[1]
    ii = (i + np.arange(-R, R + 1)) % n[2]
    return a[np.ix_(kk, jj, ii)]


@pytest.fixture(scope="module")
def case512():
    c = fx.roofline512(512)
    U, V, W = fx.fourier_faces(c.shape, c.dx, *c.modes)
    fx.set_speed(c, fx.max_face_speed(U, V, W))
    return c, U, V, W


def sample_cells(phi, rng, count):
    inter = np.argwhere((phi > 0.05) & (phi < 0.95))
    pick = inter[rng.choice(len(inter), count // 2, replace=False)]
    rand = rng.integers(0, phi.shape[0], size=(count - count // 2, 3))
    return np.concatenate([pick, rand])


@pytest.mark.parametrize("dtype,nsteps,tol,scheme", [("f32", 2, 1e-5, "rk4"), ("f64", 1, 1e-12, "rk4"),
                                                    ("f32", 3, 1e-5, "rk2")])
def test_fullsize_sampled_parity(lib, case512, dtype, nsteps, tol, scheme):
    pf = lib
    c, U, V, W = case512
    np_dt = np.float32 if dtype == "f32" else np.float64
    tdt = torch.float32 if dtype == "f32" else torch.float64
    inputs = [a.astype(np_dt).astype(np.float64) for a in (c.phi0, U, V, W)]
    n = c.shape[0]
    st = torch.cuda.Stream()
    # RK2 at 0.9 x its diffusive limit (Eq. 26, three axes), below RK4's step
    dt = c.dt if scheme == "rk4" else min(c.dt, 0.9 * c.dx * c.dx / (6.0 * c.gamma * c.eps))
    s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, dt, dtype=dtype, scheme=scheme)
    s.autotune(reps=1, stream=st)
    print("variant", s.variant_name, flush=True)
    g = [torch.tensor(a, dtype=tdt, device="cuda") for a in inputs]
    m0 = s.reduce(g[0], stream=st)
    with torch.cuda.stream(st):
        s.step(*g, nsteps=nsteps, stream=st)
    m1 = s.reduce(g[0], stream=st)
    out = g[0].cpu().numpy().astype(np.float64)
    del g
    s.close()
    drift = abs(m1[0] - m0[0]) / m0[0]
    assert drift <= (1e-6 if dtype == "f32" else 1e-13), drift
    R = (8 if scheme == "rk4" else 4) * nsteps + 2
    rng = np.random.default_rng(17)
    worst = 0.0
    for (k, j, i) in sample_cells(inputs[0], rng, 24):
        pp = [patch(a, k, j, i, R) for a in inputs]
        ref = oracle.step(*pp, dx=c.dx, eps=c.eps, gamma=c.gamma, dt=dt, nsteps=nsteps,
                          fp32=(dtype == "f32"), scheme=4 if scheme == "rk4" else 2)
        worst = max(worst, abs(out[k, j, i] - ref[R, R, R]))
    print(dtype, scheme, "worst sampled |gpu - oracle| =", worst, "mass drift", drift, flush=True)
    assert worst <= tol * np.abs(out).max()


def _drops_f32(n, dx, centres, radii, eps, dtype=np.float32):
    """The fixture's drop union, built window by window straight into the storage dtype (the
    union of tanh profiles is the profile of the union, and rounding commutes with max)."""
    phi = np.zeros((n, n, n), dtype=dtype)
    for c, r in zip(centres, radii):
        reach = r + 60.0 * eps
        ix, ox = fx._axis_offsets(n, dx, c[0], n * dx, reach)
        iy, oy = fx._axis_offsets(n, dx, c[1], n * dx, reach)
        iz, oz = fx._axis_offsets(n, dx, c[2], n * dx, reach)
        dist = np.sqrt(oz[:, None, None] ** 2 + oy[None, :, None] ** 2 + ox[None, None, :] ** 2)
        prof = fx.tanh_profile(r - dist, eps).astype(dtype)
        sel = np.ix_(iz, iy, ix)
        phi[sel] = np.maximum(phi[sel], prof)
    return phi


@pytest.mark.parametrize("dtype,n", [("f32", 1024), ("f64", 816)])
def test_4gib_fields_switch_to_per_plane_addressing(lib, dtype, n):
    """At 1024^3 FP32 (4 GiB) and 816^3 FP64 (4.35 GB, ragged against the 32x16 tiles) every
    field is past the 32-bit offsets of one buffer descriptor, and the z-marches switch to
    per-plane descriptors by themselves. Two RK4 steps of the default (fused) variant, checked
    against the oracle on sampled patches as above (FP32 1e-5 against the FP32-storage mode,
    FP64 1e-12). Velocity: U(y, z), V(z, x), W(x, y), products of sines; each component is
    constant along its own axis, so the discrete divergence vanishes exactly."""
    pf = lib
    np_dt = np.float32 if dtype == "f32" else np.float64
    dx = 1.0 / n
    eps, gamma, nsteps = dx, 1.1, 2
    dt = fx.rk4_dt_3d(dx, gamma, eps)
    rng = np.random.default_rng(29)
    centres, radii = rng.uniform(0.2, 0.8, size=(3, 3)), np.array([0.12, 0.08, 0.1])
    print(f"building {n}^3 {dtype} inputs", flush=True)
    phi = _drops_f32(n, dx, centres, radii, eps, np_dt)
    x = ((np.arange(n) + 0.5) * dx).astype(np.float64)
    s1, c2 = np.sin(2 * np.pi * x + 0.3), np.cos(4 * np.pi * x + 1.1)
    full = (n, n, n)
    U = np.ascontiguousarray(np.broadcast_to(np.multiply.outer(c2, s1).astype(np_dt)[:, :, None], full))
    V = np.ascontiguousarray(np.broadcast_to(np.multiply.outer(s1, c2).astype(np_dt)[:, None, :], full))
    W = np.ascontiguousarray(np.broadcast_to(np.multiply.outer(c2, s1).astype(np_dt)[None, :, :], full))
    inputs = (phi, U, V, W)
    assert phi.nbytes >= 4 * 2 ** 30 or phi.nbytes > 2 ** 32 - 1
    st = torch.cuda.Stream()
    s = pf.Solver((n, n, n), dx, eps, gamma, dt, dtype=dtype)
    print("variant", s.variant_name, flush=True)
    g = [torch.from_numpy(a).cuda() for a in inputs]
    m0 = s.reduce(g[0], stream=st)
    with torch.cuda.stream(st):
        s.step(*g, nsteps=nsteps, stream=st)
    m1 = s.reduce(g[0], stream=st)
    out = g[0].cpu().numpy()
    del g
    s.close()
    torch.cuda.empty_cache()
    drift = abs(m1[0] - m0[0]) / m0[0]
    print("mass drift", drift, flush=True)
    assert drift <= (1e-6 if dtype == "f32" else 1e-13)
    R = 8 * nsteps + 2
    worst = 0.0
    samples = sample_cells(phi, np.random.default_rng(31), 16)
    for (k, j, i) in samples:
        pp = [patch(a, k, j, i, R).astype(np.float64) for a in inputs]
        ref = oracle.step(*pp, dx=dx, eps=eps, gamma=gamma, dt=dt, nsteps=nsteps,
                          fp32=dtype == "f32")
        worst = max(worst, abs(float(out[k, j, i]) - ref[R, R, R]))
    print("worst sampled |gpu - oracle| =", worst, flush=True)
    assert worst <= (1e-5 if dtype == "f32" else 1e-12)


@pytest.mark.parametrize("form", [-1, 1])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-3)])
def test_adjoint_workload_full_grid(lib, dtype, tol, form):
    """The adjoint workload at its full size (128^3, 8-mode field, delta = 1e-3/dx): one adjoint
    step in the configuration the benchmark times (default variant: fused sweeps recompute the
    stage inputs, tiled reverse stages) against the oracle's FP64 adjoint on every cell, for
    lambda and the three face-velocity gradients, at the fixed bars: 1e-12 in FP64, and 1e-3 for
    FP32 storage against the FP64 oracle. With this delta the problem is well conditioned: the
    oracle's own output moves by about 2e-14 (FP64) and 9e-6 (FP32) when phi is scaled by
    1 + u (seeded noise, u the storage's unit roundoff); the test prints that response.
    Run with the reverse RK4 stages the handle chooses (one per launch at this size) and with
    two per launch."""
    pf = lib
    c = fx.adjoint_case(128)
    U, V, W = oracle.velocity_from_coeffs(c.shape, dx=c.dx, phases=c.modes[0], coeffs=c.modes[1])
    fx.set_speed(c, fx.max_face_speed(U, V, W))
    rng = np.random.default_rng(11)
    lam = rng.standard_normal(c.shape)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":  # the oracle sees the values the GPU stores
        phi, U, V, W, lam = (a.astype(np.float32).astype(np.float64) for a in (c.phi0, U, V, W, lam))
    else:
        phi = c.phi0
    ref = oracle.adjoint_step(phi, U, V, W, lam, dx=c.dx, eps=c.eps, gamma=c.gamma, dt=c.dt,
                              delta=c.delta)
    n = c.shape[0]
    s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, c.dt, dtype=dtype, delta=c.delta)
    s.set_adjoint_form(form)
    print(dtype, "variant", s.variant_name, "adjoint form", form, flush=True)
    g = [torch.tensor(a, dtype=tdt, device="cuda") for a in (phi, U, V, W)]
    L = torch.tensor(lam, dtype=tdt, device="cuda")
    grads = [torch.zeros_like(L) for _ in range(3)]
    s.adjoint_step(*g, 0.0, L, *grads)
    torch.cuda.synchronize()
    s.close()
    u = 1e-16 if dtype == "f64" else 2.0 ** -24
    wobble = np.random.default_rng(12).standard_normal(c.shape)
    ref_p = oracle.adjoint_step(phi * (1 + u * wobble), U, V, W, lam, dx=c.dx, eps=c.eps,
                                gamma=c.gamma, dt=c.dt, delta=c.delta)
    for k, (got, want) in enumerate(zip([L] + grads, ref)):
        got = got.cpu().numpy().astype(np.float64)
        assert np.isfinite(got).all(), k
        scale = np.abs(want).max()
        err = float(np.abs(got - want).max() / scale)
        resp = float(np.abs(ref_p[k] - want).max() / scale)
        print("output", k, "error", err, "oracle response to unit roundoff", resp, flush=True)
        assert err <= tol, (k, err, tol)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fullsize_nonuniform_sampled_parity(lib, case512, dtype):
    """The non-uniform leg at its benchmark size: 512^3 with widths varying 2x smoothly along
    every axis and eps tuned to the local mesh, delta = 1e-3/dx, a default-variant handle (the
    per-stage NU kernel, the tiled NU reverse stages). One RK4 step and one adjoint step on the
    whole grid; sampled cells against the oracle on periodic patches whose widths are sliced
    alike. A step's output reaches 8 cells of input; the adjoint's lambda and face gradients reach
    8 cells of the cotangent and 16 of phi (through the stage inputs), so patches of radius 10 and
    18 make the centre values exact. FP64 within 1e-12 of each output's largest sampled value;
    FP32 storage: the step within 1e-5 of the oracle's FP32-storage mode, the adjoint within 1e-3
    of the FP64 oracle."""
    pf = lib
    c, U, V, W = case512
    n = c.shape[0]
    h = [fx.smooth_widths(n, 1.0, 2.0, 0.9 * a) for a in range(3)]
    dt = min(c.dt, 0.1 * min(map(min, h)) ** 2 / (c.gamma * c.eps * max(map(max, h)) / c.dx))
    delta = 1e-3 / c.dx
    np_dt = np.float32 if dtype == "f32" else np.float64
    tdt = torch.float32 if dtype == "f32" else torch.float64
    inputs = [a.astype(np_dt).astype(np.float64) for a in (c.phi0, U, V, W)]
    lam = np.random.default_rng(23).standard_normal(c.shape).astype(np_dt).astype(np.float64)
    s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, dt, dtype=dtype, delta=delta)
    s.set_spacing(*h, eps_mode=1)
    print(dtype, "variant", s.variant_name, flush=True)
    g = [torch.tensor(a, dtype=tdt, device="cuda") for a in inputs]
    phi1 = g[0].clone()
    s.step(phi1, *g[1:], nsteps=1)
    out = phi1.cpu().numpy().astype(np.float64)
    del phi1
    L = torch.tensor(lam, dtype=tdt, device="cuda")
    grads = [torch.zeros_like(L) for _ in range(3)]
    s.adjoint_step(*g, 0.0, L, *grads)
    adj = [t.cpu().numpy().astype(np.float64) for t in [L] + grads]
    del g, L, grads
    s.close()
    kw = dict(dx=c.dx, eps=c.eps, gamma=c.gamma, dt=dt, delta=delta, eps_mode=1)
    cells = sample_cells(inputs[0], np.random.default_rng(29), 12)

    def widths(k, j, i, R):
        return dict(hx=h[0][(i + np.arange(-R, R + 1)) % n], hy=h[1][(j + np.arange(-R, R + 1)) % n],
                    hz=h[2][(k + np.arange(-R, R + 1)) % n])

    worst, scale = 0.0, 0.0
    for (k, j, i) in cells:
        R = 10
        pp = [patch(a, k, j, i, R) for a in inputs]
        ref = oracle.step_nu(*pp, **widths(k, j, i, R), fp32=(dtype == "f32"), **kw)
        worst = max(worst, abs(out[k, j, i] - ref[R, R, R]))
        scale = max(scale, abs(ref[R, R, R]))
    print(dtype, "step: worst sampled |gpu - oracle|", worst, "of", scale, flush=True)
    assert worst <= (1e-12 if dtype == "f64" else 1e-5) * max(scale, 1.0)
    worst, scale = [0.0] * 4, [0.0] * 4
    for (k, j, i) in cells:
        R = 18
        pp = [patch(a, k, j, i, R) for a in inputs]
        ref = oracle.adjoint_step_nu(*pp, patch(lam, k, j, i, R), **widths(k, j, i, R), t=0.0, **kw)
        for q in range(4):
            worst[q] = max(worst[q], abs(adj[q][k, j, i] - ref[q][R, R, R]))
            scale[q] = max(scale[q], abs(ref[q][R, R, R]))
    print(dtype, "adjoint: worst sampled |gpu - oracle|", worst, "of", scale, flush=True)
    tol = 1e-12 if dtype == "f64" else 1e-3
    for q in range(4):
        assert scale[q] > 0.0, q
        assert worst[q] <= tol * scale[q], (q, worst[q], scale[q])
