"""GPU parity of the non-uniform rectilinear mesh (phasefield_set_spacing) against the oracle.

The oracle's reading of the paper's remark on non-uniform anisotropic Cartesian grids (Sec.
3.3.3, closing list) is pinned on the CPU in test_oracle_nonuniform.py. Here the per-stage kernel
in its non-uniform form runs RK4, RK3, RK2 and Euler on randomly and smoothly stretched meshes,
periodic and walled, with eps fixed or tuned to the local mesh, steady and time-varying
velocity, ragged multi-tile and one-plane grids, against oracle.step_nu: FP64 within 1e-12
relative L-inf, FP32 storage within 1e-5 of the oracle's FP32-storage mode. Also: equal widths
agree with the uniform kernels, the volume-weighted mass, graph replay, and the refusals.

The adjoint step on these meshes (the plain vector-Jacobian product of the non-uniform step,
pinned on the CPU in test_oracle_adjoint_nonuniform.py) against oracle.adjoint_step_nu for every
scheme, periodic and walled axes, both eps rules, steady and time-varying velocity, one-plane
grids and a fused handle: FP64 within 1e-12 relative L-inf for lambda and the three face
gradients, FP32 storage within 1e-3 of the FP64 oracle; with the stage inputs kept by
phasefield_step_stages bit for bit the recomputing adjoint's results, and the stored new phi bit
for bit phasefield_step's. The tiled form of the non-uniform adjoint (three tile shapes, fixed
and per-launch chunks) bit for bit its one-thread-per-cell form.
"""
import numpy as np
import pytest
import torch

import oracle
import pf_fixtures as fx

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
SCH = {"euler": 1, "rk2": 2, "rk3": 3, "rk4": 4}


def rel_linf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def nu_case(seed, shape, ratio=2.5, smooth=False, walls=(False, False, False)):
    """Drops on a stretched mesh with a solenoidal face velocity (largest component 1); on a
    walled axis the velocity through the wall faces is zero."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    if smooth:
        h = [fx.smooth_widths(n, 1.0, ratio, 0.7 * a) for a, n in enumerate((nx, ny, nz))]
    else:
        h = [fx.random_widths(rng, n, 1.0, ratio) for n in (nx, ny, nz)]
    A = [rng.standard_normal(shape) for _ in range(3)]
    if nz == 1:
        A[0][:] = 0.0
        A[1][:] = 0.0
    # zero potential on the edges that bound a wall face keeps the wall faces closed
    if walls[0]:
        A[1][:, :, 0] = 0.0
        A[2][:, :, 0] = 0.0
    if walls[1]:
        A[0][:, 0, :] = 0.0
        A[2][:, 0, :] = 0.0
    if walls[2]:
        A[0][0] = 0.0
        A[1][0] = 0.0
    U, V, W = fx.edge_curl_nu(*A, *h)
    s = 1.0 / fx.max_face_speed(U, V, W)
    xc, yc = fx.cell_centres(h[0]), fx.cell_centres(h[1])
    zc = fx.cell_centres(h[2]) if nz > 1 else np.array([0.5])
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    r = np.sqrt((X - 0.45) ** 2 + (Y - 0.5) ** 2 + ((Z - 0.55) ** 2 if nz > 1 else 0.0))
    hmax = max(float(np.max(a)) for a in h[:2 if nz == 1 else 3])
    phi = 0.5 * (1.0 + np.tanh((0.3 - r) / (2.0 * hmax)))
    return phi, U * s, V * s, W * s, h, hmax


def stable_dt(h, eps, eps_mode, dxref, gamma=1.0, nz=2):
    """0.08 of the smallest width (advection) and at most 0.1 h_min^2 / (gamma eps_max), the
    explicit diffusion limit on the finest axis with the largest eps of the mesh (local eps
    grows with the coarsest width of a cell)."""
    axes = h if nz > 1 else h[:2]
    hmin = min(float(np.min(a)) for a in axes)
    hmax = max(float(np.max(a)) for a in axes)
    eps_max = eps * hmax / dxref if eps_mode == 1 else eps
    return min(0.08 * hmin, 0.1 * hmin * hmin / (gamma * eps_max))


def run(pf, phi, U, V, W, h, *, dtype, dx, eps, gamma, dt, nsteps, scheme="rk4", eps_mode=0,
        walls=(False, False, False), vel_mode=0, vel_T=1.0, t0=0.0, stream=True, variant=-1):
    nz, ny, nx = phi.shape
    tdt = torch.float64 if dtype == "f64" else torch.float32
    s = pf.Solver((nx, ny, nz), dx, eps, gamma, dt, dtype=dtype, scheme=scheme, walls=walls,
                  vel_mode=vel_mode, vel_T=vel_T, variant=variant)
    if h is not None:
        s.set_spacing(*h, eps_mode=eps_mode)
    g = [torch.tensor(a, dtype=tdt, device="cuda") for a in (phi, U, V, W)]
    st = torch.cuda.Stream() if stream else None
    if st is not None:
        with torch.cuda.stream(st):
            s.step(*g, t0=t0, nsteps=nsteps, stream=st)
    else:
        s.step(*g, t0=t0, nsteps=nsteps)
    torch.cuda.synchronize()
    out = g[0].cpu().numpy().astype(np.float64)
    return out, s


CASES = [
    # dtype, shape, walls, eps_mode, scheme, smooth
    ("f64", (12, 20, 70), (False, False, False), 0, "rk4", False),
    ("f64", (12, 20, 70), (False, False, False), 1, "rk4", True),
    ("f32", (12, 20, 70), (False, False, False), 1, "rk4", False),
    ("f64", (10, 16, 128), (False, False, False), 1, "rk4", False),   # 64-wide tiles
    ("f64", (1, 36, 50), (False, False, False), 1, "rk4", False),     # one plane
    ("f32", (1, 36, 50), (True, True, False), 0, "rk4", True),
    ("f64", (14, 18, 40), (True, False, True), 1, "rk4", False),
    ("f64", (14, 18, 40), (False, True, False), 0, "rk3", False),
    ("f64", (14, 18, 40), (False, False, False), 1, "rk2", False),
    ("f64", (14, 18, 40), (True, True, True), 1, "euler", False),
    ("f32", (20, 9, 33), (False, False, False), 0, "rk3", False),
]


@pytest.mark.parametrize("dtype,shape,walls,eps_mode,scheme,smooth", CASES)
def test_nonuniform_matches_oracle(lib, dtype, shape, walls, eps_mode, scheme, smooth):
    phi, U, V, W, h, hmax = nu_case(sum(shape), shape, smooth=smooth, walls=walls)
    if dtype == "f32":
        phi, U, V, W = (a.astype(np.float32).astype(np.float64) for a in (phi, U, V, W))
    dxref = 1.0 / max(shape)
    eps = 1.1 * (dxref if eps_mode else hmax)
    kw = dict(dx=dxref, eps=eps, gamma=1.0, dt=stable_dt(h, eps, eps_mode, dxref, nz=shape[0]),
              nsteps=7)
    print("case", dtype, shape, walls, eps_mode, scheme, flush=True)
    ref = oracle.step_nu(phi, U, V, W, hx=h[0], hy=h[1], hz=h[2], scheme=SCH[scheme],
                         eps_mode=eps_mode, walls=walls, fp32=dtype == "f32", **kw)
    got, s = run(lib, phi, U, V, W, h, dtype=dtype, scheme=scheme, eps_mode=eps_mode,
                 walls=walls, **kw)
    s.close()
    err = rel_linf(got, ref)
    print("error", err, flush=True)
    assert err <= (TOL64 if dtype == "f64" else TOL32), err
    assert np.abs(got - phi).max() > 1e-3  # the run moved the field


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_nonuniform_time_varying_velocity_and_graph_replay(lib, dtype):
    """cos(pi t/T) velocity (whole-loop graph of 20 steps from t0) and steady velocity replayed
    from the 8-step graphs (20 steps), each against the oracle and against launches on the NULL
    stream (no graph)."""
    shape = (10, 24, 36)
    phi, U, V, W, h, hmax = nu_case(3, shape)
    if dtype == "f32":
        phi, U, V, W = (a.astype(np.float32).astype(np.float64) for a in (phi, U, V, W))
    kw = dict(dx=1.0 / 36, eps=1.1 / 36, gamma=1.0, dt=stable_dt(h, 1.1 / 36, 1, 1.0 / 36),
              nsteps=20)
    for vel_mode in (1, 0):
        ref = oracle.step_nu(phi, U, V, W, hx=h[0], hy=h[1], hz=h[2], eps_mode=1, vel_mode=vel_mode,
                             vel_T=0.2, t0=0.05, fp32=dtype == "f32", **kw)
        got, s1 = run(lib, phi, U, V, W, h, dtype=dtype, eps_mode=1, vel_mode=vel_mode, vel_T=0.2,
                      t0=0.05, **kw)
        eager, s2 = run(lib, phi, U, V, W, h, dtype=dtype, eps_mode=1, vel_mode=vel_mode,
                        vel_T=0.2, t0=0.05, stream=False, **kw)
        s1.close()
        s2.close()
        assert np.array_equal(got, eager)
        assert rel_linf(got, ref) <= (TOL64 if dtype == "f64" else TOL32)


def test_equal_widths_agree_with_the_uniform_kernels(lib):
    """Equal widths through the non-uniform form agree with the uniform per-stage and fused
    kernels to rounding; clearing the widths returns the handle to the uniform kernels
    bit for bit."""
    pf = lib
    shape = (12, 20, 40)
    phi, U, V, W, _, _ = nu_case(5, shape, ratio=1.0)
    dx = 1.0 / 40
    U, V, W = fx.random_edge_faces(np.random.default_rng(5), shape, dx)
    s = 1.0 / fx.max_face_speed(U, V, W)
    U, V, W = U * s, V * s, W * s
    h = [np.full(n, dx) for n in (40, 20, 12)]
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, nsteps=6)
    uni, s0 = run(pf, phi, U, V, W, None, dtype="f64", **kw)
    s0.close()
    nu, s1 = run(pf, phi, U, V, W, h, dtype="f64", eps_mode=1, **kw)
    assert rel_linf(nu, uni) <= 1e-13
    s1.set_spacing(None, None, None)
    g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi, U, V, W)]
    s1.step(*g, nsteps=6)
    torch.cuda.synchronize()
    assert np.array_equal(g[0].cpu().numpy(), uni)
    s1.close()


def test_nonuniform_mass_and_refusals(lib):
    pf = lib
    shape = (16, 18, 20)
    phi, U, V, W, h, hmax = nu_case(9, shape, walls=(True, False, False))
    nz, ny, nx = shape
    s = pf.Solver((nx, ny, nz), 1.0 / 20, 1.1 / 20, 1.0, stable_dt(h, 1.1 / 20, 1, 1.0 / 20),
                  dtype="f64", walls=(True, False, False))
    s.set_spacing(*h, eps_mode=1)
    g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi, U, V, W)]
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        m0 = s.reduce(g[0], stream=st)
        s.step(*g, nsteps=40, stream=st)
        m1 = s.reduce(g[0], stream=st)
    want = oracle.reduce_nu(phi, hx=h[0], hy=h[1], hz=h[2])
    assert abs(m0[0] - want[0]) <= 1e-13 * want[0] and m0[1:] == want[1:]
    assert abs(m1[0] - m0[0]) <= 1e-13 * m0[0]
    with pytest.raises(pf.PhaseFieldError) as ei:
        s.autotune(reps=1)
    assert ei.value.status == pf.PF_ERR_UNSUPPORTED
    bad = [np.array(h[0]), h[1], h[2]]
    bad[0][3] = 0.0
    with pytest.raises(pf.PhaseFieldError) as ei:
        s.set_spacing(*bad)
    assert ei.value.status == pf.PF_ERR_INVALID
    with pytest.raises(pf.PhaseFieldError):
        s.set_spacing(*h, eps_mode=2)
    s.close()


F, T = False, True
ADJ_CASES = [
    # dtype, shape (nz, ny, nx), walls (x, y, z), eps_mode, scheme, vel_mode, variant (None: default)
    ("f64", (12, 20, 70), (F, F, F), 0, "rk4", 0, None),
    ("f64", (12, 20, 70), (F, F, F), 1, "rk4", 1, "fused_32x16"),  # per-stage on a fused handle
    ("f64", (14, 18, 40), (T, F, T), 1, "rk4", 1, None),
    ("f64", (14, 18, 40), (F, T, F), 0, "rk3", 1, None),
    ("f64", (14, 18, 40), (T, T, T), 1, "rk2", 0, None),
    ("f64", (9, 11, 7), (F, F, T), 1, "euler", 1, None),
    ("f64", (1, 36, 50), (T, F, F), 1, "rk4", 1, None),            # one plane
    ("f64", (10, 16, 130), (F, F, F), 1, "rk3", 0, "global"),
    ("f32", (12, 20, 70), (F, F, F), 1, "rk4", 1, None),
    ("f32", (14, 18, 40), (T, F, T), 0, "rk2", 0, None),
]


@pytest.mark.parametrize("dtype,shape,walls,eps_mode,scheme,vel_mode,vname", ADJ_CASES)
def test_nonuniform_adjoint_matches_oracle(lib, dtype, shape, walls, eps_mode, scheme, vel_mode,
                                           vname):
    pf = lib
    phi, U, V, W, h, hmax = nu_case(sum(shape) + 11, shape, walls=walls)
    if dtype == "f32":
        phi, U, V, W = (a.astype(np.float32).astype(np.float64) for a in (phi, U, V, W))
    nz, ny, nx = shape
    rng = np.random.default_rng(sum(shape))
    lam = rng.standard_normal(shape)
    dxref = 1.0 / max(shape)
    eps = 1.1 * (dxref if eps_mode else hmax)
    t, vel_T = 0.1, 0.7
    kw = dict(dx=dxref, eps=eps, gamma=1.2, dt=stable_dt(h, eps, eps_mode, dxref, 1.2, nz),
              delta=0.05 / dxref)
    print("case", dtype, shape, walls, eps_mode, scheme, vel_mode, vname, flush=True)
    ref = oracle.adjoint_step_nu(phi, U, V, W, lam, hx=h[0], hy=h[1], hz=h[2], t=t,
                                 scheme=SCH[scheme], vel_mode=vel_mode, vel_T=vel_T,
                                 eps_mode=eps_mode, walls=walls, **kw)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    kd = pf.PF_F64 if dtype == "f64" else pf.PF_F32
    names = [pf.phasefield_variant_name(kd, k) for k in range(pf.phasefield_variant_count(kd))]
    s = pf.Solver((nx, ny, nz), scheme=scheme, walls=walls, dtype=dtype, vel_mode=vel_mode,
                  vel_T=vel_T, variant=-1 if vname is None else names.index(vname), **kw)
    s.set_spacing(*h, eps_mode=eps_mode)
    g = [torch.tensor(a, dtype=tdt, device="cuda") for a in (phi, U, V, W)]
    L = torch.tensor(lam, dtype=tdt, device="cuda")
    grads = [torch.zeros_like(L) for _ in range(3)]
    s.adjoint_step(*g, t, L, *grads)
    # the same step keeping its stage inputs, and the adjoint reading them
    ns = s.stage_count
    ys = [torch.full_like(g[0], float("nan")) for _ in range(ns)]
    phi1 = torch.full_like(g[0], float("nan"))
    s.step_stages(g[0], *g[1:], t, *ys, phi_next=phi1)
    phi_ref = g[0].clone()
    s.step(phi_ref, *g[1:], t0=t, nsteps=1)
    L1 = torch.tensor(lam, dtype=tdt, device="cuda")
    grads1 = [torch.zeros_like(L) for _ in range(3)]
    s.adjoint_step_stages(g[0], ys, *g[1:], t, L1, *grads1)
    torch.cuda.synchronize()
    s.close()
    tol = TOL64 if dtype == "f64" else 1e-3
    for k, (got, want) in enumerate(zip([L] + grads, ref)):
        err = rel_linf(got.cpu().numpy().astype(np.float64), want)
        print("output", k, "error", err, flush=True)
        assert err <= tol, (k, err)
    for a, w in enumerate(walls):  # the wall faces' velocity entries stay untouched
        if w:
            sl = [slice(None)] * 3
            sl[2 - a] = 0
            assert not grads[a][tuple(sl)].any()
    assert torch.equal(phi1, phi_ref)
    for x, y in zip([L] + grads, [L1] + grads1):
        assert torch.equal(x, y)


@pytest.mark.parametrize("dtype,walls,eps_mode,scheme", [("f64", (F, F, F), 1, "rk4"),
                                                         ("f64", (T, F, T), 0, "rk4"),
                                                         ("f32", (F, T, F), 1, "rk4"),
                                                         ("f64", (F, F, F), 1, "rk3")])
def test_nonuniform_adjoint_tiled_equals_plain(lib, dtype, walls, eps_mode, scheme):
    """On a ragged grid (13 x 21 x 70): the adjoint through the tiled NU kernel (64x8 with
    16-plane chunks, 64x4 with 32, 32x4 with per-launch chunks, the default handle) and through
    the large-array variant (which takes the one-thread-per-cell form) bit for bit the
    one-thread-per-cell form."""
    pf = lib
    shape = (13, 21, 70)
    phi, U, V, W, h, hmax = nu_case(77, shape, walls=walls)
    nz, ny, nx = shape
    lam = np.random.default_rng(7).standard_normal(shape)
    dxref = 1.0 / 70
    eps = 1.1 * (dxref if eps_mode else hmax)
    kw = dict(dx=dxref, eps=eps, gamma=1.2, dt=stable_dt(h, eps, eps_mode, dxref, 1.2, nz),
              delta=0.05 / dxref)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    kd = pf.PF_F64 if dtype == "f64" else pf.PF_F32
    names = [pf.phasefield_variant_name(kd, k) for k in range(pf.phasefield_variant_count(kd))]
    outs = []
    for vname in ("global", "tiled_64x8x16", "tiled_64x4x32", "tiled_32x4", "tiled_64x8x16_big",
                  None):
        print("case", dtype, walls, eps_mode, scheme, vname, flush=True)
        s = pf.Solver((nx, ny, nz), scheme=scheme, walls=walls, dtype=dtype, vel_mode=1,
                      vel_T=0.6, variant=-1 if vname is None else names.index(vname), **kw)
        s.set_spacing(*h, eps_mode=eps_mode)
        g = [torch.tensor(a, dtype=tdt, device="cuda") for a in (phi, U, V, W)]
        L = torch.tensor(lam, dtype=tdt, device="cuda")
        grads = [torch.zeros_like(L) for _ in range(3)]
        s.adjoint_step(*g, 0.05, L, *grads)
        torch.cuda.synchronize()
        s.close()
        outs.append([L] + grads)
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert torch.equal(x, y)
    assert float(outs[0][0].abs().max()) > 0.0 and float(outs[0][1].abs().max()) > 0.0


@pytest.mark.parametrize("cache,keep_all", [(True, False), (False, False), (None, True)])
def test_nonuniform_rollout_matches_oracle_chain(lib, cache, keep_all):
    """The checkpointed Rollout on a stretched 24^3 mesh (widths varying 2x along every axis,
    local eps; 14 steps, checkpoint 5: segments 5, 5, 4; cos-reversed velocity from 8 modes)
    with stage caching, recomputing stages, and keeping every step: dL/dphi0 and dL/dcoeffs
    against the oracle's chain of non-uniform steps and adjoint steps and the coefficient
    transpose (FP64, 1e-11)."""
    pf = lib
    n, nsteps, ckpt, vel_T = 24, 14, 5, 0.05
    c = fx.adjoint_case(n)
    th, co = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in c.modes)
    p0 = pf.make_params(c.shape, c.dx, c.eps, 1.0, 1.0)
    u, v, w = pf.velocity_from_coeffs(p0, th, co)
    torch.cuda.synchronize()
    fx.set_speed(c, max(float(x.abs().max()) for x in (u, v, w)))
    h = [fx.smooth_widths(n, 1.0, 2.0, 0.9 * a) for a in range(3)]
    hmin = min(float(np.min(a)) for a in h)
    dt = min(0.5 * c.dt * hmin / c.dx, stable_dt(h, c.eps, 1, c.dx, c.gamma))
    s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, dt, delta=c.delta, vel_mode=1, vel_T=vel_T)
    s.set_spacing(*h, eps_mode=1)
    print("case", cache, keep_all, "dt", dt, flush=True)
    phi0 = torch.tensor(c.phi0, dtype=torch.float64, device="cuda").requires_grad_(True)
    cc = torch.tensor(c.modes[1], dtype=torch.float64, device="cuda").requires_grad_(True)
    phiT = pf.Rollout.apply(phi0, cc, s, th, nsteps, ckpt, 0.0, cache, keep_all)
    target = torch.tensor(c.extra["target"], dtype=torch.float64, device="cuda")
    L = 0.5 * ((phiT - target) ** 2).sum()
    L.backward()
    torch.cuda.synchronize()
    s.close()
    gphi, gco = phi0.grad.cpu().numpy(), cc.grad.cpu().numpy()
    U, V, W = oracle.velocity_from_coeffs(c.shape, dx=c.dx, phases=c.modes[0], coeffs=c.modes[1])
    kw = dict(hx=h[0], hy=h[1], hz=h[2], dx=c.dx, eps=c.eps, gamma=c.gamma, dt=dt,
              delta=c.delta, vel_mode=1, vel_T=vel_T, eps_mode=1)
    states = [c.phi0]
    for k in range(nsteps):
        states.append(oracle.step_nu(states[-1], U, V, W, t0=k * dt, **kw))
    lam = states[-1] - c.extra["target"]
    gu, gv, gw = (np.zeros(c.shape) for _ in range(3))
    for k in reversed(range(nsteps)):
        lam, a, b, d = oracle.adjoint_step_nu(states[k], U, V, W, lam, t=k * dt, **kw)
        gu += a
        gv += b
        gw += d
    cg = oracle.velocity_from_coeffs_T(c.shape, dx=c.dx, phases=c.modes[0], Ubar=gu, Vbar=gv,
                                       Wbar=gw)
    e_phi, e_co = rel_linf(gphi, lam), rel_linf(gco, cg)
    print("rollout vs oracle chain: dL/dphi0", e_phi, "dL/dcoeffs", e_co, flush=True)
    assert e_phi <= 1e-11 and e_co <= 1e-11
    assert np.abs(gphi).max() > 0.0 and np.abs(gco).max() > 0.0
