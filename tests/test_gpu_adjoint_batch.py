"""GPU parity of the discrete adjoint, velocity synthesis, autograd rollout and batched driver.

Bars: FP64 adjoint and synthesis <= 1e-12 relative L-inf against the oracle; the rollout
gradient against central finite differences of the GPU forward; FP32 gradients against the
FP64 oracle at 1e-3; batched instances bit-identical to their single solves.
"""
import numpy as np
import pytest
import torch

import oracle
import pf_fixtures as fx

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_linf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def adj_case(seed, shape):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    dx = 1.0 / max(shape)
    phi = fx.drops_ic(shape, dx, [(0.5 * nx * dx, 0.5 * ny * dx, 0.5 * nz * dx)],
                      [0.3 * max(shape) * dx], 1.5 * dx) * 0.8 + 0.2 * rng.uniform(size=shape)
    U, V, W = fx.random_edge_faces(rng, shape, dx)
    s = 1.0 / fx.max_face_speed(U, V, W)
    lam = rng.standard_normal(shape)
    return rng, phi, U * s, V * s, W * s, lam, dx


@pytest.mark.parametrize("scheme,shape", [("rk4", (12, 10, 14)), ("rk4", (1, 20, 18)),
                                          ("euler", (9, 11, 7)), ("rk4", (20, 16, 70)),
                                          ("rk2", (12, 10, 14)), ("rk2", (1, 20, 18)),
                                          ("rk3", (12, 10, 14)), ("rk3", (1, 20, 18))])
def test_adjoint_step_fp64_matches_oracle(lib, scheme, shape):
    pf = lib
    rng, phi, U, V, W, lam, dx = adj_case(1, shape)
    kw = dict(dx=dx, eps=dx, gamma=1.2, dt=0.12 * dx, delta=0.05 / dx, vel_mode=1, vel_T=0.8)
    ref = oracle.adjoint_step(phi, U, V, W, lam, t=0.1,
                              scheme={"rk4": 4, "rk3": 3, "rk2": 2, "euler": 1}[scheme], **kw)
    nz, ny, nx = shape
    s = pf.Solver((nx, ny, nz), scheme=scheme, **kw)
    g = [dev(a) for a in (phi, U, V, W)]
    L = dev(lam)
    grads = [torch.zeros_like(g[0]) for _ in range(3)]
    s.adjoint_step(*g, 0.1, L, *grads)
    torch.cuda.synchronize()
    assert rel_linf(host(L), ref[0]) <= 1e-12, rel_linf(host(L), ref[0])
    for a, b in zip(grads, ref[1:]):
        assert rel_linf(host(a), b) <= 1e-12, rel_linf(host(a), b)
    # NULL gradients skip the velocity part and leave lam unchanged
    L2 = dev(lam)
    s.adjoint_step(*g, 0.1, L2)
    torch.cuda.synchronize()
    assert torch.equal(L2, L)
    # the gradients accumulate onto what the arrays hold; a NULL one is skipped on its own
    g0 = [rng.standard_normal(shape) * np.abs(b).max() for b in ref[1:]]
    acc = [dev(x) for x in g0]
    L3 = dev(lam)
    s.adjoint_step(*g, 0.1, L3, acc[0], None, acc[2])
    torch.cuda.synchronize()
    assert torch.equal(L3, L)
    assert torch.equal(acc[1], dev(g0[1]))
    for ax in (0, 2):
        assert rel_linf(host(acc[ax]) - g0[ax], ref[1 + ax]) <= 1e-12
    s.close()


@pytest.mark.parametrize("dtype,shape,scheme", [("f64", (20, 16, 70), "rk4"), ("f32", (33, 9, 65), "rk4"),
                                                ("f64", (1, 12, 5), "rk4"), ("f64", (20, 16, 70), "rk2"),
                                                ("f64", (20, 16, 70), "rk3"), ("f32", (70, 37, 130), "rk4"),
                                                ("f64", (45, 20, 66), "rk4"), ("f32", (3, 40, 64), "rk4")])
def test_tiled_adjoint_bitwise_equals_plain(lib, dtype, shape, scheme):
    """The tiled adjoint stage kernel and the one-thread-per-cell kernel (paired with the
    'global' forward variant) give bit-identical lam and velocity gradients, for every adjoint
    tile shape and chunk length (lent by the per-stage forward variant of that shape; none in
    its name: chosen per launch), the large-array addressing form (a '_big' variant) and the
    RK4 reverse stages run two per launch (64x8 and 32x16 tiles lent by fused variants or chosen
    for the grid, 32- and 64-plane chunks or chunks chosen per launch, ragged tiles, several
    chunks)."""
    pf = lib
    rng, phi, U, V, W, lam, dx = adj_case(4, shape)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    kd = pf.PF_F64 if dtype == "f64" else pf.PF_F32
    names = [pf.phasefield_variant_name(kd, v) for v in range(pf.phasefield_variant_count(kd))]
    kw = dict(dx=dx, eps=dx, gamma=1.2, dt=0.12 * dx, delta=0.05 / dx, dtype=dtype, scheme=scheme)
    nz, ny, nx = shape
    # (variant, adjoint form): form 1 runs the RK4 reverse stages two per launch, 0 one per
    # launch, -1 lets the handle choose (one per launch on these small grids)
    picks = [("global", -1), ("tiled_64x8x64", -1), ("tiled_64x8x16", -1), ("tiled_64x4x16", -1),
             ("tiled_32x4x16", -1), ("tiled_64x8x16_big", -1), ("fused_32x16x32", 0),
             ("tiled_64x4", -1), ("tiled_32x4", -1), ("fused_64x8", -1), ("fused_64x8", 1),
             ("fused_64x8x32", 1), ("fused_32x16x64", 1), ("fused_32x16", 1), ("tiled_64x8", 1)]
    res = []
    for nm, form in picks:
        s = pf.Solver((nx, ny, nz), variant=names.index(nm), **kw)
        s.set_adjoint_form(form)
        g = [dev(a, tdt) for a in (phi, U, V, W)]
        L = dev(lam, tdt)
        grads = [torch.zeros_like(g[0]) for _ in range(3)]
        s.adjoint_step(*g, 0.0, L, *grads)
        torch.cuda.synchronize()
        res.append([L] + grads)
        s.close()
    for pick, other in zip(picks[1:], res[1:]):
        for a, b in zip(res[0], other):
            assert torch.equal(a, b), pick
    s = pf.Solver((nx, ny, nz), **kw)
    with pytest.raises(pf.PhaseFieldError):
        s.set_adjoint_form(2)
    s.close()


def test_adjoint_step_fp32_close_to_fp64_oracle(lib):
    pf = lib
    rng, phi, U, V, W, lam, dx = adj_case(2, (16, 16, 16))
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, delta=0.05 / dx)
    ref = oracle.adjoint_step(phi, U, V, W, lam, **kw)
    s = pf.Solver((16, 16, 16), dtype="f32", **kw)
    g = [dev(a, torch.float32) for a in (phi, U, V, W)]
    L = dev(lam, torch.float32)
    grads = [torch.zeros_like(g[0]) for _ in range(3)]
    s.adjoint_step(*g, 0.0, L, *grads)
    torch.cuda.synchronize()
    assert rel_linf(host(L), ref[0]) <= 1e-3
    for a, b in zip(grads, ref[1:]):
        assert rel_linf(host(a), b) <= 1e-3
    s.close()


def _flat_region_case():
    shape = (20, 18, 24)
    nz, ny, nx = shape
    dx = 1.0 / nx
    phi = fx.drops_ic(shape, dx, [(0.5, 0.5, 0.5)], [0.3], dx)
    phi = np.where(phi < 0.02, 0.0, np.where(phi > 0.98, 1.0, phi))
    rng = np.random.default_rng(6)
    U, V, W = fx.random_edge_faces(rng, shape, dx)
    sc = 1.0 / fx.max_face_speed(U, V, W)
    lam = rng.standard_normal(shape)
    return shape, dx, (phi, U * sc, V * sc, W * sc, lam)


@pytest.mark.parametrize("dtype,scheme", [("f64", "rk4"), ("f32", "euler"), ("f32", "rk4")])
def test_adjoint_step_delta0_flat_regions(lib, dtype, scheme):
    """delta = 0 (the plain unit normal, the default) on a field with exactly flat regions
    (phi = 0 and phi = 1 over whole blocks, where g = 0) and clipped tanh transitions: every
    output is finite (the FP32 transpose takes r = 0 where |g|^2 is below the smallest normal
    float, as FP64 does at g = 0), and it equals the oracle's adjoint (zero normal and zero
    derivative where |g| = 0) wherever the comparison is well posed: FP64 at 1e-12; FP32 storage
    for Euler, whose only stage input is phi itself, at the FP32 gradient bar 1e-3 against the
    oracle on the stored values. With delta = 0 the RK4 transpose is not well posed in FP32:
    next to a flat block the recomputed stage inputs depart from 1 by ~1e-12, which FP32 rounds
    back to exactly 1 (g = 0, no sharpening term) while FP64 resolves a unit normal there whose
    transpose contributes O(1) (the oracle itself moves by 1 % when phi is perturbed by 1e-16).
    There only finiteness and the magnitude (within 2 x the oracle's largest value) are
    checked."""
    pf = lib
    shape, dx, arrs = _flat_region_case()
    nz, ny, nx = shape
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        arrs = tuple(a.astype(np.float32).astype(np.float64) for a in arrs)
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx)
    ref = oracle.adjoint_step(*arrs, scheme={"rk4": 4, "euler": 1}[scheme], **kw)
    s = pf.Solver((nx, ny, nz), dtype=dtype, scheme=scheme, **kw)
    g = [dev(a, tdt) for a in arrs[:4]]
    L = dev(arrs[4], tdt)
    grads = [torch.zeros_like(L) for _ in range(3)]
    s.adjoint_step(*g, 0.0, L, *grads)
    torch.cuda.synchronize()
    s.close()
    tol = 1e-12 if dtype == "f64" else 1e-3
    for k, (a, b) in enumerate(zip([L] + grads, ref)):
        got = host(a)
        assert np.isfinite(got).all(), k
        err = rel_linf(got, b)
        print(dtype, scheme, "output", k, "relative L-inf vs oracle", err, flush=True)
        if dtype == "f32" and scheme == "rk4":
            assert np.abs(got).max() <= 2 * np.abs(b).max(), k
        else:
            assert err <= tol, (k, err)


@pytest.mark.parametrize("shape,M", [((12, 10, 14), 3), ((32, 32, 32), 8), ((1, 16, 20), 4),
                                     ((9, 5, 150), 12), ((6, 7, 70), 20), ((3, 2, 64), 16),
                                     ((9, 6, 70), 64)])
def test_velocity_synthesis_matches_oracle(lib, shape, M):
    """Synthesis (plane blocks of the curl, ragged and shorter than a block) and transpose (runs
    of 64 x-positions, rows wider and narrower than a run, mode chunks of 8 and 16, padded and
    whole, up to the largest mode count the library takes, 64) against the oracle."""
    pf = lib
    rng = np.random.default_rng(3)
    nz, ny, nx = shape
    dx = 1.0 / nx
    th = rng.uniform(0, 2 * np.pi, size=(3, M))
    c = rng.standard_normal((M, M, M, 3))
    ref = oracle.velocity_from_coeffs(shape, dx=dx, phases=th, coeffs=c)
    p = pf.make_params((nx, ny, nz), dx, dx, 1.0, 0.1 * dx)
    got = pf.velocity_from_coeffs(p, dev(th), dev(c))
    for a, b in zip(got, ref):
        assert rel_linf(host(a), b) <= 1e-12
    p32 = pf.make_params((nx, ny, nz), dx, dx, 1.0, 0.1 * dx, dtype="f32")
    got32 = pf.velocity_from_coeffs(p32, dev(th), dev(c))
    for a, b in zip(got32, ref):
        assert np.abs(host(a) - b).max() <= 2 * np.spacing(np.float32(np.abs(b).max()))
    # transpose
    gb = [rng.standard_normal(shape) for _ in range(3)]
    cref = oracle.velocity_from_coeffs_T(shape, dx=dx, phases=th, Ubar=gb[0], Vbar=gb[1], Wbar=gb[2])
    cg = pf.velocity_coeffs_grad(p, dev(th), *[dev(x) for x in gb])
    assert rel_linf(host(cg), cref) <= 1e-12


def _rollout_setup(pf, n=16, nsteps=12, dtype="f64", seed=5):
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    th, c = fx.random_modes(rng, 3, n)
    U, V, W = oracle.velocity_from_coeffs((n, n, n), dx=dx, phases=th, coeffs=c)
    umax = fx.max_face_speed(U, V, W)
    phi0 = fx.drops_ic((n, n, n), dx, [(0.4, 0.45, 0.5)], [0.25], dx)
    target = fx.drops_ic((n, n, n), dx, [(0.5, 0.5, 0.5)], [0.25], dx)
    dt = fx.rk4_dt_3d(dx, umax, dx)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    s = pf.Solver((n, n, n), dx, dx, umax, dt, dtype=dtype, delta=1e-3 / dx)
    return s, th, c, phi0, target, tdt, (U, V, W, umax, dt, dx)


def _loss(pf, s, th, coeffs, phi0, target, nsteps, ckpt):
    phiT = pf.Rollout.apply(phi0, coeffs, s, th, nsteps, ckpt, 0.0)
    return 0.5 * ((phiT - target) ** 2).sum()


def test_rollout_gradient_matches_oracle_and_fd(lib):
    """dL/dphi0 and dL/dcoeffs of L = 0.5 |phi_T - target|^2 through Rollout: against the
    oracle's adjoint chain (1e-11), fourth-order central differences of the GPU forward in 6 random
    directions (1e-7), and identical for checkpoint intervals 1, 5 and 12."""
    pf = lib
    nsteps = 12
    s, th, c, phi0, target, tdt, (U, V, W, umax, dt, dx) = _rollout_setup(pf, nsteps=nsteps)
    thd, tg = dev(th), dev(target)
    grads = {}
    for ck in (1, 5, 12):
        p0 = dev(phi0).requires_grad_(True)
        cc = dev(c).requires_grad_(True)
        L = _loss(pf, s, thd, cc, p0, tg, nsteps, ck)
        L.backward()
        grads[ck] = (host(p0.grad), host(cc.grad))
    for ck in (5, 12):
        assert np.array_equal(grads[ck][0], grads[1][0]) and np.array_equal(grads[ck][1], grads[1][1])
    # oracle chain
    states = [phi0]
    kw = dict(dx=dx, eps=dx, gamma=umax, dt=dt, delta=1e-3 / dx)
    for n in range(nsteps):
        states.append(oracle.step(states[-1], U, V, W, **kw))
    lam = states[-1] - target
    gu, gv, gw = (np.zeros_like(U) for _ in range(3))
    for n in reversed(range(nsteps)):
        lam, a, b, d = oracle.adjoint_step(states[n], U, V, W, lam, t=n * dt, **kw)
        gu += a
        gv += b
        gw += d
    cg = oracle.velocity_from_coeffs_T(phi0.shape, dx=dx, phases=th, Ubar=gu, Vbar=gv, Wbar=gw)
    assert rel_linf(grads[1][0], lam) <= 1e-11
    assert rel_linf(grads[1][1], cg) <= 1e-11
    # finite differences of the GPU forward
    rng = np.random.default_rng(9)
    with torch.no_grad():
        for d in range(6):
            v0 = rng.standard_normal(phi0.shape) if d % 2 == 0 else np.zeros(phi0.shape)
            vc = rng.standard_normal(c.shape) if d % 2 == 1 else np.zeros(c.shape)
            h = 1e-5

            def L_at(sgn):
                return float(_loss(pf, s, thd, dev(c + sgn * h * vc), dev(phi0 + sgn * h * v0),
                                   tg, nsteps, 5))

            # fourth-order central difference: the normal g/sqrt(|g|^2 + delta^2) has large
            # higher derivatives where |g| ~ delta, which the two-point formula does not resolve
            fd = (8 * (L_at(1) - L_at(-1)) - (L_at(2) - L_at(-2))) / (12 * h)
            an = float(np.sum(grads[1][0] * v0) + np.sum(grads[1][1] * vc))
            assert an == pytest.approx(fd, rel=1e-7), (d, an, fd)
    s.close()


def _batch_instances(sizes, seed=4):
    cases = []
    for i, n in enumerate(sizes):
        rng = np.random.default_rng(seed + i)
        nx, ny, nz = n
        dx = 1.0 / max(n)
        phi = fx.drops_ic((nz, ny, nx), dx, *fx.random_drops(rng, 3, 0.1, 0.25), dx)
        U, V, W = fx.random_edge_faces(rng, (nz, ny, nx), dx)
        s = 1.0 / fx.max_face_speed(U, V, W)
        cases.append((n, dx, phi, U * s, V * s, W * s))
    return cases


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("mode", ["default", "fused", "per-stage", "fused-persistent",
                                  "per-stage-persistent", "shape64", "shape64-persistent"])
def test_batch_bitwise_equals_single_solves(lib, dtype, mode):
    """Both batched modes (chosen through instance 0's variant), each in both launch forms (one
    workgroup per tile entry, or a persistent resident grid), and the fused sweeps on 64x8 tiles
    (set_shape), give every instance exactly its own single solve, over uneven, ragged and
    degenerate grids."""
    pf = lib
    sizes = [(32, 32, 32), (48, 40, 24), (17, 9, 33), (64, 64, 8), (5, 70, 3), (96, 1, 1),
             (40, 24, 130)]
    cases = _batch_instances(sizes)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    kd = pf.PF_F64 if dtype == "f64" else pf.PF_F32
    names = [pf.phasefield_variant_name(kd, v) for v in range(pf.phasefield_variant_count(kd))]
    pick = {"default": -1, "fused": names.index("fused_32x16x32"), "shape64": -1,
            "per-stage": names.index("tiled_64x8x16")}[mode.replace("-persistent", "")]
    params, singles = [], []
    for (n, dx, phi, U, V, W) in cases:
        params.append(pf.make_params(n, dx, dx, 1.0, fx.rk4_dt_3d(dx, 1.0, dx), dtype=dtype))
    params[0].variant = pick
    st = torch.cuda.Stream()
    bs = pf.BatchSolver(params)
    if mode.startswith("shape64"):
        bs.set_shape("fused_64x8")
    if mode.endswith("persistent"):
        bs.set_persistent(True)
    bt = [[dev(a, tdt) for a in cs[2:]] for cs in cases]
    with torch.cuda.stream(st):
        bs.step([b[0] for b in bt], [b[1] for b in bt], [b[2] for b in bt], [b[3] for b in bt],
                nsteps=19, stream=st)
    st.synchronize()
    for p, cs, b in zip(params, cases, bt):
        s = pf.Solver(tuple(p.n), p.dx, p.eps, p.gamma, p.dt, dtype=dtype)  # default variant
        g = [dev(a, tdt) for a in cs[2:]]
        s.step(*g, nsteps=19)
        torch.cuda.synchronize()
        assert torch.equal(g[0], b[0]), p.n[:]
        s.close()
    bs.close()


@pytest.mark.parametrize("dtype,zwall", [("f32", False), ("f64", False), ("f32", True)])
def test_batch_autotune(lib, dtype, zwall):
    """The batch autotuner times every tile shape in both launch forms on private fields, leaves
    the batch in the fastest combination (the minimum of the reported times) and the caller's
    fields untouched; the tuned batch then gives every instance its single solve bit for bit. A
    walled z axis keeps every shape (the fused sweeps take walls on every axis)."""
    pf = lib
    sizes = [(32, 32, 32), (48, 40, 24), (64, 64, 8), (17, 9, 33)]
    cases = _batch_instances(sizes, seed=41)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    walls = [(False, False, True) if (zwall and k == 1) else (False, False, False)
             for k in range(len(sizes))]
    params = [pf.make_params(n, dx, dx, 1.0, fx.rk4_dt_3d(dx, 1.0, dx), dtype=dtype, walls=wl)
              for (n, dx, *_r), wl in zip(cases, walls)]
    bs = pf.BatchSolver(params)
    bt = [[dev(a, tdt) for a in cs[2:]] for cs in cases]
    keep = [b[0].clone() for b in bt]
    st = torch.cuda.Stream()
    shape, persistent, times = bs.autotune(reps=1, stream=st)
    print(dtype, "zwall" if zwall else "", "autotune", shape, persistent, times, flush=True)
    assert all(torch.equal(b[0], k) for b, k in zip(bt, keep))  # caller data untouched
    assert len(times) == 6 and all(t > 0 for t in times.values())
    assert times[(shape, persistent)] == min(times.values())
    with torch.cuda.stream(st):
        bs.step(*zip(*bt), nsteps=11, stream=st)
    st.synchronize()
    bs.close()
    for p, cs, b, wl in zip(params, cases, bt, walls):
        s = pf.Solver(tuple(p.n), p.dx, p.eps, p.gamma, p.dt, dtype=dtype, walls=wl)
        g = [dev(a, tdt) for a in cs[2:]]
        s.step(*g, nsteps=11)
        torch.cuda.synchronize()
        assert torch.equal(g[0], b[0]), p.n[:]
        s.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_matches_oracle(lib, dtype):
    """Batched instances of uneven sizes (32^3, 48^3 and a ragged 17 x 40 x 24 grid) after 12
    RK4 steps against the oracle (FP64 at 1e-12; FP32 storage at 1e-5 against the oracle's
    FP32-storage mode), in the default batched mode."""
    pf = lib
    sizes = [(32, 32, 32), (48, 48, 48), (17, 40, 24)]
    cases = _batch_instances(sizes, seed=21)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    nsteps = 12
    params = [pf.make_params(n, dx, dx, 1.0, fx.rk4_dt_3d(dx, 1.0, dx), dtype=dtype)
              for (n, dx, *_rest) in cases]
    bs = pf.BatchSolver(params)
    st = torch.cuda.Stream()
    ins = []
    for (n, dx, phi, U, V, W) in cases:
        arrs = (phi, U, V, W)
        if dtype == "f32":
            arrs = tuple(a.astype(np.float32).astype(np.float64) for a in arrs)
        ins.append(arrs)
    bt = [[dev(a, tdt) for a in arrs] for arrs in ins]
    with torch.cuda.stream(st):
        bs.step(*zip(*bt), nsteps=nsteps, stream=st)
    st.synchronize()
    bs.close()
    for (n, dx, *_rest), arrs, b in zip(cases, ins, bt):
        ref = oracle.step(*arrs, dx=dx, eps=dx, gamma=1.0, dt=fx.rk4_dt_3d(dx, 1.0, dx),
                          nsteps=nsteps, fp32=(dtype == "f32"))
        err = rel_linf(host(b[0]), ref)
        print(dtype, n, "batched vs oracle", err, flush=True)
        assert err <= (1e-12 if dtype == "f64" else 1e-5), (n, err)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("mode,zwall", [("default", False), ("fused", False), ("per-stage", False),
                                        ("fused-persistent", False), ("default", True),
                                        ("fused", True), ("per-stage", True)])
def test_batch_with_walls(lib, dtype, mode, zwall):
    """Instances with walls on x, on x and y, on y, and periodic ones, in one batch: every
    instance equals its own single solve bit for bit, and two of them match the oracle with the
    same walls (FP64 1e-12, FP32 1e-5 against the FP32-storage mode); with an instance walled on
    all three axes as well, in each mode."""
    pf = lib
    sizes = [(32, 32, 32), (48, 40, 24), (17, 9, 33), (40, 24, 30)]
    walls = [(True, False, False), (True, True, False), (False, False, False), (False, True, False)]
    if zwall:
        sizes.append((24, 20, 28))
        walls.append((True, True, True))
    cases = _batch_instances(sizes, seed=31)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    kd = pf.PF_F64 if dtype == "f64" else pf.PF_F32
    names = [pf.phasefield_variant_name(kd, v) for v in range(pf.phasefield_variant_count(kd))]
    pick = {"default": -1, "fused": names.index("fused_32x16x32"),
            "per-stage": names.index("tiled_64x8x16")}[mode.replace("-persistent", "")]
    params = []
    ins = []
    for (n, dx, phi, U, V, W), wl in zip(cases, walls):
        params.append(pf.make_params(n, dx, dx, 1.0, fx.rk4_dt_3d(dx, 1.0, dx), dtype=dtype, walls=wl))
        arrs = (phi, U, V, W)
        if dtype == "f32":
            arrs = tuple(a.astype(np.float32).astype(np.float64) for a in arrs)
        ins.append(arrs)
    params[0].variant = pick
    bs = pf.BatchSolver(params)
    if mode.endswith("persistent"):
        bs.set_persistent(True)
    bt = [[dev(a, tdt) for a in arrs] for arrs in ins]
    st = torch.cuda.Stream()
    nsteps = 11
    with torch.cuda.stream(st):
        bs.step(*zip(*bt), nsteps=nsteps, stream=st)
    st.synchronize()
    bs.close()
    for p, arrs, b, wl in zip(params, ins, bt, walls):
        s = pf.Solver(tuple(p.n), p.dx, p.eps, p.gamma, p.dt, dtype=dtype, walls=wl)
        g = [dev(a, tdt) for a in arrs]
        s.step(*g, nsteps=nsteps)
        torch.cuda.synchronize()
        assert torch.equal(g[0], b[0]), (p.n[:], wl)
        s.close()
    for k in (1, len(sizes) - 1):
        (n, dx, *_rest), arrs, b = cases[k], ins[k], bt[k]
        ref = oracle.step(*arrs, dx=dx, eps=dx, gamma=1.0, dt=fx.rk4_dt_3d(dx, 1.0, dx),
                          nsteps=nsteps, fp32=(dtype == "f32"), walls=walls[k])
        err = rel_linf(host(b[0]), ref)
        print(dtype, n, walls[k], "batched vs oracle", err, flush=True)
        assert err <= (1e-12 if dtype == "f64" else 1e-5), (n, err)


def test_batch_workload_full_size_bitwise(lib):
    """The batched workload at its full size (96 FP32 instances of 32^3-128^3, seeded drops and
    8-mode fields, 62.7M cells), in the configuration the benchmark times (default mode, steps
    replayed from a captured graph): after 10 steps every instance equals its own single solve
    bit for bit (single solves are checked against the oracle elsewhere)."""
    pf = lib
    cases = fx.batch_cases(count=96)
    st = torch.cuda.Stream()
    params, fields = [], []
    for c in cases:
        n = c.shape[0]
        phases, coeffs = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in c.modes)
        p0 = pf.make_params((n, n, n), c.dx, c.eps, 1.0, 1.0, dtype="f32")
        u, v, w = pf.velocity_from_coeffs(p0, phases, coeffs)
        torch.cuda.synchronize()
        fx.set_speed(c, max(float(t.abs().max()) for t in (u, v, w)))
        params.append(pf.make_params((n, n, n), c.dx, c.eps, c.gamma, c.dt, dtype="f32"))
        fields.append([torch.tensor(c.phi0, dtype=torch.float32, device="cuda"), u, v, w])
    bs = pf.BatchSolver(params)
    bf = [[f[0].clone(), f[1], f[2], f[3]] for f in fields]
    with torch.cuda.stream(st):
        bs.step(*zip(*bf), nsteps=10, stream=st)
    st.synchronize()
    bs.close()
    for p, f, b in zip(params, fields, bf):
        s = pf.Solver(tuple(p.n), p.dx, p.eps, p.gamma, p.dt, dtype="f32")
        phi = f[0].clone()
        s.step(phi, f[1], f[2], f[3], nsteps=10)
        torch.cuda.synchronize()
        s.close()
        assert torch.equal(phi, b[0]), tuple(p.n)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scheme", ["rk3", "rk2", "euler"])
def test_batch_other_schemes(lib, dtype, scheme):
    """RK3, RK2 and Euler batches (one scheme per batch; per-stage sweeps, one launch per stage,
    Euler then a batched copy) over uneven, ragged and walled grids: every instance bit for bit
    its own single solve after 11 steps (one graph replay and a remainder), in both launch forms;
    the fused shapes and mixed schemes refused; the periodic 32^3 instance against the oracle
    (FP64 1e-12; FP32 storage 1e-5 against the oracle's FP32-storage mode)."""
    pf = lib
    F, T = False, True
    sizes = [(32, 32, 32), (48, 40, 24), (17, 9, 33), (5, 70, 3)]
    walls = [(F, F, F), (T, F, F), (F, T, T), (F, F, F)]
    cases = _batch_instances(sizes, seed=61)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    nsteps = 11
    params = [pf.make_params(n, dx, dx, 1.0, 0.05 * dx, dtype=dtype, scheme=scheme, walls=wl)
              for (n, dx, *_r), wl in zip(cases, walls)]
    ins = []
    for (n, dx, phi, U, V, W) in cases:
        arrs = (phi, U, V, W)
        if dtype == "f32":
            arrs = tuple(a.astype(np.float32).astype(np.float64) for a in arrs)
        ins.append(arrs)
    mixed = list(params)
    mixed[1] = pf.make_params(sizes[1], cases[1][1], cases[1][1], 1.0, 0.05 * cases[1][1],
                              dtype=dtype, scheme="rk4")
    with pytest.raises(pf.PhaseFieldError) as ei:
        pf.BatchSolver(mixed)
    assert ei.value.status == pf.PF_ERR_UNSUPPORTED
    outs = []
    for persistent in (False, True):
        bs = pf.BatchSolver(params)
        with pytest.raises(pf.PhaseFieldError) as ei:
            bs.set_shape("fused_32x16")
        assert ei.value.status == pf.PF_ERR_UNSUPPORTED
        bs.set_persistent(persistent)
        bt = [[dev(a, tdt) for a in arrs] for arrs in ins]
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            bs.step(*zip(*bt), nsteps=nsteps, stream=st)
        st.synchronize()
        bs.close()
        outs.append([b[0] for b in bt])
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    for p, arrs, b, wl in zip(params, ins, outs[0], walls):
        s = pf.Solver(tuple(p.n), p.dx, p.eps, p.gamma, p.dt, dtype=dtype, scheme=scheme, walls=wl)
        g = [dev(a, tdt) for a in arrs]
        s.step(*g, nsteps=nsteps)
        torch.cuda.synchronize()
        s.close()
        assert torch.equal(g[0], b), p.n[:]
    n, dx = cases[0][0], cases[0][1]
    ref = oracle.step(*ins[0], dx=dx, eps=dx, gamma=1.0, dt=0.05 * dx, nsteps=nsteps,
                      scheme={"rk3": 3, "rk2": 2, "euler": 1}[scheme], fp32=(dtype == "f32"))
    err = rel_linf(host(outs[0][0]), ref)
    print(dtype, scheme, "batched vs oracle", err, flush=True)
    assert err <= (1e-12 if dtype == "f64" else 1e-5), err
    assert np.abs(host(outs[0][0]) - ins[0][0]).max() > 1e-4  # the steps moved the field
