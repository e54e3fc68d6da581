"""GPU parity of the forward step, reduction, graphs and error paths (through the C ABI).

Bar: FP64 storage <= 1e-12 relative L-inf against the FP64 oracle; FP32 storage <= 1e-5 against
the oracle's FP32-storage mode (relative L-inf = max|a-b| / max|b|). Every stage-kernel variant
must agree bitwise with every other.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import pf_fixtures as fx

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel_linf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def random_case(rng, shape, umax=1.0):
    nz, ny, nx = shape
    dx = 1.0 / max(shape)
    phi = fx.drops_ic(shape, dx, [(0.5 * nx * dx, 0.4 * ny * dx, 0.5 * nz * dx)],
                      [0.3 * max(shape) * dx], 1.5 * dx)
    phi = 0.8 * phi + 0.2 * rng.uniform(size=shape)
    U, V, W = fx.random_edge_faces(rng, shape, dx)
    if nz == 1:
        W = np.zeros(shape)
        zero = np.zeros(shape)
        U, V, _ = fx.edge_curl(zero, zero, rng.standard_normal(shape) * dx, dx)
    s = umax / max(fx.max_face_speed(U, V, W), 1e-30)
    return phi, U * s, V * s, W * s, dx


def gpu_run(pf, phi, U, V, W, *, dx, eps, gamma, dt, nsteps, dtype="f64", scheme="rk4",
            delta=0.0, vel_mode=0, vel_T=1.0, t0=0.0, variant=-1, use_graph=True, stream=None):
    nz, ny, nx = phi.shape
    tdt = torch.float64 if dtype == "f64" else torch.float32
    s = pf.Solver((nx, ny, nz), dx, eps, gamma, dt, dtype=dtype, scheme=scheme, delta=delta,
                  vel_mode=vel_mode, vel_T=vel_T, variant=variant, use_graph=use_graph)
    g = [dev(a, tdt) for a in (phi, U, V, W)]
    s.step(*g, t0=t0, nsteps=nsteps, stream=stream)
    torch.cuda.synchronize()
    out = g[0].cpu().numpy().astype(np.float64)
    s.close()
    return out


# (nz, ny, nx): ragged tiles, degenerate axes, and nx both a multiple of the 16-byte piece (two
# doubles / four floats: the fused sweeps' 16-byte plane loads) and not
SHAPES = [(16, 20, 24), (5, 9, 70), (1, 33, 17), (1, 1, 37), (3, 2, 1), (7, 6, 65), (2, 1, 3),
          (33, 17, 9), (6, 5, 4)]


@pytest.mark.parametrize("shape", SHAPES)
def test_rk4_fp64_all_variants_match_oracle_and_each_other(lib, shape):
    pf = lib
    rng = np.random.default_rng(sum(shape))
    phi, U, V, W, dx = random_case(rng, shape)
    kw = dict(dx=dx, eps=dx, gamma=1.3, dt=0.15 * dx, nsteps=7, delta=0.0)
    ref = oracle.step(phi, U, V, W, **kw)
    outs = []
    for v in range(pf.phasefield_variant_count(pf.PF_F64)):
        print("case", shape, "variant", pf.phasefield_variant_name(pf.PF_F64, v), flush=True)
        outs.append(gpu_run(pf, phi, U, V, W, variant=v, **kw))
        assert rel_linf(outs[-1], ref) <= TOL64, (v, rel_linf(outs[-1], ref))
    for v, o in enumerate(outs[1:], 1):
        assert np.array_equal(o, outs[0]), f"variant {v} differs from variant 0"


@pytest.mark.parametrize("shape", [(40, 36, 70), (1, 33, 130), (9, 5, 7), (40, 36, 68), (3, 7, 8)])
def test_fp32_all_variants_match_oracle_and_each_other(lib, shape):
    """Every FP32 variant (per-stage and fused two-stage sweeps) against the oracle's FP32
    storage mode, and bit-identical to each other; odd step count."""
    pf = lib
    rng = np.random.default_rng(11 + sum(shape))
    phi, U, V, W, dx = random_case(rng, shape)
    phi, U, V, W = (a.astype(np.float32).astype(np.float64) for a in (phi, U, V, W))
    kw = dict(dx=dx, eps=dx, gamma=1.2, dt=0.15 * dx, nsteps=5)
    ref = oracle.step(phi, U, V, W, fp32=True, **kw)
    outs = []
    for v in range(pf.phasefield_variant_count(pf.PF_F32)):
        print("case", shape, "variant", pf.phasefield_variant_name(pf.PF_F32, v), flush=True)
        outs.append(gpu_run(pf, phi, U, V, W, variant=v, dtype="f32", **kw))
        assert rel_linf(outs[-1], ref) <= TOL32, (v, rel_linf(outs[-1], ref))
    for v, o in enumerate(outs[1:], 1):
        assert np.array_equal(o, outs[0]), f"variant {v} differs from variant 0"


@pytest.mark.parametrize("scheme", ["rk2", "rk3"])
@pytest.mark.parametrize("dtype,shape", [("f64", (16, 20, 24)), ("f64", (5, 9, 70)),
                                         ("f64", (1, 33, 17)), ("f64", (3, 2, 1)),
                                         ("f64", (7, 6, 65)), ("f32", (40, 36, 68)),
                                         ("f32", (9, 5, 7)), ("f32", (1, 33, 130))])
def test_rk2_rk3_all_variants_match_oracle_and_each_other(lib, dtype, shape, scheme):
    """The explicit midpoint rule (Eq. 26) and the low-storage RK3 (Eq. 27) of Sec. 2.3 on every
    variant: RK2's per-stage form (two launches) and fused form (one sweep, the midpoint value
    kept in LDS), RK3's per-stage form (three launches; fused variants fall back to it), all
    bitwise equal and matching the oracle, over an odd and an even step count (the fused form
    alternates phi with a second buffer)."""
    pf = lib
    kd = pf.PF_F64 if dtype == "f64" else pf.PF_F32
    rng = np.random.default_rng(21 + sum(shape))
    phi, U, V, W, dx = random_case(rng, shape)
    if dtype == "f32":
        phi, U, V, W = (a.astype(np.float32).astype(np.float64) for a in (phi, U, V, W))
    for nsteps in (7, 4):
        kw = dict(dx=dx, eps=dx, gamma=1.3, dt=0.1 * dx, nsteps=nsteps)
        ref = oracle.step(phi, U, V, W, scheme={"rk2": 2, "rk3": 3}[scheme], fp32=dtype == "f32", **kw)
        outs = []
        for v in range(pf.phasefield_variant_count(kd)):
            print("case", dtype, shape, nsteps, "variant", pf.phasefield_variant_name(kd, v),
                  flush=True)
            outs.append(gpu_run(pf, phi, U, V, W, variant=v, dtype=dtype, scheme=scheme, **kw))
            err = rel_linf(outs[-1], ref)
            assert err <= (TOL64 if dtype == "f64" else TOL32), (v, err)
        for v, o in enumerate(outs[1:], 1):
            assert np.array_equal(o, outs[0]), f"variant {v} differs from variant 0"


@pytest.mark.parametrize("shape", [(12, 10, 14), (1, 24, 20)])
def test_euler_and_cos_reversal_fp64(lib, shape):
    rng = np.random.default_rng(3)
    phi, U, V, W, dx = random_case(rng, shape)
    for scheme, sch in (("euler", 1), ("rk2", 2), ("rk3", 3), ("rk4", 4)):
        kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, nsteps=9, delta=0.01 / dx, vel_mode=1,
                  vel_T=0.37, t0=0.05)
        ref = oracle.step(phi, U, V, W, scheme=sch, **kw)
        got = gpu_run(lib, phi, U, V, W, scheme=scheme, **kw)
        assert rel_linf(got, ref) <= TOL64
        # one plane: the one-launch step equals the per-stage launches of the 'global' variant
        if shape[0] == 1:
            names = [lib.phasefield_variant_name(lib.PF_F64, v)
                     for v in range(lib.phasefield_variant_count(lib.PF_F64))]
            per_stage = gpu_run(lib, phi, U, V, W, scheme=scheme, variant=names.index("global"), **kw)
            assert np.array_equal(got, per_stage), scheme


@pytest.mark.parametrize("shape", [(16, 20, 24), (1, 40, 33), (9, 70, 5)])
def test_fp32_storage_matches_oracle_fp32_mode(lib, shape):
    rng = np.random.default_rng(5)
    phi, U, V, W, dx = random_case(rng, shape)
    phi, U, V, W = (a.astype(np.float32).astype(np.float64) for a in (phi, U, V, W))
    kw = dict(dx=dx, eps=dx, gamma=1.1, dt=0.15 * dx, nsteps=40)
    ref = oracle.step(phi, U, V, W, fp32=True, **kw)
    got = gpu_run(lib, phi, U, V, W, dtype="f32", **kw)
    assert rel_linf(got, ref) <= TOL32, rel_linf(got, ref)


def test_vortex2d_full_period_fp64(lib):
    """Drop in the reversing single vortex, 64 x 64, 2560 RK4 steps to t = T (Sec. 3.3.1)."""
    c = fx.vortex2d(64)
    kw = dict(dx=c.dx, eps=c.eps, gamma=c.gamma, dt=c.dt, nsteps=c.nsteps, vel_mode=1,
              vel_T=c.vel_T)
    ref = oracle.step(c.phi0, c.U, c.V, c.W, **kw)
    got = gpu_run(lib, c.phi0, c.U, c.V, c.W, **kw)
    assert rel_linf(got, ref) <= TOL64, rel_linf(got, ref)
    e_shape = np.abs(got - c.phi0).sum() * c.dx * c.dx
    print("E_shape(64) =", e_shape)
    assert 0 < e_shape < 0.05


def test_deformation3d_full_reversal_32(lib):
    c = fx.deformation3d(32)
    nsteps = int(math.ceil(c.vel_T / c.dt))
    dt = c.vel_T / nsteps
    kw = dict(dx=c.dx, eps=c.eps, gamma=c.gamma, dt=dt, nsteps=nsteps, vel_mode=1, vel_T=c.vel_T)
    ref = oracle.step(c.phi0, c.U, c.V, c.W, **kw)
    got = gpu_run(lib, c.phi0, c.U, c.V, c.W, **kw)
    assert rel_linf(got, ref) <= TOL64
    a32 = [x.astype(np.float32).astype(np.float64) for x in (c.phi0, c.U, c.V, c.W)]
    ref32 = oracle.step(*a32, fp32=True, **kw)
    got32 = gpu_run(lib, *a32, dtype="f32", **kw)
    assert rel_linf(got32, ref32) <= TOL32, rel_linf(got32, ref32)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_deformation3d_64_mass_and_bounds(lib, dtype):
    """On the crossover line (eps = dx, gamma = max|u|) at 0.9 x Eq. 28: mass conserved to
    round-off and phi inside [0, 1] up to the storage precision (Sec. 2.2, Sec. 2.3)."""
    pf = lib
    c = fx.deformation3d(64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    s = pf.Solver((64, 64, 64), c.dx, c.eps, c.gamma, c.dt, dtype=dtype, vel_mode=1, vel_T=c.vel_T)
    g = [dev(a, tdt) for a in (c.phi0, c.U, c.V, c.W)]
    m0 = s.reduce(g[0])[0]
    lo, hi = 1.0, 0.0
    for blk in range(10):
        s.step(*g, t0=blk * 20 * c.dt, nsteps=20)
        mass, mn, mx, bad = s.reduce(g[0])
        lo, hi = min(lo, mn), max(hi, mx)
        assert bad == 0
    drift = abs(mass - m0) / m0
    eps_m = np.finfo(np.float64 if dtype == "f64" else np.float32).eps
    print(dtype, "mass drift", drift, "min", lo, "max-1", hi - 1)
    assert drift <= (1e-12 if dtype == "f64" else 1e-6)
    assert lo >= -eps_m and hi <= 1 + eps_m
    s.close()


def test_reduce_matches_oracle(lib):
    pf = lib
    rng = np.random.default_rng(7)
    shape = (13, 17, 19)
    phi = rng.uniform(-0.1, 1.1, size=shape)
    s = pf.Solver((19, 17, 13), 0.05, 0.05, 1.0, 0.01)
    g = dev(phi)
    mass, mn, mx, bad = s.reduce(g)
    om, omn, omx, obad = oracle.reduce(phi, dx=0.05)
    assert mass == pytest.approx(om, rel=1e-13) and mn == omn and mx == omx and bad == obad == 0
    phi[3, 4, 5] = np.nan
    phi[0, 0, 1] = np.inf
    mass, mn, mx, bad = s.reduce(dev(phi))
    om, omn, omx, obad = oracle.reduce(phi, dx=0.05)
    assert bad == obad == 2 and mn == omn and mx == omx
    assert mass == pytest.approx(om, rel=1e-13)
    gn = dev(phi)
    with pytest.raises(pf.PhaseFieldError) as ei:
        pf._capi._check(pf.lib.phasefield_reduce(s.handle, gn.data_ptr(),
                                                 (pf._capi.ctypes.c_double * 4)(), 0))
    assert ei.value.status == pf.PF_ERR_NONFINITE
    s.close()


def test_shift_equivariance_bitwise(lib):
    rng = np.random.default_rng(9)
    shape = (18, 21, 70)
    phi, U, V, W, dx = random_case(rng, shape)
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, nsteps=4)
    a = gpu_run(lib, phi, U, V, W, **kw)
    sh = (5, -7, 33)
    r = lambda x: np.roll(x, sh, axis=(0, 1, 2))  # noqa: E731
    b = gpu_run(lib, r(phi), r(U), r(V), r(W), **kw)
    assert np.array_equal(b, r(a))


@pytest.mark.parametrize("kind", ["tiled", "fused"])
def test_graph_replay_matches_eager(lib, kind):
    """Graph replays (8 steps per graph) agree bitwise with plain launches, replay after replay
    with eager work and synchronisations in between; 19 steps = two replays + an odd remainder
    (which, for a fused variant, ends on the alternate buffer and is copied back)."""
    pf = lib
    rng = np.random.default_rng(11)
    shape = (20, 24, 28)
    phi, U, V, W, dx = random_case(rng, shape)
    st = torch.cuda.Stream()
    names = [pf.phasefield_variant_name(pf.PF_F64, v)
             for v in range(pf.phasefield_variant_count(pf.PF_F64))]
    variant = [i for i, n in enumerate(names) if n.startswith(kind)][0]
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, variant=variant)
    sg = pf.Solver((28, 24, 20), use_graph=True, **kw)
    se = pf.Solver((28, 24, 20), use_graph=False, **kw)
    a = [dev(x) for x in (phi, U, V, W)]
    b = [dev(x) for x in (phi, U, V, W)]
    for rep in range(4):
        with torch.cuda.stream(st):
            sg.step(*a, nsteps=19, stream=st)
            se.step(*b, nsteps=19, stream=st)
            junk = torch.ones(1000, device="cuda").sum()  # unrelated eager work between replays
        st.synchronize()
        assert float(junk) == 1000.0
        assert torch.equal(a[0], b[0]), rep
    sg.close()
    se.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_time_varying_loop_graph_matches_eager(lib, dtype):
    """With the cos(pi t / T) velocity a loop of 16 or more steps is captured whole into one
    graph (each step has its own time factors) and replayed when the same loop (t0, nsteps,
    buffers) comes again: bitwise equal to plain launches, replay after replay with eager work
    and synchronisations in between, and after a different loop has replaced the graph."""
    pf = lib
    rng = np.random.default_rng(12)
    shape = (20, 24, 28)
    phi, U, V, W, dx = random_case(rng, shape)
    st = torch.cuda.Stream()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, dtype=dtype, vel_mode=1, vel_T=0.07)
    sg = pf.Solver((28, 24, 20), use_graph=True, **kw)
    se = pf.Solver((28, 24, 20), use_graph=False, **kw)
    a = [dev(x, tdt) for x in (phi, U, V, W)]
    b = [dev(x, tdt) for x in (phi, U, V, W)]
    for rep, (t0, n) in enumerate([(0.0, 21), (0.0, 21), (0.013, 21), (0.0, 40), (0.0, 21)]):
        with torch.cuda.stream(st):
            sg.step(*a, t0=t0, nsteps=n, stream=st)
            se.step(*b, t0=t0, nsteps=n, stream=st)
            junk = torch.ones(1000, device="cuda").sum()  # unrelated eager work between replays
        st.synchronize()
        assert float(junk) == 1000.0
        assert torch.equal(a[0], b[0]), rep
    sg.close()
    se.close()


def test_argument_errors(lib):
    pf = lib
    with pytest.raises(pf.PhaseFieldError) as ei:
        pf.Solver((8, 8, 8), -1.0, 0.1, 1.0, 0.01)
    assert ei.value.status == pf.PF_ERR_INVALID
    p = pf.make_params((8, 8, 8), 0.1, 0.1, 1.0, 0.01)
    p.bc[0] = 7  # not a pf_bc value
    with pytest.raises(pf.PhaseFieldError) as ei:
        pf.phasefield_create(p)
    assert ei.value.status == pf.PF_ERR_INVALID
    s = pf.Solver((8, 8, 8), 0.1, 0.1, 1.0, 0.01)
    t = torch.zeros(8 * 8 * 8 + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(pf.PhaseFieldError) as ei:  # misaligned pointer reaches the C ABI
        pf._capi._check(pf.lib.phasefield_step(s.handle, t.data_ptr() + 8, t.data_ptr(),
                                               t.data_ptr(), t.data_ptr(), 0.0, 1, 0))
    assert ei.value.status == pf.PF_ERR_INVALID
    with pytest.raises(pf.PhaseFieldError) as ei:
        pf._capi._check(pf.lib.phasefield_step(s.handle, None, t.data_ptr(), t.data_ptr(),
                                               t.data_ptr(), 0.0, 1, 0))
    assert ei.value.status == pf.PF_ERR_INVALID
    s.close()


def test_autotune_and_persistent_cache(lib, tmp_path, monkeypatch):
    """phasefield_autotune times every variant, the winner is used by later handles of the same
    shape, and PF_TUNE_CACHE persists choices by variant name."""
    pf = lib
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PF_TUNE_CACHE", str(cache))
    s = pf.Solver((48, 40, 36), 1 / 48, 1 / 48, 1.0, 0.1 / 48, dtype="f32")
    best, times = s.autotune(reps=1)
    assert len(times) == pf.phasefield_variant_count(pf.PF_F32) and all(t > 0 for t in times.values())
    name = pf.phasefield_variant_name(pf.PF_F32, best)
    assert s.variant == best and times[name] == min(times.values())
    s.close()
    assert cache.read_text().split() == ["0", "48", "40", "36", name]
    s2 = pf.Solver((48, 40, 36), 1 / 48, 1 / 48, 1.0, 0.1 / 48, dtype="f32")
    assert s2.variant == best
    s2.close()
    # a cache written by hand (by name) is honoured once the variable points at it
    other = tmp_path / "other.txt"
    other.write_text("1 40 40 40 tiled_32x4x16\n1 40 40 40 no_such_variant\n")
    monkeypatch.setenv("PF_TUNE_CACHE", str(other))
    s3 = pf.Solver((40, 40, 40), 1 / 40, 1 / 40, 1.0, 0.1 / 40, dtype="f64")
    assert s3.variant_name == "tiled_32x4x16"
    s3.close()


def test_default_variant_on_one_plane_grids(lib):
    """Grids of one plane take the per-stage (march-free plane) kernel at every size, never a
    fused sweep; 64x8 tiles from 256^2 cells, the per-stage rule's tiles below. Thicker grids
    take the fused sweeps from 104^3 cells (FP32; on 32x16 tiles below 256^3 cells and 64x8 from
    there) and from 128^3 cells (FP64, 32x16), the per-stage kernels below."""
    pf = lib
    cases = [((1024, 1024, 1), "f32", "tiled_64x8"), ((512, 512, 1), "f64", "tiled_64x8"),
             ((64, 64, 1), "f64", "tiled_32x4"), ((96, 4000, 1), "f32", "tiled_32x4"),
             ((1024, 1024, 2), "f32", "fused_32x16"), ((256, 256, 256), "f32", "fused_64x8"),
             ((96, 96, 96), "f32", "tiled_32x4"), ((112, 112, 112), "f32", "fused_32x16"),
             ((120, 120, 120), "f64", "tiled_32x4"), ((128, 128, 128), "f64", "fused_32x16")]
    for n, dtype, want in cases:
        s = pf.Solver(n, 1.0 / n[0], 1.0 / n[0], 1.0, 0.1 / n[0], dtype=dtype)
        assert s.variant_name == want, (n, dtype, s.variant_name)
        s.close()
