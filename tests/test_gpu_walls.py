"""GPU parity of the solid-wall boundaries (through the C ABI).

Walls on any axes run on every kernel: per-stage (tiled, one-plane, one-thread-per-cell) and the
fused two-stage sweeps (mirror reads; in x and y the ghost cells of the middle stage copied from
their mirror partners, in z the ghost planes evaluated from mirrored inputs and velocities). A
handle with walls and variant -1 takes the walled default (per-stage in FP64, fused 32x16 in
FP32 from about 144^3 cells). Bars as for the periodic grids: FP64 <= 1e-12 relative L-inf against the
oracle with the same walls, FP32 <= 1e-5 against its FP32-storage mode, every variant bitwise
equal to every other. The face velocity on the wall faces is random (it must be ignored).
"""
import numpy as np
import pytest
import torch

import oracle
import pf_fixtures as fx

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5


def rel_linf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def wall_case(seed, shape):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    dx = 1.0 / max(shape)
    phi = fx.drops_ic(shape, dx, [(0.2 * nx * dx, 0.7 * ny * dx, 0.3 * nz * dx)],
                      [0.3 * max(shape) * dx], 1.3 * dx)
    phi = 0.85 * phi + 0.15 * rng.uniform(size=shape)
    U, V, W = fx.random_edge_faces(rng, shape, dx)
    s = 1.0 / max(fx.max_face_speed(U, V, W), 1e-30)
    return phi, U * s, V * s, W * s, dx


def run(pf, phi, U, V, W, *, variant, dtype, walls, **kw):
    nz, ny, nx = phi.shape
    tdt = torch.float64 if dtype == "f64" else torch.float32
    s = pf.Solver((nx, ny, nz), kw["dx"], kw["eps"], kw["gamma"], kw["dt"], dtype=dtype,
                  scheme=kw.get("scheme", "rk4"), variant=variant, walls=walls)
    g = [torch.tensor(np.ascontiguousarray(a), dtype=tdt, device="cuda") for a in (phi, U, V, W)]
    s.step(*g, nsteps=kw["nsteps"])
    torch.cuda.synchronize()
    out = g[0].cpu().numpy().astype(np.float64)
    s.close()
    return out


CASES = [("f64", (12, 10, 70), (True, False, False)), ("f64", (9, 33, 17), (False, True, False)),
         ("f64", (20, 6, 9), (False, False, True)), ("f64", (7, 13, 66), (True, True, True)),
         ("f64", (1, 30, 40), (True, True, False)), ("f64", (3, 2, 1), (False, True, True)),
         ("f32", (18, 12, 68), (True, False, True)), ("f32", (1, 37, 33), (True, True, False)),
         ("f32", (20, 45, 70), (True, True, False)), ("f64", (16, 40, 36), (True, True, False)),
         ("f32", (24, 70, 130), (True, False, False)), ("f64", (21, 35, 67), (False, True, False))]


@pytest.mark.parametrize("dtype,shape,walls", CASES)
def test_walls_every_variant_matches_oracle_and_each_other(lib, dtype, shape, walls):
    pf = lib
    kd = pf.PF_F64 if dtype == "f64" else pf.PF_F32
    phi, U, V, W, dx = wall_case(sum(shape), shape)
    if dtype == "f32":
        phi, U, V, W = (a.astype(np.float32).astype(np.float64) for a in (phi, U, V, W))
    kw = dict(dx=dx, eps=dx, gamma=1.2, dt=0.1 * dx, nsteps=5)
    ref = oracle.step(phi, U, V, W, walls=walls, fp32=dtype == "f32", **kw)
    outs = []
    for v in range(pf.phasefield_variant_count(kd)):
        print("case", dtype, shape, walls, "variant", pf.phasefield_variant_name(kd, v), flush=True)
        outs.append(run(pf, phi, U, V, W, variant=v, dtype=dtype, walls=walls, **kw))
        err = rel_linf(outs[-1], ref)
        assert err <= (TOL64 if dtype == "f64" else TOL32), (v, err)
    for v, o in enumerate(outs[1:], 1):
        assert np.array_equal(o, outs[0]), f"variant {v} differs from variant 0"


@pytest.mark.parametrize("scheme,sch,walls", [("euler", 1, (True, False, True)),
                                              ("rk2", 2, (True, False, True)),
                                              ("rk2", 2, (True, True, False))])
def test_walls_other_schemes(lib, scheme, sch, walls):
    phi, U, V, W, dx = wall_case(5, (10, 12, 14))
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.08 * dx, nsteps=7, scheme=scheme)
    ref = oracle.step(phi, U, V, W, walls=walls, **{**kw, "scheme": sch})
    got = run(lib, phi, U, V, W, variant=-1, dtype="f64", walls=walls, **kw)
    assert rel_linf(got, ref) <= TOL64
    names = [lib.phasefield_variant_name(lib.PF_F64, v) for v in range(lib.phasefield_variant_count(lib.PF_F64))]
    fused = run(lib, phi, U, V, W, variant=names.index("fused_32x16x32"), dtype="f64", walls=walls, **kw)
    assert np.array_equal(fused, got)


def test_walls_conserve_mass(lib):
    pf = lib
    shape = (24, 20, 28)
    phi, U, V, W, dx = wall_case(7, shape)
    walls = (True, True, True)
    nz, ny, nx = shape
    s = pf.Solver((nx, ny, nz), dx, dx, 1.0, 0.1 * dx, dtype="f64", walls=walls)
    g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi, U, V, W)]
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        m0 = s.reduce(g[0], stream=st)[0]
        s.step(*g, nsteps=60, stream=st)
        m1 = s.reduce(g[0], stream=st)[0]
    assert abs(m1 - m0) / m0 < 1e-13, (m0, m1)
    s.close()


ADJ_CASES = [("rk4", (True, False, False), (14, 18, 40)), ("rk4", (False, True, True), (20, 16, 70)),
             ("rk4", (True, True, True), (9, 11, 7)), ("rk3", (True, True, False), (12, 10, 14)),
             ("rk2", (False, False, True), (12, 10, 14)), ("euler", (True, False, True), (9, 11, 7)),
             ("rk4", (True, True, False), (1, 20, 18))]


@pytest.mark.parametrize("scheme,walls,shape", ADJ_CASES)
def test_walls_adjoint_matches_oracle(lib, scheme, walls, shape):
    """The adjoint step on walled axes (stage input and cotangent read through mirror indices)
    against the oracle's walled adjoint (FP64 1e-12 for lambda and the three face gradients,
    whose wall-face entries stay untouched), and bitwise across the plain kernel, the tiled
    tiles and chunk lengths, the large-array form and a fused handle; FP32 against the FP64
    oracle at 1e-3."""
    pf = lib
    phi, U, V, W, dx = wall_case(sum(shape) + 3, shape)
    nz, ny, nx = shape
    rng = np.random.default_rng(len(scheme))
    lam = rng.standard_normal(shape)
    kw = dict(dx=dx, eps=dx, gamma=1.2, dt=0.1 * dx, delta=0.05 / dx, vel_mode=1, vel_T=0.8)
    ref = oracle.adjoint_step(phi, U, V, W, lam, t=0.1, walls=walls,
                              scheme={"rk4": 4, "rk3": 3, "rk2": 2, "euler": 1}[scheme], **kw)
    names = [pf.phasefield_variant_name(pf.PF_F64, v) for v in range(pf.phasefield_variant_count(pf.PF_F64))]
    outs = []
    for vname in ("global", "tiled_64x8x16", "tiled_32x4", "tiled_64x8x16_big", "fused_32x16"):
        print("case", scheme, walls, shape, vname, flush=True)
        s = pf.Solver((nx, ny, nz), scheme=scheme, walls=walls, variant=names.index(vname), **kw)
        g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi, U, V, W)]
        L = torch.tensor(lam, dtype=torch.float64, device="cuda")
        grads = [torch.zeros_like(L) for _ in range(3)]
        s.adjoint_step(*g, 0.1, L, *grads)
        torch.cuda.synchronize()
        s.close()
        outs.append([L] + grads)
    for k, (got, want) in enumerate(zip(outs[0], ref)):
        err = rel_linf(got.cpu().numpy(), want)
        print("output", k, "error", err, flush=True)
        assert err <= TOL64, (k, err)
    for a, w in enumerate(walls):
        if w:
            sl = [slice(None)] * 3
            sl[2 - a] = 0
            assert not outs[0][1 + a][tuple(sl)].any()
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert torch.equal(x, y)
    # FP32 storage against the FP64 oracle
    s = pf.Solver((nx, ny, nz), scheme=scheme, walls=walls, dtype="f32", **kw)
    g = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in (phi, U, V, W)]
    L = torch.tensor(lam, dtype=torch.float32, device="cuda")
    grads = [torch.zeros_like(L) for _ in range(3)]
    s.adjoint_step(*g, 0.1, L, *grads)
    torch.cuda.synchronize()
    s.close()
    for k, (got, want) in enumerate(zip([L] + grads, ref)):
        err = rel_linf(got.cpu().numpy().astype(np.float64), want)
        assert err <= 1e-3, (k, err)


@pytest.mark.parametrize("dtype,shape,walls,want", [
    ("f64", (20, 20, 20), (False, False, True), "tiled_32x4"),
    ("f64", (200, 200, 192), (True, False, False), "tiled_64x8"),
    ("f32", (40, 36, 128), (False, True, False), "tiled_64x8"),
    ("f32", (40, 36, 96), (False, True, False), "tiled_32x4"),
    ("f32", (150, 150, 160), (True, True, True), "fused_32x16"),
    ("f32", (150, 150, 160), (False, False, False), None)])
def test_walled_default_variant(lib, dtype, shape, walls, want):
    """variant -1 on a grid with walls takes the walled default (the tuning cache is for periodic
    grids); a periodic grid keeps the periodic default."""
    pf = lib
    nz, ny, nx = shape
    s = pf.Solver((nx, ny, nz), 1.0 / nx, 1.0 / nx, 1.0, 0.1 / nx, dtype=dtype, walls=walls)
    name = s.variant_name
    s.close()
    print(dtype, shape, walls, name, flush=True)
    if want is None:
        assert name.startswith("fused_")
    else:
        assert name == want
