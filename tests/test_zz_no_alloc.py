"""phasefield_step_noalloc (stage buffers in the library's fixed device array, no handle, no
allocation) against phasefield_step on a handle: bit-identical results on two calls in a row,
the second on a smaller grid, in both storage precisions, for RK4 (fused and per-stage
variants), RK3 and Euler; a grid beyond the array is refused."""
import ctypes

import numpy as np
import pytest
import torch

import pf_fixtures as fx

pytestmark = pytest.mark.gpu


def case(shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    dx = 1.0 / max(shape)
    phi = fx.drops_ic(shape, dx, *fx.random_drops(rng, 3, 0.1, 0.3), dx)
    U, V, W = fx.random_edge_faces(rng, shape, dx)
    s = 1.0 / fx.max_face_speed(U, V, W)
    return dx, phi, U * s, V * s, W * s


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("scheme,variant", [("rk4", -1), ("rk4", "fused_32x16"),
                                            ("rk4", "tiled_64x4"), ("rk3", -1), ("euler", -1)])
def test_noalloc_step_matches_handle_step(lib, dtype, scheme, variant):
    pf = lib
    tdt = torch.float64 if dtype == "f64" else torch.float32
    kd = pf.PF_F64 if dtype == "f64" else pf.PF_F32
    if isinstance(variant, str):
        names = [pf.phasefield_variant_name(kd, v) for v in range(pf.phasefield_variant_count(kd))]
        variant = names.index(variant)
    for shape, nsteps, seed in (((40, 36, 97), 7, 1), ((17, 20, 33), 6, 2)):
        dx, phi, U, V, W = case(shape, seed)
        nz, ny, nx = shape
        p = pf.make_params((nx, ny, nz), dx, dx, 1.0, fx.rk4_dt_3d(dx, 1.0, dx) * 0.8,
                           dtype=dtype, scheme=scheme, variant=variant, vel_mode=1, vel_T=0.3)
        a = [torch.tensor(x, dtype=tdt, device="cuda") for x in (phi, U, V, W)]
        b = [x.clone() for x in a]
        print(dtype, scheme, variant, shape, nsteps, "steps", flush=True)
        pf.phasefield_step_noalloc(p, *a, t0=0.05, nsteps=nsteps)
        s = pf.Solver((nx, ny, nz), dx, dx, 1.0, p.dt, dtype=dtype, scheme=scheme,
                      variant=variant, vel_mode=1, vel_T=0.3)
        s.step(*b, t0=0.05, nsteps=nsteps)
        torch.cuda.synchronize()
        s.close()
        assert torch.equal(a[0], b[0]), shape
        assert not torch.equal(a[0], torch.tensor(phi, dtype=tdt, device="cuda"))


def test_noalloc_refuses_grid_beyond_scratch(lib):
    pf = lib
    cap = pf.phasefield_noalloc_scratch_bytes()
    assert cap == 64 << 20
    n = 150  # 3 x 150^3 x 8 bytes > 64 MiB
    p = pf.make_params((n, n, n), 1.0 / n, 1.0 / n, 1.0, 1e-4, dtype="f64")
    t = torch.zeros(16, dtype=torch.float64, device="cuda")
    ptr = ctypes.c_void_p(t.data_ptr())
    st = pf.lib.phasefield_step_noalloc(ctypes.byref(p), ptr, ptr, ptr, ptr, 0.0, 1, None)
    assert st == pf.PF_ERR_INVALID
    assert "scratch" in pf.phasefield_last_error()
