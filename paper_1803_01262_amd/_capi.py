"""ctypes binding of libphasefield.so: the C ABI of include/phasefield.h, one Python function per
entry point with the same name. Argument marshalling only — every computation runs in the HIP
library. Tensors must be contiguous CUDA (HIP) tensors of the handle's storage dtype; streams
default to torch's current stream.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphasefield.so")

PF_OK, PF_ERR_INVALID, PF_ERR_UNSUPPORTED, PF_ERR_DEVICE, PF_ERR_OOM, PF_ERR_NONFINITE = range(6)
PF_F32, PF_F64 = 0, 1
PF_BC_PERIODIC, PF_BC_WALL = 0, 1
PF_EULER, PF_RK2, PF_RK3, PF_RK4 = 1, 2, 3, 4
PF_VEL_STEADY, PF_VEL_COS_REVERSAL = 0, 1

_STATUS = {0: "PF_OK", 1: "PF_ERR_INVALID", 2: "PF_ERR_UNSUPPORTED", 3: "PF_ERR_DEVICE",
           4: "PF_ERR_OOM", 5: "PF_ERR_NONFINITE"}


class PhaseFieldError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    """pf_params (see include/phasefield.h)."""
    _fields_ = [("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double), ("eps", ctypes.c_double),
                ("gamma", ctypes.c_double), ("dt", ctypes.c_double), ("delta", ctypes.c_double),
                ("bc", ctypes.c_int32 * 3), ("dtype", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("vel_mode", ctypes.c_int32), ("vel_T", ctypes.c_double),
                ("variant", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("crossover_margin_eq17", ctypes.c_double),
                ("crossover_margin_eq24", ctypes.c_double),
                ("dt_max_scheme", ctypes.c_double), ("dt_over_dtmax", ctypes.c_double)]


def _build_once():
    """Compile the library when nothing is built yet (a fresh tree); a failed build raises."""
    import importlib.util
    import sys
    print(f"{LIB_PATH} is not built; building it now", file=sys.stderr, flush=True)
    spec = importlib.util.spec_from_file_location(
        "pf_hip_build", os.path.join(os.path.dirname(os.path.abspath(__file__)), "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.build(verbose=False)


def _load():
    if not os.path.exists(LIB_PATH):
        try:
            _build_once()
        except Exception as e:  # no compiler, or the build failed: no fallback
            raise ImportError(f"{LIB_PATH} is not built and building it failed ({e}); run "
                              "__graft_entry__.build() or python paper_1803_01262_amd/build.py") from e
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                              "python paper_1803_01262_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, d, i32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32
    sig = {
        "phasefield_default_params": (None, [P(Params)]),
        "phasefield_check_params": (i32, [P(Params), d, P(Report)]),
        "phasefield_create": (i32, [P(Params), P(vp)]),
        "phasefield_destroy": (i32, [vp]),
        "phasefield_step": (i32, [vp, vp, vp, vp, vp, d, i32, vp]),
        "phasefield_adjoint_step": (i32, [vp, vp, vp, vp, vp, d, vp, vp, vp, vp, vp]),
        "phasefield_step_stages": (i32, [vp, vp, vp, vp, vp, vp, d, vp, vp, vp, vp]),
        "phasefield_adjoint_step_stages": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, d, vp, vp, vp,
                                                 vp, vp]),
        "phasefield_reduce": (i32, [vp, vp, P(d), vp]),
        "phasefield_velocity_from_coeffs": (i32, [P(Params), i32, vp, vp, vp, vp, vp, vp]),
        "phasefield_velocity_coeffs_grad": (i32, [P(Params), i32, vp, vp, vp, vp, vp, vp]),
        "phasefield_variant_count": (i32, [i32]),
        "phasefield_variant_name": (ctypes.c_char_p, [i32, i32]),
        "phasefield_autotune": (i32, [vp, i32, P(i32), P(d), vp]),
        "phasefield_solver_variant": (i32, [vp]),
        "phasefield_set_adjoint_form": (i32, [vp, i32]),
        "phasefield_set_spacing": (i32, [vp, vp, vp, vp, i32]),
        "phasefield_batch_create": (i32, [P(Params), i32, P(vp)]),
        "phasefield_batch_step": (i32, [vp, P(vp), P(vp), P(vp), P(vp), P(d), i32, vp]),
        "phasefield_batch_destroy": (i32, [vp]),
        "phasefield_batch_set_persistent": (i32, [vp, i32]),
        "phasefield_batch_set_shape": (i32, [vp, i32]),
        "phasefield_batch_autotune": (i32, [vp, i32, P(i32), P(i32), P(d), vp]),
        "phasefield_last_error": (ctypes.c_char_p, []),
        "phasefield_step_noalloc": (i32, [P(Params), vp, vp, vp, vp, d, i32, vp]),
        "phasefield_noalloc_scratch_bytes": (ctypes.c_size_t, []),
        "phasefield_device_copy": (i32, [vp, vp, ctypes.c_size_t, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()

EXPORTED = ("phasefield_default_params", "phasefield_check_params", "phasefield_create",
            "phasefield_destroy", "phasefield_step", "phasefield_adjoint_step",
            "phasefield_step_stages", "phasefield_adjoint_step_stages",
            "phasefield_reduce", "phasefield_velocity_from_coeffs",
            "phasefield_velocity_coeffs_grad", "phasefield_variant_count",
            "phasefield_variant_name", "phasefield_autotune", "phasefield_solver_variant",
            "phasefield_set_adjoint_form", "phasefield_set_spacing",
            "phasefield_batch_create", "phasefield_batch_step", "phasefield_batch_destroy",
            "phasefield_batch_set_persistent", "phasefield_batch_set_shape",
            "phasefield_batch_autotune",
            "phasefield_last_error", "phasefield_step_noalloc",
            "phasefield_noalloc_scratch_bytes", "phasefield_device_copy")


def _check(status: int) -> None:
    if status != PF_OK:
        raise PhaseFieldError(status, lib.phasefield_last_error().decode())


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


_TORCH_DTYPE = {PF_F32: torch.float32, PF_F64: torch.float64}


def _ptr(t, dtype: int | None = None, numel: int | None = None, name: str = "tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL), after shape/dtype checks."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != _TORCH_DTYPE[dtype]:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {_TORCH_DTYPE[dtype]}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return t.data_ptr()


def make_params(n, dx, eps, gamma, dt, *, dtype="f64", scheme="rk4", delta=0.0, vel_mode=0,
                vel_T=1.0, variant=-1, use_graph=True, walls=(False, False, False)) -> Params:
    """pf_params from keyword arguments; n = (nx, ny, nz); walls: per axis (x, y, z)."""
    p = Params()
    lib.phasefield_default_params(ctypes.byref(p))
    p.n[0], p.n[1], p.n[2] = (int(v) for v in n)
    p.dx, p.eps, p.gamma, p.dt, p.delta = float(dx), float(eps), float(gamma), float(dt), float(delta)
    p.dtype = {"f32": PF_F32, "f64": PF_F64, PF_F32: PF_F32, PF_F64: PF_F64}[dtype]
    p.scheme = {"rk4": PF_RK4, "rk3": PF_RK3, "rk2": PF_RK2, "euler": PF_EULER, PF_RK4: PF_RK4,
                PF_RK3: PF_RK3, PF_RK2: PF_RK2, PF_EULER: PF_EULER}[scheme]
    p.vel_mode = int(vel_mode)
    p.vel_T = float(vel_T)
    p.variant = int(variant)
    p.use_graph = int(bool(use_graph))
    for a, w in enumerate(walls):
        p.bc[a] = PF_BC_WALL if w else PF_BC_PERIODIC
    return p


def cells(p: Params) -> int:
    return int(p.n[0]) * int(p.n[1]) * int(p.n[2])


# ----------------------------------------------------------------- one wrapper per entry point

def phasefield_default_params() -> Params:
    p = Params()
    lib.phasefield_default_params(ctypes.byref(p))
    return p


def phasefield_check_params(p: Params, max_face_speed: float) -> Report:
    r = Report()
    _check(lib.phasefield_check_params(ctypes.byref(p), float(max_face_speed), ctypes.byref(r)))
    return r


def phasefield_create(p: Params) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib.phasefield_create(ctypes.byref(p), ctypes.byref(h)))
    return h


def phasefield_destroy(h) -> None:
    _check(lib.phasefield_destroy(h))


def phasefield_step(h, p: Params, phi, u, v, w, t0=0.0, nsteps=1, stream=None) -> None:
    n = cells(p)
    _check(lib.phasefield_step(h, _ptr(phi, p.dtype, n, "phi"), _ptr(u, p.dtype, n, "u"),
                               _ptr(v, p.dtype, n, "v"), _ptr(w, p.dtype, n, "w"),
                               float(t0), int(nsteps), _stream(stream)))


def phasefield_step_noalloc(p: Params, phi, u, v, w, t0=0.0, nsteps=1, stream=None) -> None:
    n = cells(p)
    _check(lib.phasefield_step_noalloc(ctypes.byref(p), _ptr(phi, p.dtype, n, "phi"),
                                       _ptr(u, p.dtype, n, "u"), _ptr(v, p.dtype, n, "v"),
                                       _ptr(w, p.dtype, n, "w"), float(t0), int(nsteps),
                                       _stream(stream)))


def phasefield_noalloc_scratch_bytes() -> int:
    return int(lib.phasefield_noalloc_scratch_bytes())


def phasefield_adjoint_step(h, p: Params, phi_n, u, v, w, t_n, lam, gu=None, gv=None, gw=None,
                            stream=None) -> None:
    n = cells(p)
    _check(lib.phasefield_adjoint_step(
        h, _ptr(phi_n, p.dtype, n, "phi_n"), _ptr(u, p.dtype, n, "u"), _ptr(v, p.dtype, n, "v"),
        _ptr(w, p.dtype, n, "w"), float(t_n), _ptr(lam, p.dtype, n, "lam"),
        _ptr(gu, p.dtype, n, "gu"), _ptr(gv, p.dtype, n, "gv"), _ptr(gw, p.dtype, n, "gw"),
        _stream(stream)))


def phasefield_step_stages(h, p: Params, phi, u, v, w, t, y2=None, y3=None, y4=None,
                           stream=None, phi_next=None) -> None:
    n = cells(p)
    _check(lib.phasefield_step_stages(
        h, _ptr(phi, p.dtype, n, "phi"), _ptr(phi_next, p.dtype, n, "phi_next"),
        _ptr(u, p.dtype, n, "u"), _ptr(v, p.dtype, n, "v"), _ptr(w, p.dtype, n, "w"), float(t),
        _ptr(y2, p.dtype, n, "y2"), _ptr(y3, p.dtype, n, "y3"), _ptr(y4, p.dtype, n, "y4"),
        _stream(stream)))


def phasefield_adjoint_step_stages(h, p: Params, phi_n, y2, y3, y4, u, v, w, t_n, lam, gu=None,
                                   gv=None, gw=None, stream=None) -> None:
    n = cells(p)
    _check(lib.phasefield_adjoint_step_stages(
        h, _ptr(phi_n, p.dtype, n, "phi_n"), _ptr(y2, p.dtype, n, "y2"),
        _ptr(y3, p.dtype, n, "y3"), _ptr(y4, p.dtype, n, "y4"), _ptr(u, p.dtype, n, "u"),
        _ptr(v, p.dtype, n, "v"), _ptr(w, p.dtype, n, "w"), float(t_n),
        _ptr(lam, p.dtype, n, "lam"), _ptr(gu, p.dtype, n, "gu"), _ptr(gv, p.dtype, n, "gv"),
        _ptr(gw, p.dtype, n, "gw"), _stream(stream)))


def phasefield_reduce(h, p: Params, phi, stream=None):
    """(mass, min, max, nonfinite count). Synchronises the stream. A non-finite field is
    reported through the count (the C call's PF_ERR_NONFINITE is not raised)."""
    out = (ctypes.c_double * 4)()
    st = lib.phasefield_reduce(h, _ptr(phi, p.dtype, cells(p), "phi"), out, _stream(stream))
    if st not in (PF_OK, PF_ERR_NONFINITE):
        _check(st)
    return tuple(out)


def phasefield_velocity_from_coeffs(p: Params, modes: int, phases, coeffs, u, v, w,
                                    stream=None) -> None:
    n = cells(p)
    _check(lib.phasefield_velocity_from_coeffs(
        ctypes.byref(p), int(modes), _ptr(phases, PF_F64, 3 * modes, "phases"),
        _ptr(coeffs, PF_F64, 3 * modes ** 3, "coeffs"), _ptr(u, p.dtype, n, "u"),
        _ptr(v, p.dtype, n, "v"), _ptr(w, p.dtype, n, "w"), _stream(stream)))


def phasefield_velocity_coeffs_grad(p: Params, modes: int, phases, gu, gv, gw, coeff_grad,
                                    stream=None) -> None:
    n = cells(p)
    _check(lib.phasefield_velocity_coeffs_grad(
        ctypes.byref(p), int(modes), _ptr(phases, PF_F64, 3 * modes, "phases"),
        _ptr(gu, p.dtype, n, "gu"), _ptr(gv, p.dtype, n, "gv"), _ptr(gw, p.dtype, n, "gw"),
        _ptr(coeff_grad, PF_F64, 3 * modes ** 3, "coeff_grad"), _stream(stream)))


def phasefield_variant_count(dtype=PF_F64) -> int:
    return int(lib.phasefield_variant_count(int(dtype)))


def phasefield_variant_name(dtype, v) -> str | None:
    r = lib.phasefield_variant_name(int(dtype), int(v))
    return None if r is None else r.decode()


def phasefield_autotune(h, reps=5, stream=None, dtype=PF_F64):
    """Returns (best variant, per-variant ms per step) for a handle of storage dtype."""
    nv = lib.phasefield_variant_count(int(dtype))
    times = (ctypes.c_double * max(nv, 1))()
    best = ctypes.c_int32()
    _check(lib.phasefield_autotune(h, int(reps), ctypes.byref(best), times, _stream(stream)))
    return best.value, list(times)[:nv]


def phasefield_solver_variant(h) -> int:
    return int(lib.phasefield_solver_variant(h))


def phasefield_batch_create(params_list) -> ctypes.c_void_p:
    arr = (Params * len(params_list))(*params_list)
    h = ctypes.c_void_p()
    _check(lib.phasefield_batch_create(arr, len(params_list), ctypes.byref(h)))
    return h


def phasefield_batch_step(h, params_list, phis, us, vs, ws, t0s=None, nsteps=1, stream=None):
    B = len(params_list)

    def arr(ts, name):
        return (ctypes.c_void_p * B)(*[_ptr(t, p.dtype, cells(p), name)
                                       for t, p in zip(ts, params_list)])

    t0 = None if t0s is None else (ctypes.c_double * B)(*[float(x) for x in t0s])
    _check(lib.phasefield_batch_step(h, arr(phis, "phi"), arr(us, "u"), arr(vs, "v"),
                                     arr(ws, "w"), t0, int(nsteps), _stream(stream)))


def phasefield_set_spacing(h, params, hx, hy, hz, eps_mode: int = 0) -> None:
    """Cell widths per axis (host sequences of n[0], n[1], n[2] floats), or all None."""
    if hx is None and hy is None and hz is None:
        _check(lib.phasefield_set_spacing(h, None, None, None, int(eps_mode)))
        return
    arrs = []
    for w, n, name in ((hx, params.n[0], "hx"), (hy, params.n[1], "hy"), (hz, params.n[2], "hz")):
        if w is None:
            raise ValueError("give hx, hy and hz, or none")
        vals = [float(x) for x in w]
        if len(vals) != n:
            raise ValueError(f"{name} must hold {n} widths, not {len(vals)}")
        arrs.append((ctypes.c_double * n)(*vals))
    _check(lib.phasefield_set_spacing(h, *[ctypes.cast(a, ctypes.c_void_p) for a in arrs],
                                      int(eps_mode)))


def phasefield_set_adjoint_form(h, form: int) -> None:
    _check(lib.phasefield_set_adjoint_form(h, int(form)))


def phasefield_batch_set_persistent(h, persistent: bool) -> None:
    _check(lib.phasefield_batch_set_persistent(h, int(bool(persistent))))


def phasefield_batch_set_shape(h, shape: int) -> None:
    _check(lib.phasefield_batch_set_shape(h, int(shape)))


def phasefield_batch_autotune(h, reps, stream):
    """(best shape, best persistent flag, list of 6 per-step times in ms, -1 where n/a)."""
    bs, bp = ctypes.c_int32(-1), ctypes.c_int32(-1)
    times = (ctypes.c_double * 6)()
    _check(lib.phasefield_batch_autotune(h, int(reps), ctypes.byref(bs), ctypes.byref(bp), times,
                                         _stream(stream)))
    return int(bs.value), int(bp.value), list(times)


def phasefield_batch_destroy(h) -> None:
    _check(lib.phasefield_batch_destroy(h))


def phasefield_device_copy(dst, src, stream=None) -> None:
    """dst <- src (same dtype and size, contiguous GPU tensors) with the library's copy."""
    if dst.dtype != src.dtype or dst.numel() != src.numel():
        raise ValueError("dst and src must have the same dtype and size")
    nbytes = src.numel() * src.element_size()
    _check(lib.phasefield_device_copy(_ptr(dst, name="dst"), _ptr(src, name="src"), nbytes,
                                      _stream(stream)))


def phasefield_last_error() -> str:
    return lib.phasefield_last_error().decode()
