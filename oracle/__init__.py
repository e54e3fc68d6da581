"""Oracle for the conservative, bounded phase-field step — TEST INFRASTRUCTURE ONLY.

Plain FP64 CPU statement of what the GPU library computes (paper: Mirjalili, Ivey & Mani,
arXiv:1803.01262, Sec. 2.2 five-step recipe, Eqs. 1, 11-13, 18-22, 25-28). Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import this package; the product
path never does, and this package imports nothing from the product.

The arithmetic lives in ``pf_oracle.c`` (plain C, gcc, no SIMD intrinsics, -ffp-contract=off),
loaded with ctypes. ``params`` holds the paper's parameter criteria (Eqs. 8-10, 17, 23-28,
31-32) written out in Python.

Arrays are numpy float64, C-contiguous, shape (nz, ny, nx); face arrays hold the velocity on
the low face of each cell. Every function returns new arrays and leaves its inputs alone.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import params  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (plain -O2, FP contraction off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=gnu11", "-shared",
                        "-fPIC", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("dx", ctypes.c_double), ("eps", ctypes.c_double),
                ("gamma", ctypes.c_double), ("delta", ctypes.c_double),
                ("wall", ctypes.c_int32 * 3)]


_lib = None


def _l():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d = ctypes.c_double
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        gp = ctypes.POINTER(_Grid)
        _lib.orc_rhs.argtypes = [gp, d, p, p, p, p, p]
        _lib.orc_step.argtypes = [gp, ctypes.c_int, ctypes.c_int, d, d, ctypes.c_int, d, i64,
                                  p, p, p, p]
        _lib.orc_euler_coeff_1d.argtypes = [i64, d, d, d, d, d, p, p]
        _lib.orc_euler_coeff.argtypes = [gp, d, d, p, p, p, p, p]
        _lib.orc_reduce.argtypes = [gp, p, p]
        _lib.orc_rhs_vjp.argtypes = [gp, d, p, p, p, p, p, p, p, p, p]
        _lib.orc_adjoint_step.argtypes = [gp, ctypes.c_int, d, d, ctypes.c_int, d, p, p, p, p,
                                          p, p, p, p]
        _lib.orc_velocity_from_coeffs.argtypes = [gp, ctypes.c_int, p, p, p, p, p]
        _lib.orc_velocity_from_coeffs_T.argtypes = [gp, ctypes.c_int, p, p, p, p, p]
        _lib.orc_rhs_nu.argtypes = [gp, p, p, p, ctypes.c_int, d, p, p, p, p, p]
        _lib.orc_step_nu.argtypes = [gp, p, p, p, ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d,
                                     ctypes.c_int, d, i64, p, p, p, p]
        _lib.orc_reduce_nu.argtypes = [gp, p, p, p, p, p]
        _lib.orc_rhs_vjp_nu.argtypes = [gp, p, p, p, ctypes.c_int, d, p, p, p, p, p, p, p, p, p]
        _lib.orc_adjoint_step_nu.argtypes = [gp, p, p, p, ctypes.c_int, ctypes.c_int, d, d,
                                             ctypes.c_int, d, p, p, p, p, p, p, p, p]
        _lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib.orc_max_threads.restype = ctypes.c_int
    return _lib


def set_threads(n: int) -> None:
    """Number of OpenMP threads the oracle's loops use from now on."""
    _l().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_l().orc_max_threads())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


def _grid(shape, dx, eps=0.0, gamma=0.0, delta=0.0, walls=(False, False, False)) -> _Grid:
    nz, ny, nx = shape
    return _Grid(nx, ny, nz, dx, eps, gamma, delta, (ctypes.c_int32 * 3)(*(int(bool(w)) for w in walls)))


def rhs(phi, U, V, W, *, dx, eps, gamma, delta=0.0, s=1.0, walls=(False, False, False)) -> np.ndarray:
    """f = d(phi)/dt of the semi-discrete Eq. 1 (Sec. 2.2 recipe, steps 1-5). walls: per axis
    (x, y, z), solid walls at both ends instead of periodicity (see pf_oracle.c)."""
    phi, U, V, W = map(_f64, (phi, U, V, W))
    f = np.empty_like(phi)
    g = _grid(phi.shape, dx, eps, gamma, delta, walls)
    _l().orc_rhs(ctypes.byref(g), s, _ptr(phi), _ptr(U), _ptr(V), _ptr(W), _ptr(f))
    return f


def _check_scheme(scheme):
    if scheme not in (1, 2, 3, 4):
        raise ValueError(f"scheme must be 1 (Euler), 2 (RK2), 3 (RK3) or 4 (RK4), not {scheme!r}")


def step(phi, U, V, W, *, dx, eps, gamma, dt, nsteps=1, delta=0.0, t0=0.0, scheme=4,
         fp32=False, vel_mode=0, vel_T=1.0, walls=(False, False, False)) -> np.ndarray:
    """nsteps explicit steps (scheme 1: Euler, Eq. 25; scheme 2: explicit midpoint RK2, Eq. 26;
    scheme 3: low-storage RK3, Eq. 27; scheme 4: classic RK4, Eq. 28).

    vel_mode 0: steady velocity; 1: u(x, t) = u0(x) cos(pi t / vel_T). fp32=True rounds every
    stage input and each new phi to float32 (storage precision) while computing in FP64.
    walls: per axis (x, y, z), solid walls at both ends instead of periodicity.
    """
    _check_scheme(scheme)
    out = _f64(phi).copy()
    U, V, W = map(_f64, (U, V, W))
    g = _grid(out.shape, dx, eps, gamma, delta, walls)
    _l().orc_step(ctypes.byref(g), int(scheme), int(bool(fp32)), dt, t0, int(vel_mode),
                  float(vel_T), int(nsteps), _ptr(out), _ptr(U), _ptr(V), _ptr(W))
    return out


def euler_coeff_1d(phi, *, dx, eps, gamma, u, dt) -> np.ndarray:
    """One Euler step in the printed 1D coefficient form (Eq. 13), uniform velocity u."""
    phi = _f64(phi).ravel()
    out = np.empty_like(phi)
    _l().orc_euler_coeff_1d(phi.size, dx, eps, gamma, u, dt, _ptr(phi), _ptr(out))
    return out


def euler_coeff(phi, U, V, W, *, dx, eps, gamma, dt, delta=0.0, s=1.0) -> np.ndarray:
    """One Euler step in the multi-dimensional coefficient form (Eqs. 18-22, three axes)."""
    phi, U, V, W = map(_f64, (phi, U, V, W))
    out = np.empty_like(phi)
    g = _grid(phi.shape, dx, eps, gamma, delta)
    _l().orc_euler_coeff(ctypes.byref(g), s, dt, _ptr(phi), _ptr(U), _ptr(V), _ptr(W), _ptr(out))
    return out


def reduce(phi, *, dx) -> tuple[float, float, float, float]:
    """(mass = sum(phi) dx^D, min, max, number of non-finite cells)."""
    phi = _f64(phi)
    out = np.zeros(4)
    g = _grid(phi.shape, dx)
    _l().orc_reduce(ctypes.byref(g), _ptr(phi), _ptr(out))
    return tuple(float(v) for v in out)


def rhs_vjp(phi, U, V, W, lam, *, dx, eps, gamma, delta=0.0, s=1.0, walls=(False, False, False)):
    """(J^T lam, dU, dV, dW): vector-Jacobian product of rhs() at phi (walls as in rhs())."""
    phi, U, V, W, lam = map(_f64, (phi, U, V, W, lam))
    pb, ub, vb, wb = (np.zeros_like(phi) for _ in range(4))
    g = _grid(phi.shape, dx, eps, gamma, delta, walls)
    _l().orc_rhs_vjp(ctypes.byref(g), s, _ptr(phi), _ptr(U), _ptr(V), _ptr(W), _ptr(lam),
                     _ptr(pb), _ptr(ub), _ptr(vb), _ptr(wb))
    return pb, ub, vb, wb


def adjoint_step(phi, U, V, W, lam, *, dx, eps, gamma, dt, delta=0.0, t=0.0, scheme=4,
                 vel_mode=0, vel_T=1.0, walls=(False, False, False)):
    """Adjoint of one step at phi_n: returns (lam_n, dU, dV, dW) given lam = dL/dphi_{n+1}."""
    _check_scheme(scheme)
    phi, U, V, W = map(_f64, (phi, U, V, W))
    lam = _f64(lam).copy()
    ub, vb, wb = (np.zeros_like(phi) for _ in range(3))
    g = _grid(phi.shape, dx, eps, gamma, delta, walls)
    _l().orc_adjoint_step(ctypes.byref(g), int(scheme), dt, t, int(vel_mode), float(vel_T),
                          _ptr(phi), _ptr(U), _ptr(V), _ptr(W), _ptr(lam), _ptr(ub), _ptr(vb),
                          _ptr(wb))
    return lam, ub, vb, wb


def velocity_from_coeffs(shape, *, dx, phases, coeffs):
    """Face velocity = discrete curl of the separable-mode edge potential (direct sums).

    phases: (3, M); coeffs: (M, M, M, 3) indexed [m3][m2][m1][component].
    """
    phases, coeffs = _f64(phases), _f64(coeffs)
    M = phases.shape[1]
    assert coeffs.shape == (M, M, M, 3)
    U, V, W = (np.empty(shape) for _ in range(3))
    g = _grid(shape, dx)
    _l().orc_velocity_from_coeffs(ctypes.byref(g), M, _ptr(phases), _ptr(coeffs), _ptr(U),
                                  _ptr(V), _ptr(W))
    return U, V, W


def velocity_from_coeffs_T(shape, *, dx, phases, Ubar, Vbar, Wbar) -> np.ndarray:
    """Transpose of velocity_from_coeffs: d<(U,V,W),(Ubar,Vbar,Wbar)>/d coeffs."""
    phases = _f64(phases)
    Ubar, Vbar, Wbar = map(_f64, (Ubar, Vbar, Wbar))
    M = phases.shape[1]
    cb = np.zeros((M, M, M, 3))
    g = _grid(shape, dx)
    _l().orc_velocity_from_coeffs_T(ctypes.byref(g), M, _ptr(phases), _ptr(Ubar), _ptr(Vbar),
                                    _ptr(Wbar), _ptr(cb))
    return cb


def _widths(shape, hx, hy, hz):
    nz, ny, nx = shape
    out = []
    for h, n, name in ((hx, nx, "hx"), (hy, ny, "hy"), (hz, nz, "hz")):
        h = _f64(h).ravel()
        if h.size != n or not np.all(np.isfinite(h)) or not np.all(h > 0):
            raise ValueError(f"{name} must hold {n} positive finite widths")
        out.append(h)
    return out


def rhs_nu(phi, U, V, W, *, hx, hy, hz, dx, eps, gamma, delta=0.0, s=1.0, eps_mode=0,
           walls=(False, False, False)) -> np.ndarray:
    """rhs() on a non-uniform rectilinear mesh with cell widths hx (nx), hy (ny), hz (nz).

    eps_mode 0: eps everywhere; 1: eps * max(h_x, h_y, h_z) / dx per cell (dx the reference
    spacing of eps), averaged onto faces. See pf_oracle.c for the discrete form."""
    phi, U, V, W = map(_f64, (phi, U, V, W))
    h = _widths(phi.shape, hx, hy, hz)
    f = np.empty_like(phi)
    g = _grid(phi.shape, dx, eps, gamma, delta, walls)
    _l().orc_rhs_nu(ctypes.byref(g), *(_ptr(a) for a in h), int(eps_mode), s, _ptr(phi), _ptr(U),
                    _ptr(V), _ptr(W), _ptr(f))
    return f


def step_nu(phi, U, V, W, *, hx, hy, hz, dx, eps, gamma, dt, nsteps=1, delta=0.0, t0=0.0,
            scheme=4, fp32=False, vel_mode=0, vel_T=1.0, eps_mode=0,
            walls=(False, False, False)) -> np.ndarray:
    """step() on a non-uniform rectilinear mesh (widths and eps_mode as rhs_nu)."""
    _check_scheme(scheme)
    out = _f64(phi).copy()
    U, V, W = map(_f64, (U, V, W))
    h = _widths(out.shape, hx, hy, hz)
    g = _grid(out.shape, dx, eps, gamma, delta, walls)
    _l().orc_step_nu(ctypes.byref(g), *(_ptr(a) for a in h), int(eps_mode), int(scheme),
                     int(bool(fp32)), dt, t0, int(vel_mode), float(vel_T), int(nsteps), _ptr(out),
                     _ptr(U), _ptr(V), _ptr(W))
    return out


def rhs_vjp_nu(phi, U, V, W, lam, *, hx, hy, hz, dx, eps, gamma, delta=0.0, s=1.0, eps_mode=0,
               walls=(False, False, False)):
    """(J^T lam, dU, dV, dW): vector-Jacobian product of rhs_nu() at phi."""
    phi, U, V, W, lam = map(_f64, (phi, U, V, W, lam))
    pb, ub, vb, wb = (np.zeros_like(phi) for _ in range(4))
    h = _widths(phi.shape, hx, hy, hz)
    g = _grid(phi.shape, dx, eps, gamma, delta, walls)
    _l().orc_rhs_vjp_nu(ctypes.byref(g), *(_ptr(a) for a in h), int(eps_mode), s, _ptr(phi),
                        _ptr(U), _ptr(V), _ptr(W), _ptr(lam), _ptr(pb), _ptr(ub), _ptr(vb),
                        _ptr(wb))
    return pb, ub, vb, wb


def adjoint_step_nu(phi, U, V, W, lam, *, hx, hy, hz, dx, eps, gamma, dt, delta=0.0, t=0.0,
                    scheme=4, vel_mode=0, vel_T=1.0, eps_mode=0, walls=(False, False, False)):
    """adjoint_step() on a non-uniform mesh (widths and eps_mode as rhs_nu)."""
    _check_scheme(scheme)
    phi, U, V, W = map(_f64, (phi, U, V, W))
    lam = _f64(lam).copy()
    ub, vb, wb = (np.zeros_like(phi) for _ in range(3))
    h = _widths(phi.shape, hx, hy, hz)
    g = _grid(phi.shape, dx, eps, gamma, delta, walls)
    _l().orc_adjoint_step_nu(ctypes.byref(g), *(_ptr(a) for a in h), int(eps_mode), int(scheme),
                             dt, t, int(vel_mode), float(vel_T), _ptr(phi), _ptr(U), _ptr(V),
                             _ptr(W), _ptr(lam), _ptr(ub), _ptr(vb), _ptr(wb))
    return lam, ub, vb, wb


def reduce_nu(phi, *, hx, hy, hz) -> tuple[float, float, float, float]:
    """(sum(phi * cell volume), min, max, number of non-finite cells) on a non-uniform mesh."""
    phi = _f64(phi)
    h = _widths(phi.shape, hx, hy, hz)
    out = np.zeros(4)
    g = _grid(phi.shape, 1.0)
    _l().orc_reduce_nu(ctypes.byref(g), *(_ptr(a) for a in h), _ptr(phi), _ptr(out))
    return tuple(float(v) for v in out)
