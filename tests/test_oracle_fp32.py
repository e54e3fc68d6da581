"""Pins of the oracle's FP32-storage mode (no GPU).

In this mode the oracle computes in FP64 but rounds every value that a GPU run stores in float32
(each RK stage input and the new phi) to the nearest float32, ties to even. Every FP32 parity bar
of the GPU tests is taken against this mode, so it is tied here to things other than itself:

* each output is a float32 number;
* an independent statement of the four integrators (Euler, Eq. 25 regime; explicit midpoint RK2;
  the low-storage RK3; classic RK4 — the stage definitions of Sec. 2.3), written here with numpy
  from the right-hand side ``oracle.rhs`` (pinned against the printed coefficient forms
  elsewhere), rounds at exactly those points and agrees bit for bit; the same statement without
  the stage-input rounding does not, so a dropped rounding is seen;
* for gamma = 0 and a uniform velocity a Fourier mode is multiplied each step by the textbook
  amplification factor R(z) (Eq. 3 with gamma = 0); in FP32 storage the result stays within the
  rounding bound (stages + 1) n 2^-24 max|phi| of R(z)^n, while the FP64 mode matches R(z)^n
  to 1e-14 (so a mode that stopped rounding would be seen too);
* mass is conserved to the float32 level: each stored value moves by at most half an ulp, so
  |M_n - M_0| <= (stages + 1) n N 2^-25 max|phi| dV;
* the complement symmetry of Eq. 16 holds to the same level.
"""
import math

import numpy as np
import pytest

import oracle
import pf_fixtures as fx

U32 = 2.0 ** -24  # unit roundoff of float32


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def random_case(seed, shape):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    dx = 1.0 / max(shape)
    phi = f32(rng.uniform(0.0, 1.0, size=shape))
    U, V, W = fx.random_edge_faces(rng, shape, dx)
    s = 1.0 / fx.max_face_speed(U, V, W)
    U, V, W = (f32(a * s) for a in (U, V, W))
    return phi, U, V, W, dx


def numpy_step(phi, U, V, W, *, dx, eps, gamma, dt, nsteps, scheme, round_stages=True,
               round_output=True, vel_mode=0, vel_T=1.0):
    """The integrators of Sec. 2.3 in FP64 with float32 storage, stated from their definitions:
    rounding of each stage input (round_stages) and of each new phi (round_output)."""
    rs = f32 if round_stages else (lambda a: a)
    ro = f32 if round_output else (lambda a: a)

    def f(y, t):
        s = math.cos(math.pi * t / vel_T) if vel_mode == 1 else 1.0
        return oracle.rhs(y, U, V, W, dx=dx, eps=eps, gamma=gamma, s=s)

    phi = np.array(phi, dtype=np.float64)
    for n in range(nsteps):
        t = n * dt
        if scheme == 1:
            phi = ro(phi + dt * f(phi, t))
        elif scheme == 2:
            k1 = f(phi, t)
            y = rs(phi + 0.5 * dt * k1)
            phi = ro(phi + dt * f(y, t + 0.5 * dt))
        elif scheme == 3:
            # Wray's low-storage form: u1 = u0 + dt g1 k1, u2 = u1 + dt (g2 k2 + z2 k1),
            # u3 = u2 + dt (g3 k3 + z3 k2); stage times t, t + g1 dt, t + (g1 + g2 + z2) dt
            g1, g2, g3, z2, z3 = 8.0 / 15.0, 5.0 / 12.0, 0.75, -17.0 / 60.0, -5.0 / 12.0
            k1 = f(phi, t)
            u1 = rs(phi + dt * g1 * k1)
            k2 = f(u1, t + g1 * dt)
            u2 = rs(u1 + dt * (g2 * k2 + z2 * k1))
            k3 = f(u2, t + (g1 + g2 + z2) * dt)
            phi = ro(u2 + dt * (g3 * k3 + z3 * k2))
        else:
            k1 = f(phi, t)
            k2 = f(rs(phi + 0.5 * dt * k1), t + 0.5 * dt)
            k3 = f(rs(phi + 0.5 * dt * k2), t + 0.5 * dt)
            k4 = f(rs(phi + dt * k3), t + dt)
            phi = ro(phi + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4))
    return phi


@pytest.mark.parametrize("scheme", [1, 2, 3, 4])
def test_fp32_outputs_are_float32(scheme):
    phi, U, V, W, dx = random_case(0, (6, 7, 9))
    out = oracle.step(phi, U, V, W, dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, nsteps=5,
                      scheme=scheme, fp32=True)
    assert np.array_equal(out, f32(out))
    # and the FP64 mode is not (the rounding is the mode's, not the input's)
    out64 = oracle.step(phi, U, V, W, dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, nsteps=5,
                        scheme=scheme, fp32=False)
    assert not np.array_equal(out64, f32(out64))


@pytest.mark.parametrize("scheme", [1, 2, 3, 4])
@pytest.mark.parametrize("vel_mode", [0, 1])
def test_fp32_mode_bitwise_equals_independent_statement(scheme, vel_mode):
    phi, U, V, W, dx = random_case(1, (5, 8, 7))
    kw = dict(dx=dx, eps=dx, gamma=1.3, dt=0.1 * dx, nsteps=6, scheme=scheme,
              vel_mode=vel_mode, vel_T=0.05)
    out = oracle.step(phi, U, V, W, fp32=True, **kw)
    ref = numpy_step(phi, U, V, W, **kw)
    assert np.array_equal(out, ref)
    if scheme > 1:
        # a driver that forgets to round the stage inputs gives other bits: the test sees it
        bad = numpy_step(phi, U, V, W, round_stages=False, **kw)
        assert not np.array_equal(out, bad)
    # likewise one that rounds only the stage inputs
    bad = numpy_step(phi, U, V, W, round_output=False, **kw)
    assert not np.array_equal(out, bad)


@pytest.mark.parametrize("scheme,stages", [(2, 2), (3, 3), (4, 4)])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fp32_gamma0_amplification_within_rounding_bound(scheme, stages, axis):
    """gamma = 0, uniform u along one axis: phi = 1/2 + A cos(k x) advances by the textbook
    amplification R(z) per step, z = -i u dt sin(k dx)/dx; FP32 storage stays within
    (stages + 1) n 2^-24 max|phi| of it (each step rounds `stages` stage inputs and phi once,
    and |R| <= 1 does not amplify earlier roundings)."""
    n_cells, m, nsteps = 16, 3, 40
    dx = 1.0 / n_cells
    shape = [1, 1, 1]
    shape[2 - axis] = n_cells
    x = np.arange(n_cells) * dx
    k = 2 * np.pi * m
    amp = 0.3
    phi0 = f32(0.5 + amp * np.cos(k * x)).reshape(shape)
    vel = [np.zeros(shape) for _ in range(3)]
    u = 0.75
    vel[axis][:] = u
    dt = 0.5 * dx
    out = oracle.step(phi0, *vel, dx=dx, eps=dx, gamma=0.0, dt=dt, nsteps=nsteps, scheme=scheme,
                      fp32=True).ravel()
    # exact evolution of the (rounded) initial data, mode by mode
    z = -1j * u * dt * np.sin(2 * np.pi * np.fft.fftfreq(n_cells)) / dx
    if scheme == 4:
        R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    else:  # RK2 and RK3 polynomials for the linear problem
        R = 1 + z + z ** 2 / 2 + (z ** 3 / 6 if scheme == 3 else 0)
    exact = np.real(np.fft.ifft(np.fft.fft(phi0.ravel()) * R ** nsteps))
    bound = (stages + 1) * nsteps * U32 * np.abs(phi0).max()
    err = np.abs(out - exact).max()
    assert err <= bound, (err, bound)
    assert err > 1e-13  # rounding happened (the FP64 mode matches to 1e-14)
    out64 = oracle.step(phi0, *vel, dx=dx, eps=dx, gamma=0.0, dt=dt, nsteps=nsteps,
                        scheme=scheme).ravel()
    assert np.abs(out64 - exact).max() <= 1e-14


@pytest.mark.parametrize("scheme,stages", [(1, 1), (2, 2), (3, 3), (4, 4)])
def test_fp32_mass_conserved_to_float32_level(scheme, stages):
    phi, U, V, W, dx = random_case(2, (8, 9, 10))
    nsteps = 20
    out = oracle.step(phi, U, V, W, dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, nsteps=nsteps,
                      scheme=scheme, fp32=True)
    m0 = oracle.reduce(phi, dx=dx)[0]
    m1 = oracle.reduce(out, dx=dx)[0]
    bound = (stages + 1) * nsteps * phi.size * 0.5 * U32 * 1.0 * dx ** 3
    assert abs(m1 - m0) <= bound, (abs(m1 - m0), bound)
    assert abs(m1 - m0) > 0.0  # storage rounding moved the mass (FP64 keeps it to ~1e-16)


@pytest.mark.parametrize("scheme,stages", [(2, 2), (4, 4)])
def test_fp32_complement_symmetry_to_float32_level(scheme, stages):
    """Eq. 16: step(1 - phi) = 1 - step(phi) for a solenoidal field; in FP32 storage each of the
    two runs is within its rounding of the exact one, so they agree to twice that bound."""
    phi, U, V, W, dx = random_case(3, (7, 6, 8))
    nsteps = 10
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, nsteps=nsteps, scheme=scheme, fp32=True)
    a = oracle.step(phi, U, V, W, **kw)
    b = oracle.step(f32(1.0 - phi), U, V, W, **kw)
    err = np.abs((1.0 - b) - a).max()
    assert err <= 2 * (stages + 1) * nsteps * U32, err
