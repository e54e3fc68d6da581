"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test ties the oracle to something other than itself: the printed coefficient forms
(Eqs. 13, 18-22), telescoping conservation, the complement symmetry of Eq. 16, the Euler
boundedness theorem of Sec. 2.2, the analytic tanh equilibrium (Sec. 1), the textbook RK2 and RK4
amplification factors for pure advection (Eq. 3 with gamma = 0), the boundedness of RK2 at its
Eq. 26 step above the crossover line (Sec. 2.3, Fig. 6), shift equivariance and the printed
parameter criteria.
"""
import math

import numpy as np
import pytest

import oracle
import pf_fixtures as fx
from oracle import params

EPS64 = np.finfo(np.float64).eps


def rand_phi(rng, shape):
    return rng.uniform(0.0, 1.0, size=shape)


def solenoidal(rng, shape, dx, umax=1.0):
    U, V, W = fx.random_edge_faces(rng, shape, dx)
    if shape[0] == 1:  # 2D: keep the field in-plane (only Az), so W = 0
        zero = np.zeros(shape)
        Az = rng.standard_normal(shape) * dx
        U, V, W = fx.edge_curl(zero, zero, Az, dx)
    s = umax / fx.max_face_speed(U, V, W)
    return U * s, V * s, W * s


# --------------------------------------------------------------------- coefficient forms


def test_flux_form_matches_eq13_1d():
    """Euler step of the flux form == printed 1D coefficient form (Eq. 13, sign per Eq. 13)."""
    rng = np.random.default_rng(0)
    for trial in range(20):
        n = int(rng.integers(5, 40))
        dx = 1.0 / n
        eps = dx * rng.uniform(0.5, 2.0)
        gamma = rng.uniform(0.2, 3.0)
        u = rng.uniform(-1.5, 1.5)
        dt = 0.3 * dx * dx / (gamma * eps)
        phi = rand_phi(rng, (1, 1, n))
        U = np.full((1, 1, n), u)
        Z = np.zeros((1, 1, n))
        flux = oracle.step(phi, U, Z, Z, dx=dx, eps=eps, gamma=gamma, dt=dt, scheme=1)
        coef = oracle.euler_coeff_1d(phi, dx=dx, eps=eps, gamma=gamma, u=u, dt=dt)
        np.testing.assert_allclose(flux.ravel(), coef, rtol=0, atol=2e-15)


@pytest.mark.parametrize("shape", [(1, 12, 10), (6, 7, 8), (1, 9, 1), (5, 1, 1)])
def test_flux_form_matches_eqs18_22(shape):
    """Euler step of the flux form == multi-D coefficient form (Eqs. 18, 19, 21, 22)."""
    rng = np.random.default_rng(1)
    dx = 0.1
    for trial in range(5):
        eps, gamma, s = dx * rng.uniform(0.5, 2), rng.uniform(0.3, 2.0), rng.uniform(-1, 1)
        dt = 0.2 * dx * dx / (gamma * eps)
        phi = rand_phi(rng, shape)
        U, V, W = solenoidal(rng, shape, dx)
        vm = 0
        flux = oracle.step(phi, U * s, V * s, W * s, dx=dx, eps=eps, gamma=gamma, dt=dt,
                           scheme=1, vel_mode=vm)
        coef = oracle.euler_coeff(phi, U, V, W, dx=dx, eps=eps, gamma=gamma, dt=dt, s=s)
        np.testing.assert_allclose(flux, coef, rtol=0, atol=5e-15)


def test_eq19_divergence_term():
    """With a non-solenoidal field the centre coefficient keeps the divergence term of Eq. 19,
    and the flux form still matches the coefficient form."""
    rng = np.random.default_rng(2)
    shape, dx = (4, 5, 6), 0.2
    phi = rand_phi(rng, shape)
    U, V, W = (rng.uniform(-1, 1, size=shape) for _ in range(3))
    flux = oracle.step(phi, U, V, W, dx=dx, eps=0.2, gamma=1.0, dt=0.005, scheme=1)
    coef = oracle.euler_coeff(phi, U, V, W, dx=dx, eps=0.2, gamma=1.0, dt=0.005)
    np.testing.assert_allclose(flux, coef, rtol=0, atol=5e-15)


# --------------------------------------------------------------------- conservation


@pytest.mark.parametrize("scheme", [2, 3, 4])
@pytest.mark.parametrize("solenoidal_field", [True, False])
def test_mass_conserved_to_roundoff(solenoidal_field, scheme):
    """Sum of f telescopes to zero for any face velocity (Sec. 2.2 flux form)."""
    rng = np.random.default_rng(3)
    shape, dx = (12, 10, 14), 1.0 / 14
    phi = fx.drops_ic(shape, dx, [(0.5, 0.4, 0.5)], [0.25], dx)
    if solenoidal_field:
        U, V, W = solenoidal(rng, shape, dx)
    else:
        U, V, W = (rng.uniform(-1, 1, size=shape) for _ in range(3))
    m0 = oracle.reduce(phi, dx=dx)[0]
    # within both schemes' 3D limits (Eq. 26: dx/6 here; Eq. 28: 0.23 dx)
    out = oracle.step(phi, U, V, W, dx=dx, eps=dx, gamma=1.0, dt=0.15 * dx, nsteps=50,
                      scheme=scheme)
    m1 = oracle.reduce(out, dx=dx)[0]
    assert abs(m1 - m0) / m0 < 1e-12
    f = oracle.rhs(phi, U, V, W, dx=dx, eps=dx, gamma=1.0)
    assert abs(f.sum()) < 1e-12 * np.abs(f).sum()


# --------------------------------------------------------------------- complement symmetry


@pytest.mark.parametrize("scheme", [1, 2, 3, 4])
def test_complement_symmetry(scheme):
    """step(1 - phi) == 1 - step(phi) for a discretely solenoidal field (Eq. 16, Sec. 2.2.2)."""
    rng = np.random.default_rng(4)
    shape, dx = (8, 9, 10), 0.1
    phi = fx.drops_ic(shape, dx, [(0.4, 0.5, 0.4)], [0.3], dx) * 0.7 + 0.3 * rand_phi(rng, shape)
    U, V, W = solenoidal(rng, shape, dx)
    kw = dict(dx=dx, eps=dx, gamma=1.2, dt=0.15 * dx, nsteps=5, scheme=scheme)
    a = oracle.step(phi, U, V, W, **kw)
    b = oracle.step(1.0 - phi, U, V, W, **kw)
    np.testing.assert_allclose(1.0 - b, a, rtol=0, atol=1e-13)
    # a non-solenoidal field breaks the symmetry (the test has teeth)
    U2 = U + 0.3 * rng.uniform(-1, 1, size=shape)
    a = oracle.step(phi, U2, V, W, **kw)
    b = oracle.step(1.0 - phi, U2, V, W, **kw)
    assert np.abs(1.0 - b - a).max() > 1e-6


# --------------------------------------------------------------------- boundedness theorem


def _bounded_trial(rng, margin_lo, margin_hi, dims):
    shape = (6, 6, 6) if dims == 3 else (1, 7, 7)
    dx = 1.0 / shape[-1]
    phi = rand_phi(rng, shape)
    # sharp 0/1 cells make the theorem's extreme cases more likely
    mask = rng.uniform(size=shape)
    phi[mask < 0.2] = 0.0
    phi[mask > 0.8] = 1.0
    U, V, W = solenoidal(rng, shape, dx, umax=rng.uniform(0.2, 2.0))
    umax = fx.max_face_speed(U, V, W)
    gamma = umax * rng.uniform(0.3, 4.0)
    eps = dx * (params.crossover_eps_over_dx(gamma / umax) + rng.uniform(margin_lo, margin_hi))
    dt = params.dt_max("euler", dims, dx, gamma, eps)
    out = oracle.step(phi, U, V, W, dx=dx, eps=eps, gamma=gamma, dt=dt, scheme=1)
    return out.min(), out.max()


@pytest.mark.parametrize("dims", [2, 3])
def test_euler_boundedness_theorem(dims):
    """Above the crossover line (Eq. 17, with the face-component speed) and at the Euler
    limit (Eq. 25), one step keeps phi in [0, 1] up to rounding (Eqs. 18-22)."""
    rng = np.random.default_rng(10 + dims)
    worst = 0.0
    for trial in range(3000):
        lo, hi = _bounded_trial(rng, 0.0, 0.5 if trial % 2 else 0.0, dims)
        worst = max(worst, -lo, hi - 1.0)
    assert worst <= 4 * EPS64, worst


def test_below_crossover_can_leave_bounds():
    """Negative control: well below the line the same trials do leave [0, 1] (Sec. 2.2.1)."""
    rng = np.random.default_rng(7)
    worst = 0.0
    for trial in range(300):
        lo, hi = _bounded_trial(rng, -0.45, -0.35, 2)
        worst = max(worst, -lo, hi - 1.0)
    assert worst > 1e-3


# --------------------------------------------------------------------- tanh equilibrium


def test_tanh_profile_is_discrete_equilibrium():
    """u = 0: diffusion and sharpening balance for phi = (1 + tanh(x / 2 eps)) / 2 (Sec. 1); the
    face residual of the central scheme is -gamma eps dx^2 Phi'''/12, so max|f| falls ~4x per
    halving of dx at fixed eps. A wrong sign or weight leaves an O(1/eps) residual."""
    eps, D, L = 0.02, 1.0, 2.0
    res = []
    for n in (200, 400, 800, 1600):
        dx = L / n
        x = (np.arange(n) + 0.5) * dx
        d = np.abs(x - L / 2)
        phi = fx.tanh_profile(D / 2 - d, eps).reshape(1, 1, n)
        Z = np.zeros_like(phi)
        f = oracle.rhs(phi, Z, Z, Z, dx=dx, eps=eps, gamma=1.0)
        res.append(np.abs(f).max())
    ratios = [res[i] / res[i + 1] for i in range(len(res) - 1)]
    assert all(3.6 < r < 4.4 for r in ratios[1:]), (res, ratios)
    assert res[-1] < 2e-3 / eps  # far below the O(1/eps) size of either term alone


# --------------------------------------------------------------------- pure advection


@pytest.mark.parametrize("scheme", [2, 3, 4])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_gamma0_rk_amplification(axis, scheme):
    """gamma = 0, uniform u: a sampled Fourier mode is multiplied per step by the scheme's
    stability polynomial, z = -i u dt sin(k dx)/dx (Eq. 3 with gamma = 0): RK4
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24; any three-stage third-order scheme (the RK3)
    1 + z + z^2/2 + z^3/6; the explicit midpoint rule R(z) = 1 + z + z^2/2."""
    n, m, u, dx = 24, 3, 0.8, 1.0 / 24
    dt = 0.4 * dx / u
    k = 2 * np.pi * m
    x = (np.arange(n) + 0.5) * dx
    shape = [1, 1, 1]
    shape[2 - axis] = n
    phi = np.cos(k * x).reshape(shape)
    vel = [np.zeros(shape) for _ in range(3)]
    vel[axis][:] = u
    nsteps = 7
    out = oracle.step(phi, *vel, dx=dx, eps=dx, gamma=0.0, dt=dt, nsteps=nsteps, scheme=scheme)
    z = -1j * u * dt * np.sin(k * dx) / dx
    R = sum(z ** m / math.factorial(m) for m in range(scheme + 1))
    exact = np.real(R ** nsteps * np.exp(1j * k * x)).reshape(shape)
    np.testing.assert_allclose(out, exact, rtol=0, atol=1e-14)


def test_time_factor_cos_reversal():
    """u(x, t) = u0(x) cos(pi t / T) at the RK4 stage times: with gamma = 0 and a uniform
    field, one step equals one step of a steady field whose stage values are the cosines."""
    n, dx, T = 16, 1.0 / 16, 0.7
    rng = np.random.default_rng(8)
    phi = rand_phi(rng, (1, 1, n))
    U = np.full((1, 1, n), 0.9)
    Z = np.zeros_like(U)
    t0, dt = 0.13, 0.01
    got = oracle.step(phi, U, Z, Z, dx=dx, eps=dx, gamma=0.0, dt=dt, t0=t0, vel_mode=1, vel_T=T)
    # by hand: k_s = -s_s D phi_s with D the linear central advection operator
    D = lambda p: oracle.rhs(p, U, Z, Z, dx=dx, eps=dx, gamma=0.0)  # noqa: E731
    s = [math.cos(math.pi * t / T) for t in (t0, t0 + dt / 2, t0 + dt / 2, t0 + dt)]
    k1 = s[0] * D(phi)
    k2 = s[1] * D(phi + dt / 2 * k1)
    k3 = s[2] * D(phi + dt / 2 * k2)
    k4 = s[3] * D(phi + dt * k3)
    np.testing.assert_allclose(got, phi + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4), atol=1e-15)


def test_time_factor_cos_reversal_rk2():
    """The same for the explicit midpoint rule: s at t for the half step and at t + dt/2 for
    the whole step (a stage time of t or t + dt would differ at O(dt^2))."""
    n, dx, T = 16, 1.0 / 16, 0.7
    rng = np.random.default_rng(18)
    phi = rand_phi(rng, (1, 1, n))
    U = np.full((1, 1, n), 0.9)
    Z = np.zeros_like(U)
    t0, dt = 0.13, 0.01
    got = oracle.step(phi, U, Z, Z, dx=dx, eps=dx, gamma=0.0, dt=dt, t0=t0, vel_mode=1,
                      vel_T=T, scheme=2)
    D = lambda p: oracle.rhs(p, U, Z, Z, dx=dx, eps=dx, gamma=0.0)  # noqa: E731
    s0, s1 = math.cos(math.pi * t0 / T), math.cos(math.pi * (t0 + dt / 2) / T)
    want = phi + dt * s1 * D(phi + dt / 2 * s0 * D(phi))
    np.testing.assert_allclose(got, want, atol=1e-15)
    wrong = phi + dt * math.cos(math.pi * (t0 + dt) / T) * D(phi + dt / 2 * s0 * D(phi))
    assert np.abs(wrong - got).max() > 1e-7


# --------------------------------------------------------------------- equivariance, dims


def test_shift_equivariance_bitwise():
    rng = np.random.default_rng(9)
    shape, dx = (7, 8, 9), 0.1
    phi = rand_phi(rng, shape)
    U, V, W = solenoidal(rng, shape, dx)
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, nsteps=3)
    ref = oracle.step(phi, U, V, W, **kw)
    sh = (2, -3, 5)
    r = lambda a: np.roll(a, sh, axis=(0, 1, 2))  # noqa: E731
    got = oracle.step(r(phi), r(U), r(V), r(W), **kw)
    assert np.array_equal(got, r(ref))


def test_2d_as_z_invariant_3d():
    """A 2D problem (nz = 1) equals every plane of the same problem replicated along z."""
    rng = np.random.default_rng(10)
    dx = 0.1
    phi2 = rand_phi(rng, (1, 8, 9))
    U2, V2, W2 = solenoidal(rng, (1, 8, 9), dx)
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.1 * dx, nsteps=4)
    a = oracle.step(phi2, U2, V2, W2, **kw)
    rep = lambda x: np.repeat(x, 5, axis=0)  # noqa: E731
    b = oracle.step(rep(phi2), rep(U2), rep(V2), rep(W2), **kw)
    for k in range(5):
        np.testing.assert_allclose(b[k], a[0], rtol=0, atol=1e-15)


# --------------------------------------------------------------------- reduce


def test_reduce_closed_forms():
    shape, dx = (4, 5, 6), 0.25
    c = np.full(shape, 0.375)
    mass, mn, mx, bad = oracle.reduce(c, dx=dx)
    assert mass == 0.375 * 120 * dx ** 3 and mn == mx == 0.375 and bad == 0
    c[1, 2, 3] = np.nan
    c[0, 0, 0] = -0.5
    c[3, 4, 5] = 2.0
    mass, mn, mx, bad = oracle.reduce(c, dx=dx)
    assert (mn, mx, bad) == (-0.5, 2.0, 1.0)
    assert mass == pytest.approx((0.375 * 117 - 0.5 + 2.0) * dx ** 3, rel=1e-15)
    m2 = oracle.reduce(np.ones((1, 3, 4)), dx=0.5)[0]
    assert m2 == 12 * 0.25  # 2D cell area


# --------------------------------------------------------------------- parameter criteria


def test_eq6_equivalent_to_eq5_and_eq7_minimum():
    rng = np.random.default_rng(11)
    for _ in range(2000):
        beta = rng.uniform(0.05, 5.0)
        kdx = rng.uniform(1e-3, np.pi)
        bound = params.alpha_bound_eq6(beta, kdx)
        assert params.euler_amplification(bound * (1 - 1e-9), beta, kdx) <= 1 + 1e-12
        assert params.euler_amplification(bound * (1 + 1e-6), beta, kdx) > 1
    for beta in (0.2, 0.7, 1.0, 1.6, 4.0):
        ks = np.linspace(1e-6, np.pi, 20001)
        assert min(params.alpha_bound_eq6(beta, k) for k in ks) == pytest.approx(
            params.alpha_bound_eq7(beta), rel=1e-6)


def test_eq10_is_eq8_on_the_crossover_line():
    for g_over_u in (0.5, 1.0, 2.5):
        u, dx = 1.3, 0.01
        gamma = g_over_u * u
        eps = params.crossover_eps_over_dx(g_over_u) * dx
        assert params.dt_mod_1d(dx, gamma, eps, u) == pytest.approx(
            params.dt_mod_max_eq10(dx, u, gamma), rel=1e-12)


def test_table2_classification_by_eq23(tmp_path):
    """Sec. 3.2.1: the relaxed line of Eq. 23 lies below point 5 and above points 6 and 7;
    points 1-5 stayed bounded, 6-7 did not (Table 2). u = v = sqrt(2)/2, |u| = 1."""
    import json
    import os
    pts = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
    comp = math.sqrt(2) / 2
    for p in pts["points"]:
        m = params.margin_eq24(p["eps_over_dx"], 1.0, p["gamma_over_u"], comp)
        assert (m >= 0) == p["bounded"], (p, m)
    # Eq. 17 (with |u|_max = 1) classifies point 5 as below the line
    assert params.margin_eq17(0.9, 1.0, 0.9, 1.0) < 0


def test_table1_interface_error_of_tanh_ic():
    """E_eps of Table 1 (mean-over-cells L1 distance of the initial drop to the top hat) for the
    tanh initial condition on the dx = D/25 grid, within 4% of every printed value."""
    import json
    import os
    pts = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
    n, L = 50, 2.0
    dx = L / n
    x = (np.arange(n) + 0.5) * dx
    r = np.sqrt((x[None, :] - 1) ** 2 + (x[:, None] - 1) ** 2)
    th = (r < 0.5).astype(float)
    for p in pts["points"]:
        eps = p["eps_over_dx"] * dx
        phi = fx.drops_ic((1, n, n), dx, [(1.0, 1.0, 0.0)], [0.5], eps, window=False)[0]
        e_eps = np.abs(phi - th).mean()
        assert e_eps == pytest.approx(p["E_eps"], rel=0.04), (p, e_eps)


def test_table2_classification_reproduced_by_the_stepper():
    """Whole RK4 stepper on the 2D uniform-translation test of Sec. 3.2.1 (D = 1 drop, 2 x 2
    periodic box, dx = D/25, (u, v) = (sqrt2/2, sqrt2/2), T = 2 sqrt2, dt = min(Eq. 31, Eq. 32)):
    checked after every step, points 1-5 stay inside [0, 1] and points 6-7 leave it (Table 2)."""
    import json
    import os
    pts = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
    n, L = 50, 2.0
    dx = L / n
    u = math.sqrt(2) / 2
    U = np.full((1, n, n), u)
    Z = np.zeros_like(U)
    T = 2 * math.sqrt(2)
    for p in pts["points"]:
        eps, gamma = p["eps_over_dx"] * dx, p["gamma_over_u"]
        phi = fx.drops_ic((1, n, n), dx, [(1.0, 1.0, 0.0)], [0.5], eps, window=False)
        dt = min(params.dt_rk4_2d_eq31(dx, gamma, eps), params.dt_rk4_2d_eq32(dx, u, u, gamma))
        ns = math.ceil(T / dt)
        dt = T / ns
        lo, hi = 1.0, 0.0
        for s in range(ns):
            phi = oracle.step(phi, U, U, Z, dx=dx, eps=eps, gamma=gamma, dt=dt)
            lo, hi = min(lo, phi.min()), max(hi, phi.max())
        bounded = lo >= -EPS64 and hi <= 1 + EPS64
        assert bounded == p["bounded"], (p["point"], lo, hi)


# --------------------------------------------------------------------- RK2 boundedness


def _drop_1d_extremes(eps_over_dx, gamma_over_u, scheme_name, scheme):
    """1D drop of diameter 1 advected by u = 1 for one period in [0, 2) (Sec. 2.1, Fig. 1),
    n = 50, tanh interfaces, dt = the scheme's diffusion limit (Eqs. 25-28) rounded down to a
    whole number of steps; returns the extremes of phi over the run."""
    n, L, u = 50, 2.0, 1.0
    dx = L / n
    eps, gamma = eps_over_dx * dx, gamma_over_u * u
    x = (np.arange(n) + 0.5) * dx
    phi = fx.tanh_profile(0.5 - np.abs(x - L / 2), eps).reshape(1, 1, n)
    U = np.full_like(phi, u)
    Z = np.zeros_like(phi)
    nsteps = math.ceil(L / u / params.dt_max(scheme_name, 1, dx, gamma, eps))
    lo, hi = 1.0, 0.0
    for _ in range(nsteps):
        phi = oracle.step(phi, U, Z, Z, dx=dx, eps=eps, gamma=gamma, dt=L / u / nsteps,
                          scheme=scheme)
        lo, hi = min(lo, phi.min()), max(hi, phi.max())
    return lo, hi


@pytest.mark.parametrize("eps_over_dx,gamma_over_u", [(1.0, 1.0), (0.75, 2.0), (1.5, 1.0),
                                                       (2.0, 0.5)])
def test_rk2_at_eq26_bounded_on_and_above_the_crossover_line(eps_over_dx, gamma_over_u):
    """Sec. 2.3 and Fig. 6(a): with the explicit midpoint rule at its diffusive limit (Eq. 26),
    points on or above the crossover line (Eq. 9) keep phi in [0, 1] for a whole period."""
    assert eps_over_dx >= params.crossover_eps_over_dx(gamma_over_u) - 1e-12
    lo, hi = _drop_1d_extremes(eps_over_dx, gamma_over_u, "rk2", 2)
    assert lo >= -EPS64 and hi <= 1 + EPS64, (lo, hi)


@pytest.mark.parametrize("eps_over_dx,gamma_over_u", [(0.55, 1.0), (0.8, 0.5)])
def test_rk2_below_the_crossover_line_leaves_bounds(eps_over_dx, gamma_over_u):
    """Negative control: below the line the same runs leave [0, 1] (Fig. 6(a))."""
    assert eps_over_dx < params.crossover_eps_over_dx(gamma_over_u)
    lo, hi = _drop_1d_extremes(eps_over_dx, gamma_over_u, "rk2", 2)
    assert lo < -1e-3 and hi > 1 + 1e-3, (lo, hi)


def test_rk3_stage_times_and_eq27_factor():
    """The RK3's stage times (the velocity factor at t, t + 8dt/15, t + 2dt/3, with a wrong-time
    negative control), and Eq. 27's 2.51: the real-axis stability limit of its polynomial
    1 + z + z^2/2 + z^3/6 (the largest diffusive eigenvalue is -4 D_f gamma eps / dx^2)."""
    n, dx, T = 16, 1.0 / 16, 0.7
    rng = np.random.default_rng(28)
    phi = rand_phi(rng, (1, 1, n))
    U = np.full((1, 1, n), 0.9)
    Z = np.zeros_like(U)
    t0, dt = 0.13, 0.01
    got = oracle.step(phi, U, Z, Z, dx=dx, eps=dx, gamma=0.0, dt=dt, t0=t0, vel_mode=1,
                      vel_T=T, scheme=3)
    D = lambda p: oracle.rhs(p, U, Z, Z, dx=dx, eps=dx, gamma=0.0)  # noqa: E731
    s = [math.cos(math.pi * (t0 + c * dt) / T) for c in (0.0, 8 / 15, 2 / 3)]
    k1 = s[0] * D(phi)
    u1 = phi + dt * 8 / 15 * k1
    k2 = s[1] * D(u1)
    u2 = u1 + dt * (5 / 12 * k2 - 17 / 60 * k1)
    k3 = s[2] * D(u2)
    np.testing.assert_allclose(got, u2 + dt * (3 / 4 * k3 - 5 / 12 * k2), atol=1e-15)
    k3w = math.cos(math.pi * (t0 + dt / 2) / T) * D(u2)
    assert np.abs(u2 + dt * (3 / 4 * k3w - 5 / 12 * k2) - got).max() > 1e-9
    # stability limit on the negative real axis
    z = np.linspace(-3.0, 0.0, 3000001)
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6
    limit = -z[np.abs(R) <= 1.0].min()
    assert limit == pytest.approx(2.51, abs=0.005)
    assert params.dt_max("rk3", 2, 0.1, 1.3, 0.07) == pytest.approx(
        2.51 * 0.1 ** 2 / (4 * 2 * 1.3 * 0.07), rel=1e-15)


@pytest.mark.parametrize("eps_over_dx,gamma_over_u", [(1.0, 1.0), (0.75, 2.0), (1.5, 1.0),
                                                       (2.0, 0.5)])
def test_rk3_at_eq27_bounded_on_and_above_the_crossover_line(eps_over_dx, gamma_over_u):
    """Fig. 6(c): the RK3 at its diffusive limit (Eq. 27) keeps the 1D drop in [0, 1] for a
    whole period on and above the crossover line."""
    lo, hi = _drop_1d_extremes(eps_over_dx, gamma_over_u, "rk3", 3)
    assert lo >= -EPS64 and hi <= 1 + EPS64, (lo, hi)
