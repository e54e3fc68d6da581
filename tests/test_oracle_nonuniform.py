"""Pins of the oracle's non-uniform rectilinear mesh (no GPU).

The paper's closing remarks extend the method to non-uniform anisotropic Cartesian grids (eps
fixed by the worst case, or tuned to the local mesh) without a discrete form; the oracle's
reading is stated in pf_oracle.c. These checks tie it to things fixed independently of its code:
the pinned uniform oracle (equal widths; anisotropic constant widths reduce to a 1D uniform
problem along the varying axis), exact divided differences of quadratics on a stretched mesh,
mirror symmetry of the mesh, volume-weighted conservation, and boundedness with eps on the
crossover line of the largest local spacing.
"""
import numpy as np
import pytest

import oracle
import pf_fixtures as fx


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def random_case(rng, shape, h=None):
    nz, ny, nx = shape
    if h is None:
        h = [fx.random_widths(rng, n, 1.0, 2.5) for n in (nx, ny, nz)]
    A = [rng.standard_normal(shape) * 0.05 for _ in range(3)]
    U, V, W = fx.edge_curl_nu(*A, *h)
    phi = rng.uniform(size=shape)
    return phi, U, V, W, h


@pytest.mark.parametrize("walls", [(False, False, False), (True, False, True)])
@pytest.mark.parametrize("eps_mode", [0, 1])
def test_equal_widths_reproduce_the_uniform_oracle(walls, eps_mode):
    rng = np.random.default_rng(1)
    shape = (6, 9, 11)
    dx = 0.07
    phi, U, V, W, _ = random_case(rng, shape)
    h = [np.full(n, dx) for n in shape[::-1]]
    kw = dict(dx=dx, eps=0.9 * dx, gamma=0.8, delta=0.4, s=0.7, walls=walls)
    want = oracle.rhs(phi, U, V, W, **kw)
    got = oracle.rhs_nu(phi, U, V, W, hx=h[0], hy=h[1], hz=h[2], eps_mode=eps_mode, **kw)
    assert rel(got, want) <= 1e-14
    sk = dict(dx=dx, eps=0.9 * dx, gamma=0.8, dt=0.02, nsteps=3, delta=0.4, walls=walls)
    want = oracle.step(phi, U, V, W, **sk)
    got = oracle.step_nu(phi, U, V, W, hx=h[0], hy=h[1], hz=h[2], eps_mode=eps_mode, **sk)
    assert rel(got, want) <= 1e-14


@pytest.mark.parametrize("axis,eps_mode", [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (2, 1)])
def test_constant_anisotropic_widths_reduce_to_1d(axis, eps_mode):
    """Widths (a, b, c) per axis, a field that varies along one axis only and a velocity along
    that axis that is constant across the others: the update is the 1D uniform problem with the
    spacing of the varying axis (a mistaken axis/width pairing breaks this). With eps tuned to
    the local mesh, the 1D problem's eps is eps * max(a, b, c) / dx; the largest width is the
    z width here, so a cell's maximum must include it."""
    rng = np.random.default_rng(2)
    n = 24
    widths = (0.03, 0.021, 0.05)
    line = fx.drops_ic((1, 1, n), widths[axis], [(0.4 * n * widths[axis], 0, 0)],
                       [0.2 * n * widths[axis]], 1.5 * widths[axis])[0, 0]
    vel_line = rng.uniform(0.5, 1.0) * np.ones(n)
    shape = [3, 4, 5]  # (nz, ny, nx) of the other axes
    shape[2 - axis] = n
    shape = tuple(shape)
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    phi = np.broadcast_to(line.reshape(bshape), shape).copy()
    vel = [np.zeros(shape) for _ in range(3)]
    vel[axis] = np.broadcast_to(vel_line.reshape(bshape), shape).copy()
    h = [np.full(m, widths[a]) for a, m in enumerate(shape[::-1])]
    eps, dxref = 1.2 * widths[axis], 0.04
    kw = dict(gamma=1.1, delta=0.0)
    got = oracle.rhs_nu(phi, *vel, hx=h[0], hy=h[1], hz=h[2], dx=dxref if eps_mode else widths[axis],
                        eps=eps, eps_mode=eps_mode, s=0.9, **kw)
    eps1 = eps * max(widths) / dxref if eps_mode else eps
    one = oracle.rhs(line.reshape(1, 1, n), vel_line.reshape(1, 1, n), np.zeros((1, 1, n)),
                     np.zeros((1, 1, n)), dx=widths[axis], eps=eps1, s=0.9, **kw)
    want = np.broadcast_to(one[0, 0].reshape(bshape), shape)
    assert rel(got, want) <= 1e-13


@pytest.mark.parametrize("eps_mode", [0, 1])
def test_quadratic_on_a_stretched_line_matches_exact_differences(eps_mode):
    """phi = c0 + c1 x + c2 x^2 on a randomly stretched 1D mesh (interior cells, away from the
    periodic seam), uniform velocity u0, delta > 0. Divided differences of a quadratic are exact:
    the central gradient at cell i is c1 + c2 (x_{i+1} + x_{i-1}), the face slope between i-1
    and i is c1 + c2 (x_{i-1} + x_i). The expected f below is built from these identities and
    the cell centres alone."""
    rng = np.random.default_rng(3)
    n = 40
    h = fx.random_widths(rng, n, 1.0, 3.0)
    x = fx.cell_centres(h)
    c0, c1, c2 = 0.3, 0.7, -0.45
    phi = (c0 + c1 * x + c2 * x * x).reshape(1, 1, n)
    u0, s, gamma, eps, delta, dxref = 0.8, 0.6, 0.9, 0.02, 0.5, 0.025
    # the y and z widths are the smallest, so that max(h) of a cell is its x width (eps_mode 1)
    hy = hz = np.array([0.5 * h.min()])
    U = np.full((1, 1, n), u0)
    Z = np.zeros((1, 1, n))
    f = oracle.rhs_nu(phi, U, Z, Z, hx=h, hy=hy, hz=hz, dx=dxref, eps=eps, gamma=gamma,
                      delta=delta, s=s, eps_mode=eps_mode)[0, 0]
    p = phi[0, 0]
    i = np.arange(2, n - 2)
    grad = c1 + c2 * (x[i + 1] + x[i - 1])
    gradp = c1 + c2 * (x[i + 2] + x[i])       # at i+1
    gradm = c1 + c2 * (x[i] + x[i - 2])       # at i-1
    q = lambda pp, g: pp * (1 - pp) * g / np.sqrt(g * g + delta * delta)
    adv = -s * u0 * (p[i + 1] - p[i - 1]) / (2 * h[i])
    slope_hi = c1 + c2 * (x[i] + x[i + 1])
    slope_lo = c1 + c2 * (x[i - 1] + x[i])
    if eps_mode == 0:
        dif = gamma * eps * (slope_hi - slope_lo) / h[i]
    else:  # face eps = eps/dx * mean width = eps/dx * centre distance: a plain second difference
        second = c1 * (x[i + 1] - 2 * x[i] + x[i - 1]) + c2 * (x[i + 1] ** 2 - 2 * x[i] ** 2 + x[i - 1] ** 2)
        dif = gamma * eps / dxref * second / h[i]
    shp = -0.5 * gamma * (q(p[i + 1], gradp) - q(p[i - 1], gradm)) / h[i]
    want = adv + dif + shp
    assert np.allclose(f[i], want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    assert np.abs(grad).min() > 0  # the case exercises the normal, not its zero branch


def test_mirrored_mesh_gives_the_mirrored_update():
    """Reversing the x axis (widths, phi, and the x-velocity, which moves to the opposite face
    and changes sign) reverses the update: an index slip in the centre distances or widths
    (using the high neighbour where the low one belongs) breaks this on an irregular mesh."""
    rng = np.random.default_rng(4)
    shape = (5, 6, 13)
    phi, U, V, W, h = random_case(rng, shape)
    kw = dict(dx=0.08, eps=0.07, gamma=1.3, delta=0.2)
    f = oracle.rhs_nu(phi, U, V, W, hx=h[0], hy=h[1], hz=h[2], eps_mode=1, **kw)
    nx = shape[2]
    Um = -np.roll(U[:, :, ::-1], 1, axis=2)  # face i of the mirror = face nx - i of the original
    fm = oracle.rhs_nu(phi[:, :, ::-1], Um, V[:, :, ::-1], W[:, :, ::-1], hx=h[0][::-1], hy=h[1],
                       hz=h[2], eps_mode=1, **kw)
    assert rel(fm[:, :, ::-1], f) <= 1e-13
    assert nx % 2 == 1


def test_one_cell_axis_does_not_enter_the_local_eps():
    """On a grid of one plane the z width is not resolved: with eps tuned to the local mesh the
    update does not depend on it (the largest width is taken over the axes longer than one
    cell, as the volume is)."""
    rng = np.random.default_rng(8)
    shape = (1, 10, 12)
    phi, U, V, W, h = random_case(rng, shape)
    W = np.zeros(shape)
    kw = dict(dx=0.08, eps=0.06, gamma=1.1, delta=0.1, eps_mode=1)
    a = oracle.rhs_nu(phi, U, V, W, hx=h[0], hy=h[1], hz=[1e-3], **kw)
    b = oracle.rhs_nu(phi, U, V, W, hx=h[0], hy=h[1], hz=[10.0], **kw)
    assert np.array_equal(a, b)
    assert oracle.reduce_nu(phi, hx=h[0], hy=h[1], hz=[1e-3]) == oracle.reduce_nu(phi, hx=h[0], hy=h[1], hz=[10.0])


@pytest.mark.parametrize("eps_mode", [0, 1])
def test_walled_axis_equals_its_even_reflection(eps_mode):
    """Walls on x with mirror ghosts are the even reflection: the walled update of n cells
    equals, on its first n cells, the periodic update of 2n cells holding the field, the widths
    and the tangential velocities mirrored, and the x-velocity mirrored with its sign flipped
    (zero on the two wall faces). This ties the walled mesh to the periodic one, including the
    widths the ghost cells take."""
    rng = np.random.default_rng(7)
    shape = (4, 5, 9)
    nz, ny, nx = shape
    phi, U, V, W, h = random_case(rng, shape)
    U = U.copy()
    U[:, :, 0] = 0.0  # the wall face
    kw = dict(dx=0.1, eps=0.08, gamma=1.2, delta=0.3, eps_mode=eps_mode, s=0.8)
    got = oracle.rhs_nu(phi, U, V, W, hx=h[0], hy=h[1], hz=h[2], walls=(True, False, False), **kw)
    even = lambda a: np.concatenate([a, a[:, :, ::-1]], axis=2)
    U2 = np.zeros((nz, ny, 2 * nx))
    U2[:, :, :nx] = U
    U2[:, :, nx + 1:] = -U[:, :, 1:][:, :, ::-1]  # face 2n - i carries -U[i]
    hx2 = np.concatenate([h[0], h[0][::-1]])
    ref = oracle.rhs_nu(even(phi), U2, even(V), even(W), hx=hx2, hy=h[1], hz=h[2], **kw)
    assert rel(got, ref[:, :, :nx]) <= 1e-13


@pytest.mark.parametrize("walls", [(False, False, False), (True, True, False)])
def test_volume_weighted_mass_is_conserved(walls):
    rng = np.random.default_rng(5)
    shape = (7, 8, 9)
    phi, U, V, W, h = random_case(rng, shape)
    kw = dict(dx=0.12, eps=0.1, gamma=0.9, delta=0.1, walls=walls)
    f = oracle.rhs_nu(phi, U, V, W, hx=h[0], hy=h[1], hz=h[2], eps_mode=1, **kw)
    vol = h[2][:, None, None] * h[1][None, :, None] * h[0][None, None, :]
    scale = np.abs(f * vol).sum()
    assert abs((f * vol).sum()) <= 1e-13 * scale
    assert abs(f.sum() * vol.mean()) > 1e-6 * scale  # the weights matter on this mesh
    m0 = oracle.reduce_nu(phi, hx=h[0], hy=h[1], hz=h[2])[0]
    out = oracle.step_nu(phi, U, V, W, hx=h[0], hy=h[1], hz=h[2], eps_mode=1, dt=0.01,
                         nsteps=5, **kw)
    assert abs(oracle.reduce_nu(out, hx=h[0], hy=h[1], hz=h[2])[0] - m0) <= 1e-14 * abs(m0) * 10
    assert np.isclose(m0, float((phi * vol).sum()), rtol=1e-14)


def test_local_eps_on_the_crossover_line_stays_bounded():
    """A drop carried across a smoothly stretched 2D mesh (widths varying by 2.5x along each
    axis) with eps tuned to the local mesh: eps/h_max on the crossover line of Eq. 17 with
    gamma = |u|_max. Every cell stays in [0, 1] over the run (the property the paper's remark
    says local tuning retains); eps fixed at the finest spacing instead leaves the bounds."""
    n = 48
    hx = fx.smooth_widths(n, 1.0, 2.5, 0.3)
    hy = fx.smooth_widths(n, 1.0, 2.5, 1.9)
    hz = np.array([1.0 / n])
    xc, yc = fx.cell_centres(hx), fx.cell_centres(hy)
    X, Y = np.meshgrid(xc, yc)
    r = np.hypot(X - 0.45, Y - 0.5)
    hloc = np.maximum(hx[None, :], hy[:, None])
    phi = (0.5 * (1.0 + np.tanh((0.2 - r) / (2.0 * hloc)))).reshape(1, n, n)
    rng = np.random.default_rng(6)
    Ax = np.zeros((1, n, n)); Ay = np.zeros((1, n, n))
    Az = rng.standard_normal((1, n, n))
    U, V, W = fx.edge_curl_nu(Ax, Ay, Az, hx, hy, hz)
    umax = max(np.abs(U).max(), np.abs(V).max())
    U, V = U / umax, V / umax
    gamma = 1.0
    ratio = oracle.params.crossover_eps_over_dx(gamma)
    dxref = 1.0 / n
    hmin = min(hx.min(), hy.min())
    dt = 0.1 * hmin
    kw = dict(hx=hx, hy=hy, hz=hz, dx=dxref, gamma=gamma, dt=dt, nsteps=150)
    out = oracle.step_nu(phi, U, V, W, eps=ratio * dxref, eps_mode=1, **kw)
    assert out.min() >= 0.0 and out.max() <= 1.0, (out.min(), out.max())
    bad = oracle.step_nu(phi, U, V, W, eps=0.5 * ratio * hmin, eps_mode=0, **kw)
    assert bad.min() < 0.0 or bad.max() > 1.0
