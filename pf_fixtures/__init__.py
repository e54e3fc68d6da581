"""Seeded synthetic inputs for the phase-field step (shared by tests, smoke check and bench).

This module builds inputs only — initial phase fields, face velocities, mode coefficients and
the parameter sets of the workloads. It holds none of the step's arithmetic and imports neither
the GPU package nor the oracle. Random numbers come from numpy's PCG64 with explicit seeds.

Conventions: arrays (nz, ny, nx), x fastest; cell (i,j,k) spans [i dx, (i+1) dx] per axis;
U/V/W hold the velocity on the low x/y/z face of each cell. Periodic unit-length boxes unless a
length is given.

Initial condition (Sec. 1): phi = 0.5 (1 + tanh(s / (2 eps))), s the signed distance, positive
inside; periodic minimum-image distances; a union of drops takes s = max_k (R_k - |x - c_k|).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ------------------------------------------------------------------------ initial conditions


def tanh_profile(s: np.ndarray, eps: float) -> np.ndarray:
    return 0.5 * (1.0 + np.tanh(s / (2.0 * eps)))


def _axis_offsets(n: int, dx: float, c: float, L: float, reach: float | None):
    """Cell indices (within reach of c, periodic) and their minimum-image offsets x - c."""
    if reach is None or 2 * reach >= L:
        idx = np.arange(n)
    else:
        lo = int(math.floor((c - reach) / dx - 0.5))
        hi = int(math.ceil((c + reach) / dx - 0.5))
        idx = np.arange(lo, hi + 1) % n
        idx = np.unique(idx)
    x = (idx + 0.5) * dx
    d = x - c
    d -= L * np.round(d / L)
    return idx, d


def drops_ic(shape, dx, centres, radii, eps, window: bool = True) -> np.ndarray:
    """Union of spherical (or circular, for nz = 1) drops with a tanh profile.

    With window=True each drop is evaluated only within R + 60 eps of its centre; outside that
    distance tanh(s / 2 eps) rounds to -1 in FP64, so the result equals the full evaluation.
    """
    nz, ny, nx = shape
    L = (nx * dx, ny * dx, nz * dx)
    s = np.full(shape, -np.inf)
    for c, r in zip(centres, radii):
        reach = r + 60.0 * eps if window else None
        ix, dxo = _axis_offsets(nx, dx, c[0], L[0], reach)
        iy, dyo = _axis_offsets(ny, dx, c[1], L[1], reach)
        if nz > 1:
            iz, dzo = _axis_offsets(nz, dx, c[2], L[2], reach)
        else:
            iz, dzo = np.array([0]), np.array([0.0])
        dist = np.sqrt(dzo[:, None, None] ** 2 + dyo[None, :, None] ** 2 + dxo[None, None, :] ** 2)
        sub = s[np.ix_(iz, iy, ix)]
        s[np.ix_(iz, iy, ix)] = np.maximum(sub, r - dist)
    return tanh_profile(s, eps)


def random_drops(rng: np.random.Generator, count: int, rmin: float, rmax: float):
    centres = rng.uniform(0.0, 1.0, size=(count, 3))
    radii = rng.uniform(rmin, rmax, size=count)
    return centres, radii


# ------------------------------------------------------------------------ face velocities


def edge_curl(Ax, Ay, Az, dx):
    """Face velocity = discrete curl of an edge potential (Ax at ((i+1/2)dx, j dx, k dx),
    Ay at (i dx, (j+1/2) dx, k dx), Az at (i dx, j dx, (k+1/2) dx)); zero discrete divergence."""
    r = np.roll
    U = (r(Az, -1, 1) - Az - r(Ay, -1, 0) + Ay) / dx
    V = (r(Ax, -1, 0) - Ax - r(Az, -1, 2) + Az) / dx
    W = (r(Ay, -1, 2) - Ay - r(Ax, -1, 1) + Ax) / dx
    return U, V, W


def edge_curl_nu(Ax, Ay, Az, hx, hy, hz):
    """edge_curl on a rectilinear mesh with cell widths hx (nx), hy (ny), hz (nz): each
    difference of the potential is divided by the width of the cell it spans, so that
    sum_a (u_a[+] - u_a[-]) / h_a = 0 in every cell."""
    r = np.roll
    hx, hy, hz = (np.asarray(h, dtype=np.float64) for h in (hx, hy, hz))
    HX, HY, HZ = hx[None, None, :], hy[None, :, None], hz[:, None, None]
    U = (r(Az, -1, 1) - Az) / HY - (r(Ay, -1, 0) - Ay) / HZ
    V = (r(Ax, -1, 0) - Ax) / HZ - (r(Az, -1, 2) - Az) / HX
    W = (r(Ay, -1, 2) - Ay) / HX - (r(Ax, -1, 1) - Ax) / HY
    return U, V, W


def smooth_widths(n: int, L: float = 1.0, ratio: float = 2.0, phase: float = 0.0) -> np.ndarray:
    """n cell widths summing to L that vary smoothly and periodically between w and ratio * w
    (h_i proportional to 1 + a cos(2 pi (i + 1/2) / n + phase), a = (ratio - 1)/(ratio + 1))."""
    a = (ratio - 1.0) / (ratio + 1.0)
    h = 1.0 + a * np.cos(2.0 * np.pi * (np.arange(n) + 0.5) / n + phase)
    return h * (L / h.sum())


def random_widths(rng: np.random.Generator, n: int, L: float = 1.0, ratio: float = 2.0) -> np.ndarray:
    """n cell widths summing to L, independent U[1, ratio] draws (jumps from cell to cell)."""
    h = rng.uniform(1.0, ratio, size=n)
    return h * (L / h.sum())


def cell_centres(h) -> np.ndarray:
    """Centre coordinates of cells of widths h laid end to end from 0."""
    h = np.asarray(h, dtype=np.float64)
    return np.cumsum(h) - 0.5 * h


def zalesak_ic(n: int, eps: float, L: float = 100.0, centre=(50.0, 75.0), R: float = 15.0,
               w: float = 5.0, l: float = 25.0) -> np.ndarray:
    """Notched disk (Sec. 3.3.2) on an n x n x 1 grid of an L x L box: the tanh profile of an
    approximate signed distance, positive inside the disk and outside the notch. The notch is a
    w-wide slot rising l from the bottom of the disk, centred on its vertical axis. (The printed
    radius "0.15" is read as 15 box units, the scale of the printed w, l and box.)"""
    dx = L / n
    x = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(x, x)  # [j, i]: X = x_i, Y = y_j
    s_disk = R - np.hypot(X - centre[0], Y - centre[1])
    x0, x1 = centre[0] - w / 2, centre[0] + w / 2
    y0, y1 = centre[1] - R, centre[1] - R + l
    s_slot = np.minimum.reduce([X - x0, x1 - X, Y - y0, y1 - Y])  # > 0 inside the slot
    return tanh_profile(np.minimum(s_disk, -s_slot), eps).reshape(1, n, n)


def zalesak_faces(n: int, L: float = 100.0):
    """Solid-body rotation u = (pi (50 - y) / 314, pi (x - 50) / 314) (Sec. 3.3.2), one turn in
    t = 628, sampled on the faces: U on the x-faces depends on y only and V on the y-faces on x
    only, so the discrete divergence is exactly zero (also across the periodic seams)."""
    dx = L / n
    c = (np.arange(n) + 0.5) * dx
    U = np.broadcast_to((np.pi * (50.0 - c) / 314.0)[:, None], (n, n)).reshape(1, n, n).copy()
    V = np.broadcast_to((np.pi * (c - 50.0) / 314.0)[None, :], (n, n)).reshape(1, n, n).copy()
    return U, V, np.zeros((1, n, n))


def random_wall_stream_faces(rng: np.random.Generator, n: int, dx: float):
    """A cell-to-cell random, discretely solenoidal 2D face velocity for an n x n box with walls
    on x and y (Sec. 3.2.2 stand-in): i.i.d. standard normal stream-function values at the
    interior cell corners, zero on the walls, and its discrete curl (u = -dPsi/dy, v = dPsi/dx).
    The normal velocity on the wall faces is then exactly zero. Scaled so that the largest face
    component is 1. (The paper projects random point vectors with a Poisson solve instead.)"""
    psi = np.zeros((n + 1, n + 1))  # [j, i] at corner (i dx, j dx)
    psi[1:n, 1:n] = rng.standard_normal((n - 1, n - 1))
    U = -(psi[1:, :n] - psi[:n, :n]) / dx  # x-face (i dx, (j + 1/2) dx)
    V = (psi[:n, 1:] - psi[:n, :n]) / dx   # y-face ((i + 1/2) dx, j dx)
    s = 1.0 / max(np.abs(U).max(), np.abs(V).max())
    return (U * s).reshape(1, n, n), (V * s).reshape(1, n, n), np.zeros((1, n, n))


def random_projected_faces(rng: np.random.Generator, n: int, dx: float):
    """The 2D random velocity of Sec. 3.2.2 for an n x n box with slip walls on x and y: every
    cell centre gets a velocity of independently uniform magnitude in [0, 1) and uniform
    direction; averaged onto the MAC faces (zero normal velocity on the wall faces); made
    discretely solenoidal by a Poisson projection with no-flux walls, u <- u - grad p with
    div grad p = div u (the cell-centred Neumann Laplacian is diagonal in the type-II cosine
    basis, eigenvalues (2 cos(pi k/n) - 2 + 2 cos(pi l/n) - 2) / dx^2); scaled so that the
    largest face component is 1."""
    from scipy import fft as sfft
    mag = rng.uniform(0.0, 1.0, (n, n))
    ang = rng.uniform(0.0, 2.0 * np.pi, (n, n))
    uc, vc = mag * np.cos(ang), mag * np.sin(ang)  # [j, i] at cell centres
    U = np.zeros((n, n))
    V = np.zeros((n, n))
    U[:, 1:] = 0.5 * (uc[:, :-1] + uc[:, 1:])  # low x-face of cell i (i = 0: the wall)
    V[1:, :] = 0.5 * (vc[:-1, :] + vc[1:, :])
    div = (np.diff(np.pad(U, ((0, 0), (0, 1))), axis=1) +
           np.diff(np.pad(V, ((0, 1), (0, 0))), axis=0)) / dx
    k = np.arange(n)
    lam = (2.0 * np.cos(np.pi * k / n) - 2.0) / (dx * dx)
    lap = lam[:, None] + lam[None, :]
    dh = sfft.dctn(div, type=2, norm="ortho")
    lap[0, 0] = 1.0
    dh[0, 0] = 0.0  # the divergence sums to zero: no flux through the walls
    p = sfft.idctn(dh / lap, type=2, norm="ortho")
    U[:, 1:] -= (p[:, 1:] - p[:, :-1]) / dx
    V[1:, :] -= (p[1:, :] - p[:-1, :]) / dx
    s = 1.0 / max(np.abs(U).max(), np.abs(V).max())
    return (U * s).reshape(1, n, n), (V * s).reshape(1, n, n), np.zeros((1, n, n))


def vortex2d_faces(n: int):
    """Single-vortex field on the unit square, n x n x 1 (Sec. 3.3.1, Eq. 33).

    Psi = sin^2(pi x) sin^2(pi y) / pi at the cell corners; the face velocity is its discrete
    curl with u = -dPsi/dy, v = +dPsi/dx (u = -sin^2(pi x) sin(2 pi y) in the continuum)."""
    dx = 1.0 / n
    xn = np.arange(n) * dx
    psi = (np.sin(np.pi * xn)[None, :] ** 2) * (np.sin(np.pi * xn)[:, None] ** 2) / np.pi
    Az = (-psi)[None, :, :]
    zero = np.zeros_like(Az)
    U, V, W = edge_curl(zero, zero, Az, dx)
    return U, V, np.zeros_like(W)


def deformation3d_faces(n: int):
    """A three-dimensional deformation field on the unit cube (this project's own choice, in
    the spirit of the reversing deformation tests): the discrete curl of the edge potential
    A = (sin^2(pi y) sin^2(pi z) sin(2 pi x), -sin^2(pi x) sin^2(pi z) sin(2 pi y),
         sin^2(pi x) sin^2(pi y) sin(2 pi z)) / pi."""
    dx = 1.0 / n
    node = np.arange(n) * dx
    mid = (np.arange(n) + 0.5) * dx

    def grid(xs, ys, zs):
        return np.meshgrid(zs, ys, xs, indexing="ij")[::-1]  # x, y, z arrays of shape (n,n,n)

    s2 = lambda t: np.sin(np.pi * t) ** 2  # noqa: E731
    x, y, z = grid(mid, node, node)
    Ax = s2(y) * s2(z) * np.sin(2 * np.pi * x) / np.pi
    x, y, z = grid(node, mid, node)
    Ay = -s2(x) * s2(z) * np.sin(2 * np.pi * y) / np.pi
    x, y, z = grid(node, node, mid)
    Az = s2(x) * s2(y) * np.sin(2 * np.pi * z) / np.pi
    return edge_curl(Ax, Ay, Az, dx)


def random_edge_faces(rng: np.random.Generator, shape, dx, scale=1.0):
    """Cell-to-cell random solenoidal face velocity: curl of an i.i.d. normal edge potential."""
    Ax, Ay, Az = (rng.standard_normal(shape) * scale * dx for _ in range(3))
    return edge_curl(Ax, Ay, Az, dx)


def random_modes(rng: np.random.Generator, M: int, n: int, decay: float = 2.0):
    """Phases (3, M) and coefficients (M, M, M, 3) of a separable-mode vector potential
    (modes m = 1..M per axis, amplitudes N(0,1) / |m|^decay), scaled so that the discrete
    curl on an n^3 unit-cube grid has unit RMS over all face samples of U, V and W.

    The scale uses the exact discrete mean square: for 2M < n the sampled sines are
    orthogonal, each contributes 1/2 per axis, and a one-cell difference of
    sin(2 pi m x + t) has amplitude kappa_m = 2 sin(pi m / n) / dx. Hence
      <U^2> = (1/8) sum_m (c_z^2 kappa_{m2}^2 + c_y^2 kappa_{m3}^2), and cyclically.
    """
    assert 2 * M < n, "the unit-RMS scaling needs 2M < n"
    phases = rng.uniform(0.0, 2.0 * np.pi, size=(3, M))
    m = np.arange(1, M + 1, dtype=np.float64)
    m3, m2, m1 = np.meshgrid(m, m, m, indexing="ij")
    mag = np.sqrt(m1 ** 2 + m2 ** 2 + m3 ** 2)
    coeffs = rng.standard_normal((M, M, M, 3)) / mag[..., None] ** decay
    dx = 1.0 / n
    kap = lambda mm: 2.0 * np.sin(np.pi * mm / n) / dx  # noqa: E731
    cx, cy, cz = coeffs[..., 0], coeffs[..., 1], coeffs[..., 2]
    u2 = np.sum(cz ** 2 * kap(m2) ** 2 + cy ** 2 * kap(m3) ** 2) / 8.0
    v2 = np.sum(cx ** 2 * kap(m3) ** 2 + cz ** 2 * kap(m1) ** 2) / 8.0
    w2 = np.sum(cy ** 2 * kap(m1) ** 2 + cx ** 2 * kap(m2) ** 2) / 8.0
    rms = math.sqrt((u2 + v2 + w2) / 3.0)
    return phases, coeffs / rms


def fourier_faces(shape, dx, phases, coeffs, dtype=np.float64):
    """Face velocity of the separable-mode edge potential, built on the host with numpy
    (tensor contractions over the 1-D sine tables, then the discrete curl). An input generator
    for cases whose velocity must not come from the GPU path (e.g. inputs of oracle checks at
    large sizes); same potential and edge positions as the library's synthesis."""
    nz, ny, nx = shape
    M = phases.shape[1]
    m = np.arange(1, M + 1, dtype=np.float64)

    def tab(axis, n, off):
        i = np.arange(n, dtype=np.float64) + off
        return np.sin(2.0 * np.pi * m[:, None] * i[None, :] / n + phases[axis][:, None])

    A = []
    for c in range(3):
        X = tab(0, nx, 0.5 if c == 0 else 0.0)
        Y = tab(1, ny, 0.5 if c == 1 else 0.0)
        Z = tab(2, nz, 0.5 if c == 2 else 0.0)
        t1 = np.einsum("abc,ci->abi", coeffs[..., c], X)      # [m3][m2][i]
        t2 = np.einsum("abi,bj->aji", t1, Y)                  # [m3][j][i]
        A.append(np.einsum("aji,ak->kji", t2, Z, optimize=True).astype(dtype, copy=False))
    return edge_curl(A[0], A[1], A[2], dx)


def max_face_speed(U, V, W) -> float:
    """Largest |component| over the three face arrays (the |u|_max that sets gamma)."""
    return float(max(np.abs(U).max(), np.abs(V).max(), np.abs(W).max()))


# ------------------------------------------------------------------------ workloads


@dataclass
class Case:
    """One simulation: grid, parameters and inputs (FP64 numpy, shape (nz, ny, nx))."""
    name: str
    shape: tuple
    dx: float
    eps: float
    gamma: float
    dt: float
    nsteps: int
    phi0: np.ndarray
    U: np.ndarray | None = None
    V: np.ndarray | None = None
    W: np.ndarray | None = None
    delta: float = 0.0
    vel_mode: int = 0
    vel_T: float = 1.0
    modes: tuple | None = None  # (phases, coeffs) when the velocity comes from mode synthesis
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return int(np.prod(self.shape))


def rk4_dt_3d(dx, gamma, eps):
    """0.9 x the RK4 diffusive limit in three dimensions (2.79 dx^2 / (12 gamma eps))."""
    return 0.9 * 2.79 * dx * dx / (12.0 * gamma * eps)


def vortex2d(n: int = 64, T: float = 4.0, cfl: float = 0.1) -> Case:
    """Drop in the time-reversed single vortex (Sec. 3.3.1): R = 0.15 at (0.5, 0.75), T = 4,
    eps = dx, gamma = max|u|, dt from CFL 0.1 rounded so that T is reached exactly."""
    dx = 1.0 / n
    U, V, W = vortex2d_faces(n)
    umax = max_face_speed(U, V, W)
    nsteps = int(math.ceil(T / (cfl * dx / umax) - 1e-9))
    phi0 = drops_ic((1, n, n), dx, [(0.5, 0.75, 0.0)], [0.15], dx)
    return Case("vortex2d", (1, n, n), dx, dx, umax, T / nsteps, nsteps, phi0, U, V, W,
                vel_mode=1, vel_T=T)


def deformation3d(n: int = 256, T: float = 3.0, nsteps: int = 2000) -> Case:
    """Sphere R = 0.15 at (0.35, 0.35, 0.35) in the reversing 3D deformation field (cos(pi t/T)),
    eps = dx, gamma = max|u|, dt = 0.9 x the RK4 diffusive limit."""
    dx = 1.0 / n
    U, V, W = deformation3d_faces(n)
    umax = max_face_speed(U, V, W)
    phi0 = drops_ic((n, n, n), dx, [(0.35, 0.35, 0.35)], [0.15], dx)
    return Case("deformation3d", (n, n, n), dx, dx, umax, rk4_dt_3d(dx, umax, dx), nsteps, phi0,
                U, V, W, vel_mode=1, vel_T=T)


def random_field(n: int, seed: int, M: int, drops: int, rmin: float, rmax: float,
                 eps_over_dx: float, gamma_over_u: float, nsteps: int, name: str,
                 umax: float | None = None) -> Case:
    """Random drops in a seeded solenoidal Fourier field. The velocity is given as modes; the
    caller synthesises the faces. gamma is set from umax (max face speed of the synthesised
    field) when known; otherwise a placeholder of 0 is stored and must be filled in."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    phases, coeffs = random_modes(rng, M, n)
    centres, radii = random_drops(rng, drops, rmin, rmax)
    eps = eps_over_dx * dx
    phi0 = drops_ic((n, n, n), dx, centres, radii, eps)
    c = Case(name, (n, n, n), dx, eps, 0.0, 0.0, nsteps, phi0, modes=(phases, coeffs),
             extra={"gamma_over_u": gamma_over_u, "centres": centres, "radii": radii})
    if umax is not None:
        set_speed(c, umax)
    return c


def set_speed(c: Case, umax: float) -> None:
    """Fill gamma and dt once the face speed of the synthesised velocity is known.

    dt = 0.9 x min(RK4 diffusive limit, 2.83 dx / (3 umax + 3 gamma)); the second bound is the
    three-axis analogue of the mixed criterion used below the crossover line."""
    c.gamma = c.extra["gamma_over_u"] * umax
    c.extra["umax"] = umax
    diff = 2.79 * c.dx * c.dx / (12.0 * c.gamma * c.eps)
    mixed = 2.83 * c.dx / (3.0 * umax + 3.0 * c.gamma)
    c.dt = 0.9 * min(diff, mixed)


def roofline512(n: int = 512, seed: int = 3) -> Case:
    """512^3 bandwidth run: 64 drops (R in [0.03, 0.08]), 16 modes per axis, eps = 0.75 dx,
    gamma = 1.1 max|u|, 500 steps."""
    return random_field(n, seed, 16, 64, 0.03, 0.08, 0.75, 1.1, 500, "roofline512")


BATCH_SIZES = (32, 48, 64, 96, 128)


def batch_cases(count: int = 96, seed: int = 4, nsteps: int = 300, sizes=BATCH_SIZES):
    """Independent FP32 instances with uneven grids: n from sizes, 1-8 drops of R in
    [0.05, 0.2], 8-mode solenoidal field each, eps = dx, gamma = max|u|."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.choice(sizes))
        drops = int(rng.integers(1, 9))
        sub = int(rng.integers(0, 2 ** 31 - 1))
        out.append(random_field(n, sub, 8, drops, 0.05, 0.2, 1.0, 1.0, nsteps, "batch%d" % b))
    return out


def adjoint_case(n: int = 128, seed: int = 5, nsteps: int = 400) -> Case:
    """Adjoint workload: drop of R = 0.2 at (0.4, 0.45, 0.5) carried by a seeded 8-mode field
    for nsteps; target = drop of R = 0.2 at the centre; eps = dx, gamma = max|u|;
    |grad phi| regulariser delta = 1e-3 / dx (small against the largest interface gradient
    1 / (4 eps), and large enough that the FP32 adjoint is well conditioned where phi is flat)."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    phases, coeffs = random_modes(rng, 8, n)
    phi0 = drops_ic((n, n, n), dx, [(0.4, 0.45, 0.5)], [0.2], dx)
    target = drops_ic((n, n, n), dx, [(0.5, 0.5, 0.5)], [0.2], dx)
    return Case("adjoint", (n, n, n), dx, dx, 0.0, 0.0, nsteps, phi0, modes=(phases, coeffs),
                delta=1e-3 / dx, extra={"gamma_over_u": 1.0, "target": target})
