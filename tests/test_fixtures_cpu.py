"""Host checks of the seeded input generators that build velocity fields (no GPU): the
solenoidal constructions the method relies on (Eq. 19's divergence term must vanish)."""
import numpy as np

import pf_fixtures as fx


def wall_divergence(U, V, dx):
    """Discrete divergence of a 2D face field in a box with walls on x and y (the high face of
    the last cell is the wall face, whose velocity is zero)."""
    U, V = U[0], V[0]
    Up = np.pad(U, ((0, 0), (0, 1)))
    Vp = np.pad(V, ((0, 1), (0, 0)))
    Up[:, 0] = 0.0
    Vp[0, :] = 0.0
    return (np.diff(Up, axis=1) + np.diff(Vp, axis=0)) / dx


def test_random_projected_field_is_solenoidal_with_slip_walls():
    n = 50
    dx = 2.0 / n
    for seed in range(3):
        U, V, W = fx.random_projected_faces(np.random.default_rng(seed), n, dx)
        assert np.all(U[0][:, 0] == 0.0) and np.all(V[0][0, :] == 0.0)  # no flow through walls
        assert np.abs(wall_divergence(U, V, dx)).max() <= 1e-12 / dx
        assert max(np.abs(U).max(), np.abs(V).max()) == 1.0
        assert not W.any()
        # random from cell to cell: neighbouring faces are far from equal
        assert np.abs(np.diff(U[0][:, 1:], axis=1)).mean() > 0.1
    # different seeds, different fields
    a = fx.random_projected_faces(np.random.default_rng(0), n, dx)[0]
    b = fx.random_projected_faces(np.random.default_rng(1), n, dx)[0]
    assert np.abs(a - b).max() > 0.5


def test_random_stream_field_is_solenoidal_with_slip_walls():
    n = 50
    dx = 2.0 / n
    U, V, W = fx.random_wall_stream_faces(np.random.default_rng(0), n, dx)
    assert np.all(U[0][:, 0] == 0.0) and np.all(V[0][0, :] == 0.0)
    assert np.abs(wall_divergence(U, V, dx)).max() <= 1e-12 / dx


def test_nonuniform_edge_curl_is_solenoidal():
    """The face velocity built on a rectilinear mesh has zero discrete divergence in every cell,
    sum_a (u_a[+] - u_a[-]) / h_a, with the periodic high face of the last cell at index 0."""
    rng = np.random.default_rng(3)
    nz, ny, nx = 5, 7, 6
    h = [fx.random_widths(rng, n, 1.0, 3.0) for n in (nx, ny, nz)]
    A = [rng.standard_normal((nz, ny, nx)) for _ in range(3)]
    U, V, W = fx.edge_curl_nu(*A, *h)
    div = ((np.roll(U, -1, 2) - U) / h[0][None, None, :] + (np.roll(V, -1, 1) - V) / h[1][None, :, None]
           + (np.roll(W, -1, 0) - W) / h[2][:, None, None])
    assert np.abs(div).max() <= 1e-12 * max(np.abs(U).max(), np.abs(V).max(), np.abs(W).max()) / min(map(np.min, h))
    assert np.isclose(h[0].sum(), 1.0) and np.isclose(fx.cell_centres(h[0])[-1], 1.0 - h[0][-1] / 2)
    s = fx.smooth_widths(64, 2.0, 2.5)
    assert np.isclose(s.sum(), 2.0) and np.isclose(s.max() / s.min(), 2.5, rtol=1e-2)
