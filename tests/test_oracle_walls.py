"""Pins of the oracle's wall boundaries (no GPU).

The paper gives no discrete wall condition; the reading is zero total flux through a wall face
(no normal velocity, diffusive or sharpening flux) and mirror ghosts for the central gradient.
Pinned against the periodic oracle, which is pinned elsewhere: a walled axis of n cells behaves
exactly like the first half of a periodic axis of 2n cells carrying the mirror image of the data
(phi and the tangential velocities mirrored, the normal velocity mirrored with its sign flipped,
zero on the two faces that play the walls). Also: mass is conserved for any velocity, and the
velocity stored on a wall face has no effect.
"""
import numpy as np
import pytest

import oracle
import pf_fixtures as fx


def _double(a, ax, normal):
    """Mirror-double array a along numpy axis ax (the image of a walled axis)."""
    n = a.shape[ax]
    if not normal:
        return np.concatenate([a, np.flip(a, ax)], axis=ax)
    a0 = a.copy()
    sl = [slice(None)] * 3
    sl[ax] = 0
    a0[tuple(sl)] = 0.0  # the wall face at 0
    zero = np.zeros_like(np.take(a0, [0], axis=ax))  # the wall face at n
    tail = -np.flip(np.take(a0, range(1, n), axis=ax), ax)  # faces n+1 .. 2n-1
    return np.concatenate([a0, zero, tail], axis=ax)


def _case(seed, shape):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    dx = 1.0 / max(shape)
    phi = fx.drops_ic(shape, dx, [(0.3 * nx * dx, 0.6 * ny * dx, 0.4 * nz * dx)],
                      [0.35 * max(shape) * dx], 1.2 * dx)
    phi = 0.85 * phi + 0.15 * rng.uniform(size=shape)
    U, V, W = (rng.uniform(-1, 1, size=shape) for _ in range(3))  # any field: no projection
    return phi, U, V, W, dx


@pytest.mark.parametrize("walls", [(True, False, False), (False, True, False),
                                   (False, False, True), (True, False, True),
                                   (True, True, True)])
@pytest.mark.parametrize("scheme", [1, 2, 4])
def test_walls_equal_the_mirror_doubled_periodic_domain(walls, scheme):
    phi, U, V, W, dx = _case(1, (7, 9, 11))
    kw = dict(dx=dx, eps=dx, gamma=1.1, dt=0.05 * dx, nsteps=6, delta=0.3 / dx, scheme=scheme)
    got = oracle.step(phi, U, V, W, walls=walls, **kw)
    P, Us, Vs, Ws = phi, U, V, W
    for a, w in enumerate(walls):  # a: x, y, z; numpy axis 2 - a
        if w:
            ax = 2 - a
            P = _double(P, ax, False)
            Us = _double(Us, ax, a == 0)
            Vs = _double(Vs, ax, a == 1)
            Ws = _double(Ws, ax, a == 2)
    ref = oracle.step(P, Us, Vs, Ws, **kw)[:phi.shape[0], :phi.shape[1], :phi.shape[2]]
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-15)
    # the doubled run stays an exact mirror image (what makes the comparison meaningful)
    full = oracle.step(P, Us, Vs, Ws, **kw)
    for a, w in enumerate(walls):
        if w:
            np.testing.assert_array_equal(full, np.flip(full, 2 - a))


@pytest.mark.parametrize("walls", [(True, False, False), (True, True, True)])
def test_walls_conserve_mass_and_ignore_the_wall_face_velocity(walls):
    phi, U, V, W, dx = _case(2, (8, 10, 12))
    kw = dict(dx=dx, eps=dx, gamma=1.0, dt=0.05 * dx, nsteps=20, walls=walls)
    out = oracle.step(phi, U, V, W, **kw)
    m0, m1 = oracle.reduce(phi, dx=dx)[0], oracle.reduce(out, dx=dx)[0]
    assert abs(m1 - m0) / m0 < 1e-12
    # non-zero normal velocity on the wall faces (index 0 of a walled axis) changes nothing
    U2, V2, W2 = U.copy(), V.copy(), W.copy()
    for a, (w, arr) in enumerate(zip(walls, (U2, V2, W2))):
        if w:
            sl = [slice(None)] * 3
            sl[2 - a] = 0
            arr[tuple(sl)] += 5.0
    out2 = oracle.step(phi, U2, V2, W2, **kw)
    np.testing.assert_array_equal(out, out2)
    # and the walls do change the result compared with periodicity (the test has teeth)
    per = oracle.step(phi, U, V, W, **{**kw, "walls": (False, False, False)})
    assert np.abs(per - out).max() > 1e-3
