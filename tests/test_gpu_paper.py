"""The paper's 2D uniform-translation experiment (Sec. 3.2.1, Tables 1-2), its 1D refinement
study (Sec. 3.1) and the RK2 boundedness map (Sec. 2.3, Fig. 6(a)) on the HIP stepper.

2D translation:

A D = 1 drop in a 2 x 2 periodic box (dx = D/25) is carried by (u, v) = (sqrt2/2, sqrt2/2) for
T = 2 sqrt2 with classic RK4 at dt = min(Eq. 31, Eq. 32), for the seven (eps/dx, gamma/|u|)
points of Table 2. Checked against the paper: points 1-5 stay inside [0, 1] at every step, 6-7
leave it. Checked against the oracle: the final field and E_delta = mean |phi(T) - phi(0)|.
E_tot of Table 1 is asserted within 3 % for every point (it is dominated by E_eps, the initial
profile's own departure from the top hat, which the tanh profile reproduces within 2.4 %); the
printed E_delta column follows no reading of the unstated details that was tried (see the design
notes), so E_delta is compared with the oracle's and printed beside the paper's.

Tolerance. Several of these runs are ill-conditioned: where the tails of the drop's periodic
images meet, grad phi vanishes and the unit normal g/|g| (delta = 0, as in the paper) flips under
rounding-level changes, and points 6-7 (outside the bounded regime) amplify them further. The
GPU and the oracle evaluate each FP64 step in different operation orders, so after every step
they differ by a few units in the last place (below 2^-50 relative on the short parity runs).
The bar is derived from the oracle alone, before the GPU result is looked at: the oracle's run
is repeated step by step with every step's result multiplied by 1 + 2^-50 xi (xi seeded
standard normal noise, two seeds), which is what rounding differences of that size grow into by
the end of the run; the bar is three times the larger of the two responses (two independent
realisations of such noise, the GPU's and the oracle's, and the spread between seeds), and at
least 1e-12 relative. Each test prints the GPU's difference, the response and their ratio.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import params
import pf_fixtures as fx

pytestmark = pytest.mark.gpu

EPS64 = float(np.finfo(np.float64).eps)


def oracle_bar(ref, phi0, vel, kw, seed):
    """Bar for |GPU - oracle| on an ill-conditioned FP64 run: 3 x the oracle's response to
    per-step rounding-sized noise (relative 2^-50, two seeds), at least 1e-12 relative."""
    kw = dict(kw)
    ns = kw.pop("nsteps")
    dt = kw["dt"]
    resp = 0.0
    for sd in (seed, seed + 7919):
        rng = np.random.default_rng(sd)
        y = np.array(phi0, dtype=np.float64)
        for k in range(ns):
            y = oracle.step(y, *vel, nsteps=1, t0=k * dt, **kw)
            y *= 1.0 + 2.0 ** -50 * rng.standard_normal(y.shape)
        resp = max(resp, float(np.abs(y - ref).max()))
    return max(1e-12 * float(np.abs(ref).max()), 3.0 * resp), resp


def check_against_oracle(got, ref, phi0, vel, kw, seed, label):
    diff = float(np.abs(got - ref).max())
    tol, resp = oracle_bar(ref, phi0, vel, kw, seed)
    ratio = diff / resp if resp > 0 else float("inf")
    print(f"{label}: |gpu - oracle| {diff:.2e}, oracle noise response {resp:.2e}, ratio "
          f"{ratio:.2f}, bar {tol:.2e}", flush=True)
    assert diff <= tol, (label, diff, tol)
    return tol


def test_table2_classification_and_table1_errors_on_the_gpu(lib):
    pf = lib
    pts = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
    n, L = 50, 2.0
    dx = L / n
    u = math.sqrt(2) / 2
    U = np.full((1, n, n), u)
    Z = np.zeros_like(U)
    T = 2 * math.sqrt(2)
    x = (np.arange(n) + 0.5) * dx
    top_hat = (np.sqrt((x[None, :] - 1) ** 2 + (x[:, None] - 1) ** 2) < 0.5).astype(float)
    st = torch.cuda.Stream()
    for p in pts["points"]:
        eps, gamma = p["eps_over_dx"] * dx, p["gamma_over_u"]
        phi0 = fx.drops_ic((1, n, n), dx, [(1.0, 1.0, 0.0)], [0.5], eps, window=False)
        dt = min(params.dt_rk4_2d_eq31(dx, gamma, eps), params.dt_rk4_2d_eq32(dx, u, u, gamma))
        ns = math.ceil(T / dt)
        dt = T / ns
        s = pf.Solver((n, n, 1), dx, eps, gamma, dt, dtype="f64", use_graph=False)
        g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi0, U, U, Z)]
        lo, hi = 1.0, 0.0
        with torch.cuda.stream(st):
            for k in range(ns):
                s.step(*g, t0=k * dt, nsteps=1, stream=st)
                _, mn, mx, bad = s.reduce(g[0], stream=st)
                assert bad == 0
                lo, hi = min(lo, mn), max(hi, mx)
        got = g[0].cpu().numpy()
        s.close()
        kw = dict(dx=dx, eps=eps, gamma=gamma, dt=dt, nsteps=ns)
        ref = oracle.step(phi0, U, U, Z, **kw)
        tol = check_against_oracle(got, ref, phi0, (U, U, Z), kw, p["point"], f"point {p['point']}")
        bounded = lo >= -EPS64 and hi <= 1 + EPS64
        assert bounded == p["bounded"], (p["point"], lo, hi)
        e_delta = np.abs(got - phi0).mean()
        e_delta_ref = np.abs(ref - phi0).mean()
        assert abs(e_delta - e_delta_ref) <= tol
        e_eps = np.abs(phi0[0] - top_hat).mean()
        e_tot = np.abs(got[0] - top_hat).mean()
        assert abs(e_tot - p["E_tot"]) <= 0.03 * p["E_tot"], (p["point"], e_tot, p["E_tot"])
        print(f"point {p['point']}: {ns} steps, min {lo:.3e}, max-1 {hi - 1:.3e}, "
              f"E_delta {e_delta:.5f} (paper {p['E_delta']}), E_eps {e_eps:.5f} "
              f"(paper {p['E_eps']}), E_tot {e_tot:.5f} (paper {p['E_tot']})", flush=True)


def _gpu_run_1d(pf, phi0, U, dx, eps, gamma, dt, ns, scheme="rk4"):
    n = phi0.shape[2]
    s = pf.Solver((n, 1, 1), dx, eps, gamma, dt, dtype="f64", scheme=scheme)
    z = np.zeros_like(U)
    g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi0, U, z, z)]
    s.step(*g, nsteps=ns)
    out = g[0].cpu().numpy()
    s.close()
    return out


def test_1d_drop_refinement_on_the_gpu(lib):
    """Sec. 3.1 on the HIP stepper: a D = 1 drop advected by u = 1 over one period T = 2 of the
    periodic domain [-1, 1], RK4 at 0.9 x Eq. 28, with eps/dx fixed while dx is refined. The
    paper reports first-order convergence of E_eps, E_delta and E_tot (Figure 8) and smaller
    total errors on the crossover line than above it at the same gamma/u (Figure 9): here
    eps/dx = 1 (on the line for gamma/u = 1) against eps/dx = 2, N = 100 .. 800 cells.
    (At exactly the Eq. 28 limit the longest runs let round-off grow; 0.9 x keeps every run
    inside the stable range.) Each GPU run is also compared with the oracle, with the
    tolerance measured on the oracle as in the 2D test (grad phi vanishes at the drop's centre).
    """
    pf = lib
    T = 2.0
    errs = {}
    for eps_dx in (1.0, 2.0):
        for n in (100, 200, 400, 800):
            dx = 2.0 / n
            eps, gamma = eps_dx * dx, 1.0
            phi0 = fx.drops_ic((1, 1, n), dx, [(1.0, 0.5 * dx, 0.0)], [0.5], eps, window=False)
            U = np.ones((1, 1, n))
            Z = np.zeros_like(U)
            dt = 0.9 * params.dt_max("rk4", 1, dx, gamma, eps)
            ns = math.ceil(T / dt)
            dt = T / ns
            got = _gpu_run_1d(pf, phi0, U, dx, eps, gamma, dt, ns)
            kw = dict(dx=dx, eps=eps, gamma=gamma, dt=dt, nsteps=ns)
            ref = oracle.step(phi0, U, Z, Z, **kw)
            check_against_oracle(got, ref, phi0, (U, Z, Z), kw, n, f"eps/dx {eps_dx} N {n}")
            x = (np.arange(n) + 0.5) * dx
            top_hat = (np.abs(x - 1.0) < 0.5).astype(float)
            e = (np.abs(phi0[0, 0] - top_hat).mean(), np.abs(got[0, 0] - phi0[0, 0]).mean(),
                 np.abs(got[0, 0] - top_hat).mean())
            errs[(eps_dx, n)] = e
            print(f"eps/dx {eps_dx} N {n}: {ns} steps, E_eps {e[0]:.4e} E_delta {e[1]:.4e} "
                  f"E_tot {e[2]:.4e}", flush=True)
    for eps_dx in (1.0, 2.0):
        for n in (100, 200, 400):
            a, b = errs[(eps_dx, n)], errs[(eps_dx, 2 * n)]
            orders = [math.log2(u / v) for u, v in zip(a, b)]
            assert all(0.8 <= o <= 1.2 for o in orders), (eps_dx, n, orders)
    for n in (100, 200, 400, 800):
        assert errs[(1.0, n)][2] < errs[(2.0, n)][2], n


@pytest.mark.parametrize("eps_over_dx,gamma_over_u,bounded", [
    (1.0, 1.0, True), (0.75, 2.0, True), (1.5, 1.0, True), (2.0, 0.5, True),
    (0.55, 1.0, False), (0.8, 0.5, False)])
def test_rk2_boundedness_map_on_the_gpu(lib, eps_over_dx, gamma_over_u, bounded):
    """Sec. 2.3, Fig. 6(a): the explicit midpoint rule at its diffusive limit (Eq. 26) keeps the
    1D drop (diameter 1, u = 1, one period of [0, 2), n = 50) inside [0, 1] at every step for
    points on or above the crossover line (Eq. 9), and leaves it below the line. The extremes
    come from the library's reduction after every step; the final field matches the oracle."""
    pf = lib
    n, L, u = 50, 2.0, 1.0
    dx = L / n
    eps, gamma = eps_over_dx * dx, gamma_over_u * u
    assert (eps_over_dx >= params.crossover_eps_over_dx(gamma_over_u) - 1e-12) == bounded
    x = (np.arange(n) + 0.5) * dx
    phi0 = fx.tanh_profile(0.5 - np.abs(x - L / 2), eps).reshape(1, 1, n)
    U = np.full_like(phi0, u)
    Z = np.zeros_like(phi0)
    ns = math.ceil(L / u / params.dt_max("rk2", 1, dx, gamma, eps))
    dt = L / u / ns
    s = pf.Solver((n, 1, 1), dx, eps, gamma, dt, dtype="f64", scheme="rk2", use_graph=False)
    g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi0, U, Z, Z)]
    st = torch.cuda.Stream()
    lo, hi = 1.0, 0.0
    with torch.cuda.stream(st):
        for k in range(ns):
            s.step(*g, t0=k * dt, nsteps=1, stream=st)
            _, mn, mx, bad = s.reduce(g[0], stream=st)
            assert bad == 0
            lo, hi = min(lo, mn), max(hi, mx)
    got = g[0].cpu().numpy()
    s.close()
    kw = dict(dx=dx, eps=eps, gamma=gamma, dt=dt, nsteps=ns, scheme=2)
    ref = oracle.step(phi0, U, Z, Z, **kw)
    print(f"eps/dx {eps_over_dx} gamma/u {gamma_over_u}: {ns} steps, min {lo:.3e}, "
          f"max-1 {hi - 1:.3e}", flush=True)
    check_against_oracle(got, ref, phi0, (U, Z, Z), kw, ns,
                         f"eps/dx {eps_over_dx} gamma/u {gamma_over_u}")
    if bounded:
        assert lo >= -EPS64 and hi <= 1 + EPS64, (lo, hi)
    else:
        assert lo < -1e-3 and hi > 1 + 1e-3, (lo, hi)


@pytest.mark.parametrize("scheme,sch,limit", [("euler", 1, "euler"), ("rk2", 2, "rk2"),
                                              ("rk3", 3, "rk3"), ("rk4", 4, "rk4")])
def test_boundedness_map_on_the_gpu(lib, scheme, sch, limit):
    """Secs. 2.2-2.3, Figs. 5(a) and 6: the 1D drop (diameter 1, u = 1, one period of [0, 2),
    n = 50) over a grid of (eps/dx, gamma/u) points, each scheme at its diffusive limit
    (Eqs. 25-28). Every point on or above the crossover line (Eq. 9) keeps phi inside
    [0, 1] at every step (proven for Euler, observed by the paper for the Runge-Kutta schemes),
    and its final field matches the oracle (tolerance measured on the oracle, as above). The
    criterion is sufficient, not necessary, so below the line only the existence of unbounded
    points is checked."""
    pf = lib
    n, L, u = 50, 2.0, 1.0
    dx = L / n
    x = (np.arange(n) + 0.5) * dx
    st = torch.cuda.Stream()
    above = below_unbounded = below = 0
    for eod in (0.3, 0.5, 0.7, 0.9, 1.2, 1.6, 2.0):
        for gou in (0.25, 0.5, 1.0, 2.0, 4.0):
            eps, gamma = eod * dx, gou * u
            on_or_above = eod >= params.crossover_eps_over_dx(gou) - 1e-12
            phi0 = fx.tanh_profile(0.5 - np.abs(x - L / 2), eps).reshape(1, 1, n)
            U = np.full_like(phi0, u)
            Z = np.zeros_like(phi0)
            ns = math.ceil(L / u / params.dt_max(limit, 1, dx, gamma, eps))
            dt = L / u / ns
            s = pf.Solver((n, 1, 1), dx, eps, gamma, dt, dtype="f64", scheme=scheme,
                          use_graph=False)
            g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi0, U, Z, Z)]
            lo, hi, bad = 1.0, 0.0, 0
            with torch.cuda.stream(st):
                for k in range(ns):
                    s.step(*g, t0=k * dt, nsteps=1, stream=st)
                    try:
                        _, mn, mx, nb = s.reduce(g[0], stream=st)
                    except pf.PhaseFieldError:  # a run below the line may overflow
                        bad = 1
                        break
                    lo, hi = min(lo, mn), max(hi, mx)
            got = g[0].cpu().numpy()
            s.close()
            bounded = not bad and lo >= -EPS64 and hi <= 1 + EPS64
            if on_or_above:
                above += 1
                assert bounded, (scheme, eod, gou, lo, hi)
                kw = dict(dx=dx, eps=eps, gamma=gamma, dt=dt, nsteps=ns, scheme=sch)
                ref = oracle.step(phi0, U, Z, Z, **kw)
                check_against_oracle(got, ref, phi0, (U, Z, Z), kw, ns, f"{scheme} {eod} {gou}")
            else:
                below += 1
                below_unbounded += not bounded
    print(f"{scheme}: {above} points on or above the line, all bounded; "
          f"{below_unbounded} of {below} below it unbounded", flush=True)
    assert above >= 10 and below_unbounded >= 5


def test_reinitialisation_relaxes_a_top_hat_to_the_tanh_profile(lib):
    """Reinitialisation mode (u = 0; Eq. 1 with only its diffusive and sharpening terms, the
    gamma/|u| -> infinity limit discussed in Sec. 2.3): a 1D top hat of width 1 in [0, 2) relaxes
    to a steady state that keeps the mass, stays in [0, 1], matches the oracle, and approaches
    the tanh profile of the same interfaces as dx is refined at fixed eps (the central scheme's
    O(dx^2) equilibrium error: about 4 x per halving)."""
    pf = lib
    L, eps, gamma = 2.0, 0.02, 1.0
    errs = []
    for n in (100, 200, 400):
        dx = L / n
        x = (np.arange(n) + 0.5) * dx
        top_hat = (np.abs(x - 1.0) < 0.5).astype(float).reshape(1, 1, n)
        Z = np.zeros_like(top_hat)
        dt = 0.9 * params.dt_max("rk4", 1, dx, gamma, eps)
        s = pf.Solver((n, 1, 1), dx, eps, gamma, dt, dtype="f64")
        g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (top_hat, Z, Z, Z)]
        steps, change = 0, 1.0
        while change > 1e-12 and steps < 40000:
            prev = g[0].clone()
            s.step(*g, nsteps=400)
            steps += 400
            change = float((g[0] - prev).abs().max())
        mass, mn, mx, _ = s.reduce(g[0])
        got = g[0].cpu().numpy()
        s.close()
        ref = oracle.step(top_hat, Z, Z, Z, dx=dx, eps=eps, gamma=gamma, dt=dt, nsteps=steps)
        assert np.abs(got - ref).max() <= 1e-12, n
        assert change <= 1e-12 and abs(mass - 1.0) < 1e-12 and mn >= 0.0 and mx <= 1.0
        tanh = fx.tanh_profile(0.5 - np.abs(x - 1.0), eps).reshape(1, 1, n)
        errs.append(np.abs(got - tanh).max())
        print(f"n {n} (eps/dx {eps / dx:.0f}): steady after {steps} steps, max|phi - tanh| "
              f"{errs[-1]:.3e}", flush=True)
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.0 < r < 5.0 for r in ratios), ratios


def test_zalesak_disk_one_revolution(lib):
    """Sec. 3.3.2 on the HIP stepper: the notched disk (R = 15, notch 5 x 25, in a 100 x 100 box;
    the printed "R = 0.15" is read as 15 box units) turned once by u = (pi (50 - y) / 314,
    pi (x - 50) / 314) in t = 628, RK4 at dt = dx/4, eps/dx = 0.7 and gamma / max|u| = 2.5
    (on the crossover line). At N = 100, 200, 400: phi stays in [0, 1] (checked every 8 steps),
    mass is conserved, and the shape error mean|phi(T) - phi(0)| falls with refinement (the
    paper's Fig. 12 shows the same trend). At N = 100 the first quarter turn matches the oracle
    (tolerance measured on the oracle, as above)."""
    pf = lib
    L = 100.0
    errs = []
    for n in (100, 200, 400):
        dx = L / n
        eps = 0.7 * dx
        U, V, W = fx.zalesak_faces(n)
        gamma = 2.5 * fx.max_face_speed(U, V, W)
        phi0 = fx.zalesak_ic(n, eps)
        dt = dx / 4
        ns = int(round(628.0 / dt))
        s = pf.Solver((n, n, 1), dx, eps, gamma, dt, dtype="f64")
        g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi0, U, V, W)]
        st = torch.cuda.Stream()
        lo, hi = 1.0, 0.0
        with torch.cuda.stream(st):
            m0 = s.reduce(g[0], stream=st)[0]
            if n == 100:
                s.step(*g, nsteps=ns // 4, stream=st)
                quarter = g[0].cpu().numpy()
                done = ns // 4
            else:
                done = 0
            while done < ns:
                m = min(8, ns - done)
                s.step(*g, nsteps=m, stream=st)
                done += m
                _, mn, mx, bad = s.reduce(g[0], stream=st)
                assert bad == 0
                lo, hi = min(lo, mn), max(hi, mx)
            m1 = s.reduce(g[0], stream=st)[0]
        got = g[0].cpu().numpy()
        s.close()
        assert lo >= -EPS64 and hi <= 1 + EPS64, (n, lo, hi)
        assert abs(m1 - m0) / m0 < 1e-12, (n, m0, m1)
        errs.append(np.abs(got - phi0).mean())
        print(f"N {n}: {ns} steps, min {lo:.2e}, max-1 {hi - 1:.2e}, shape error {errs[-1]:.4e}",
              flush=True)
        if n == 100:
            kw = dict(dx=dx, eps=eps, gamma=gamma, dt=dt, nsteps=ns // 4)
            ref = oracle.step(phi0, U, V, W, **kw)
            check_against_oracle(quarter, ref, phi0, (U, V, W), kw, n, "Zalesak N 100 quarter turn")
    assert errs[1] < errs[0] and errs[2] < errs[1], errs


@pytest.mark.parametrize("field", ["projected", "stream"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_velocity_field_with_slip_walls(lib, seed, field):
    """Sec. 3.2.2 on the HIP stepper: a D = 1 drop at the centre of a 2 x 2 box with slip walls
    (walls on x and y), a steady velocity that changes randomly from cell to cell, solenoidal,
    with largest face component 1, T = 10, dx = D/25, RK4 at min(Eq. 31, Eq. 32), for the seven
    (eps/dx, gamma/u) points of Table 2. Two constructions of the field: the paper's (random
    point vectors of uniform magnitude and direction, made solenoidal by a Poisson projection with
    no-flux walls) and a random stream function vanishing on the walls. The paper finds every
    point bounded at all times except point 7; so does this run, for each field and seed checked.
    Point 2 is compared with the oracle (bar derived on the oracle, as above)."""
    pf = lib
    pts = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
    n, L, T = 50, 2.0, 10.0
    dx = L / n
    make = fx.random_projected_faces if field == "projected" else fx.random_wall_stream_faces
    U, V, W = make(np.random.default_rng(100 + seed), n, dx)
    walls = (True, True, False)
    st = torch.cuda.Stream()
    for p in pts["points"]:
        eps, gamma = p["eps_over_dx"] * dx, p["gamma_over_u"]
        phi0 = fx.drops_ic((1, n, n), dx, [(1.0, 1.0, 0.0)], [0.5], eps, window=False)
        dt = min(params.dt_rk4_2d_eq31(dx, gamma, eps), params.dt_rk4_2d_eq32(dx, 1.0, 1.0, gamma))
        ns = math.ceil(T / dt)
        dt = T / ns
        s = pf.Solver((n, n, 1), dx, eps, gamma, dt, dtype="f64", walls=walls, use_graph=False)
        g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi0, U, V, W)]
        lo, hi = 1.0, 0.0
        with torch.cuda.stream(st):
            for k in range(ns):
                s.step(*g, nsteps=1, stream=st)
                _, mn, mx, bad = s.reduce(g[0], stream=st)
                assert bad == 0
                lo, hi = min(lo, mn), max(hi, mx)
        got = g[0].cpu().numpy()
        s.close()
        bounded = lo >= -EPS64 and hi <= 1 + EPS64
        print(f"{field} seed {seed} point {p['point']}: {ns} steps, min {lo:.2e}, "
              f"max-1 {hi - 1:.2e}", flush=True)
        assert bounded == (p["point"] != 7), (p["point"], lo, hi)
        if p["point"] == 2:
            kw = dict(dx=dx, eps=eps, gamma=gamma, dt=dt, nsteps=ns, walls=walls)
            ref = oracle.step(phi0, U, V, W, **kw)
            check_against_oracle(got, ref, phi0, (U, V, W), kw, seed,
                                 f"{field} random field seed {seed} point 2")


def test_drop_in_shear_flow_second_order(lib):
    """Sec. 3.3.1 on the HIP stepper: the R = 0.15 drop at (0.5, 0.75) in the reversing single
    vortex (Eq. 33, T = 4), RK4 at dt = dx/8, eps/dx = 0.7 and gamma / max|u| = 2.5 (on the
    crossover line), at N = 64, 128, 256, 512. The paper reports E_shape of Eq. 34 (the L1
    distance between phi(T) and phi(0)) falling at about second order (Fig. 11). A sweep over
    N = 64 ... 1024 (ratios 1.5 and 4/3) shows second order up to N = 256 (least squares 2.4 over
    64-256) and a slower rate above it (1.5 over 128-1024): with eps/dx fixed, the first-order
    floor that Sec. 3.1 explains (the sign switch of n, E_delta ~ dx; and E_eps ~ eps ~ dx) takes
    over at fine meshes; dt = dx/16 changes E_shape at N = 512 by 1e-5 relative, so the rate is
    spatial. Asserted: each of the two doublings up to N = 256 at order >= 1.5, the finest
    doubling at order > 0.5, and the mean order over 64-512 in [1.5, 2.5]; phi stays in [0, 1]
    (checked at t = T/2 and T) and the mass is conserved."""
    pf = lib
    T = 4.0
    errs = []
    for n in (64, 128, 256, 512):
        dx = 1.0 / n
        eps = 0.7 * dx
        U, V, W = fx.vortex2d_faces(n)
        gamma = 2.5 * fx.max_face_speed(U, V, W)
        phi0 = fx.drops_ic((1, n, n), dx, [(0.5, 0.75, 0.0)], [0.15], eps)
        ns = 8 * n * 4  # dt = dx / 8 to t = 4
        dt = T / ns
        s = pf.Solver((n, n, 1), dx, eps, gamma, dt, dtype="f64", vel_mode=1, vel_T=T)
        g = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (phi0, U, V, W)]
        m0, _, _, _ = s.reduce(g[0])
        s.step(*g, t0=0.0, nsteps=ns // 2)
        _, mn_half, mx_half, _ = s.reduce(g[0])
        s.step(*g, t0=T / 2, nsteps=ns - ns // 2)
        m1, mn, mx, _ = s.reduce(g[0])
        got = g[0].cpu().numpy()
        s.close()
        lo, hi = min(mn_half, mn), max(mx_half, mx)
        assert lo >= -EPS64 and hi <= 1 + EPS64, (n, lo, hi)
        assert abs(m1 - m0) / m0 < 1e-12, (n, m0, m1)
        errs.append(np.abs(got - phi0).sum() * dx * dx)
        print(f"N {n}: {ns} steps, E_shape {errs[-1]:.4e}", flush=True)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    mean_order = math.log2(errs[0] / errs[-1]) / (len(errs) - 1)
    print("observed orders", orders, "mean", mean_order, flush=True)
    assert orders[0] >= 1.5 and orders[1] >= 1.5 and orders[2] > 0.5, orders
    assert 1.5 <= mean_order <= 2.5, mean_order


def _drop1d_errors(pf, n, eps, gamma, oracle_check=False):
    """E_eps, E_delta of the 1D drop (D = 1 in [0, 2), u = 1, T = 2, RK4 at 0.9 x Eq. 28), as L1
    norms over the domain, from a GPU run."""
    L, u, T = 2.0, 1.0, 2.0
    dx = L / n
    x = (np.arange(n) + 0.5) * dx
    phi0 = fx.tanh_profile(0.5 - np.abs(x - 1.0), eps).reshape(1, 1, n)
    top_hat = (np.abs(x - 1.0) < 0.5).astype(float)
    U = np.full_like(phi0, u)
    Z = np.zeros_like(phi0)
    dt = 0.9 * params.dt_max("rk4", 1, dx, gamma, eps)
    ns = math.ceil(T / dt)
    dt = T / ns
    got = _gpu_run_1d(pf, phi0, U, dx, eps, gamma, dt, ns)
    if oracle_check:
        ref = oracle.step(phi0, U, Z, Z, dx=dx, eps=eps, gamma=gamma, dt=dt, nsteps=ns)
        assert np.abs(got - ref).max() <= 1e-12
    return (np.abs(phi0[0, 0] - top_hat).sum() * dx, np.abs(got[0, 0] - phi0[0, 0]).sum() * dx)


def test_1d_error_dependences_fig7(lib):
    """Sec. 3.1, Fig. 7, on the HIP stepper (1D drop, RK4, gamma/u = 1 unless varied):
    (b) at fixed dx = 1/320, E_eps is first order in eps (eps = 1/40, 1/80, 1/160) and E_delta
    stays far below it; (c) at fixed eps = dx = 1/400, gamma/u = 1, 2, 4 changes the total error
    by under 10 %; (a) at fixed eps = 1/25, E_eps does not depend on dx and E_delta falls with dx
    (dx = 1/50 .. 1/400). The paper reads (a) as first order; this discretisation gives second
    order there (E_delta ~ dx^2 / eps at fixed eps), first order appearing when eps/dx is held
    fixed (Fig. 8, tested above)."""
    pf = lib
    # (b)
    eb = [_drop1d_errors(pf, 640, eps, 1.0, oracle_check=eps == 1 / 40) for eps in (1 / 40, 1 / 80, 1 / 160)]
    orders_b = [math.log2(eb[i][0] / eb[i + 1][0]) for i in range(2)]
    print("(b) E_eps, E_delta:", eb, "orders", orders_b, flush=True)
    assert all(0.9 <= o <= 1.1 for o in orders_b), orders_b
    assert all(ed < 0.05 * ee for ee, ed in eb)
    # (c)
    ec = [_drop1d_errors(pf, 800, 1 / 400, g) for g in (1.0, 2.0, 4.0)]
    tot = [ee + ed for ee, ed in ec]
    print("(c) E_eps, E_delta:", ec, flush=True)
    assert max(tot) / min(tot) < 1.1, tot
    # (a)
    ea = [_drop1d_errors(pf, n, 1 / 25, 1.0) for n in (100, 200, 400, 800)]
    orders_a = [math.log2(ea[i][1] / ea[i + 1][1]) for i in range(3)]
    print("(a) E_eps, E_delta:", ea, "E_delta orders", orders_a, flush=True)
    assert max(e[0] for e in ea) / min(e[0] for e in ea) < 1.01
    assert all(1.0 <= o <= 2.5 for o in orders_a), orders_a
