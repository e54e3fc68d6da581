#!/usr/bin/env python3
"""Throughput benchmark of the phase-field step on one MI355X.

Workload (default): 512^3 periodic unit cube, FP32 storage, 64 seeded drops (R in [0.03, 0.08]),
a seeded divergence-free 16-mode Fourier velocity (synthesised on the GPU), eps = 0.75 dx,
gamma = 1.1 max|u|, classic RK4. One "step" is one full RK4 step of the whole grid (four stage
launches). Prints ONE JSON line with Gcell-updates/s, the stage kernel's achieved HBM bandwidth
against the 8 TB/s peak, extra measurements (FP64, adjoint/forward cost, batched vs looped) and
the FP64 CPU oracle's throughput on a bounded sample of the same recipe.

  python bench.py [--steps 500] [--warmup 10] [--quick] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s & % HBM peak (fwd, adjoint, batched vs looped) at FP32/FP64 tol"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # dense FP64, MI355X
# Algorithmic words per RK4 cell-update (the roofline's unit): the fixed-buffer stage schedule
# moves 6 + 8 + 8 + 6 = 28 words (stage input, face velocities, bases and accumulator in; stage
# value and accumulator out). The fused two-stage sweeps keep the middle stage value on chip and
# move 6 + 7 = 13 words, which is reported beside it as the fused minimum.
ALG_WORDS = 28
WORDS_PER_CELL_STEP = {"tiled": 28, "global": 28, "fused": 13}
LAUNCHES_PER_STEP = {"tiled": 4, "global": 4, "fused": 2}
GRAPH_STEPS = 8  # steps per captured graph in the library (steady velocity)
# the explicit midpoint rule: per-stage S1 reads phi, U, V, W and writes ya; S2 reads ya, phi, U,
# V, W and writes phi. Fused: one sweep reads phi, U, V, W and writes the new phi.
RK2_WORDS_PER_CELL_STEP = {"tiled": 11, "global": 11, "fused": 5}


def kind(variant_name: str) -> str:
    return variant_name.split("_")[0]
KERNEL_SOURCES = ("paper_1803_01262_amd/csrc/pf_tiled_body.h", "paper_1803_01262_amd/csrc/pf_cell.h",
                  "paper_1803_01262_amd/csrc/stage_tiled.hip", "paper_1803_01262_amd/csrc/pf_fused_body.h",
                  "paper_1803_01262_amd/csrc/pf_fused_launch.h",
                  "paper_1803_01262_amd/csrc/stage_fused_f32.hip",
                  "paper_1803_01262_amd/csrc/stage_fused_f64.hip")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cuda_timer(st, fn, reps=1):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def setup_roofline(pf, fx, n, dtype, st, seed=3):
    """Fields of the roofline workload on the GPU: phi from the seeded drops, faces from the
    library's velocity synthesis; gamma and dt from the synthesised max face speed."""
    import torch
    c = fx.roofline512(n, seed=seed)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    phases, coeffs = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in c.modes)
    p0 = pf.make_params((n, n, n), c.dx, c.eps, 1.0, 1.0, dtype=dtype)
    u, v, w = pf.velocity_from_coeffs(p0, phases, coeffs, stream=st)
    torch.cuda.synchronize()
    umax = max(float(t.abs().max()) for t in (u, v, w))
    fx.set_speed(c, umax)
    phi = torch.tensor(c.phi0, dtype=tdt, device="cuda")
    return c, phi, u, v, w


def time_forward(pf, c, phi, u, v, w, dtype, steps, warmup, st, autotune=True, variant=-1,
                 scheme="rk4", dt=None):
    import torch
    n = c.shape[0]
    s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, c.dt if dt is None else dt, dtype=dtype,
                  variant=variant, scheme=scheme)
    tuned = None
    if autotune and variant < 0:
        best, times = s.autotune(reps=3, stream=st)
        tuned = {k: round(t, 4) for k, t in times.items()}
    with torch.cuda.stream(st):
        # capture and instantiate the step graph before any timed step: one graph-length run,
        # then phi restored in place (the graph is keyed on the buffer addresses)
        keep = phi.clone()
        s.step(phi, u, v, w, nsteps=GRAPH_STEPS, stream=st)
        phi.copy_(keep)
        del keep
        if warmup:
            s.step(phi, u, v, w, nsteps=warmup, stream=st)
        m0 = s.reduce(phi, stream=st)
        ms = cuda_timer(st, lambda: s.step(phi, u, v, w, nsteps=steps, stream=st)) / steps
        m1 = s.reduce(phi, stream=st)
    name = s.variant_name
    s.close()
    return ms, name, tuned, m0, m1


def nonuniform_timing(pf, fx, st, dtype, n=512, steps=20):
    """RK4 on a smoothly stretched n^3 mesh (widths varying 2x along every axis, eps tuned to the
    local mesh): the per-stage kernel's non-uniform form against its uniform form (tiled_64x4)
    on the same grid; and the adjoint step (stage recompute and four reverse stages, velocity
    gradients accumulated) of a handle with the default variant, whose tile shape the tiled
    adjoint takes, on both meshes. Fields and velocity of the roofline workload (timing does not
    depend on the velocity's divergence on the stretched mesh)."""
    import torch
    c, phi, u, v, w = setup_roofline(pf, fx, n, dtype, st)
    h = [fx.smooth_widths(n, 1.0, 2.0, 0.9 * a) for a in range(3)]
    dt = min(c.dt, 0.1 * min(map(min, h)) ** 2 / (c.gamma * c.eps * max(map(max, h)) / c.dx))
    res = {}
    names = [pf.phasefield_variant_name(pf.PF_F32 if dtype == "f32" else pf.PF_F64, k)
             for k in range(pf.phasefield_variant_count(pf.PF_F32 if dtype == "f32" else pf.PF_F64))]
    for label, widths in (("nonuniform", h), ("uniform_tiled_64x4", None)):
        s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, dt, dtype=dtype,
                      variant=names.index("tiled_64x4"))
        if widths is not None:
            s.set_spacing(*widths, eps_mode=1)
        with torch.cuda.stream(st):
            keep = phi.clone()
            s.step(phi, u, v, w, nsteps=GRAPH_STEPS, stream=st)
            ms = cuda_timer(st, lambda: s.step(phi, u, v, w, nsteps=steps, stream=st)) / steps
            phi.copy_(keep)
            del keep
        s.close()
        s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, dt, dtype=dtype)
        if widths is not None:
            s.set_spacing(*widths, eps_mode=1)
        with torch.cuda.stream(st):
            lam = torch.ones_like(phi)
            grads = [torch.zeros_like(phi) for _ in range(3)]
            s.adjoint_step(phi, u, v, w, 0.0, lam, *grads, stream=st)
            ms_adj = cuda_timer(st, lambda: s.adjoint_step(phi, u, v, w, 0.0, lam, *grads,
                                                           stream=st), 5)
            del lam, grads
        s.close()
        esz = 4 if dtype == "f32" else 8
        res[label] = {"ms_per_step": round(ms, 4), "gcell_s": round(c.cells / ms / 1e6, 2),
                      "frac_of_8tbs_28_words": round(ALG_WORDS * esz * c.cells / ms / 1e6 / HBM_PEAK_GBS, 4),
                      "adjoint_ms_default_variant": round(ms_adj, 4)}
    res["nonuniform_over_uniform"] = round(res["nonuniform"]["ms_per_step"] /
                                           res["uniform_tiled_64x4"]["ms_per_step"], 3)
    res["adjoint_nonuniform_over_uniform"] = round(
        res["nonuniform"]["adjoint_ms_default_variant"] /
        res["uniform_tiled_64x4"]["adjoint_ms_default_variant"], 3)
    del phi, u, v, w
    torch.cuda.empty_cache()
    return res


def copy_ceiling(pf, st, nbytes=2 ** 31, reps=10):
    """Read + write bandwidth (GB/s) of a plain device copy of nbytes: torch's copy of float32
    elements and the library's 16-byte streaming copy (phasefield_device_copy)."""
    import torch
    with torch.cuda.stream(st):
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        ms_t = cuda_timer(st, lambda: b.copy_(a), reps)
        pf.phasefield_device_copy(b, a, stream=st)
        ms_l = cuda_timer(st, lambda: pf.phasefield_device_copy(b, a, stream=st), reps)
    del a, b
    torch.cuda.empty_cache()
    return {"torch_copy_gbs": round(2 * nbytes / ms_t / 1e6, 1),
            "library_copy_gbs": round(2 * nbytes / ms_l / 1e6, 1)}


def velocity_timing(pf, fx, st, n=512, dtype="f32", reps=3):
    """Velocity synthesis from the roofline workload's 16-mode potential, and its transpose (the
    coefficient gradient of a face field), one whole library call each (scratch allocation and
    the closing synchronisation included). Floors: the faces written once (3 words per cell at
    8 TB/s) and the last contraction's 3M fused multiply-adds per cell at the FP64 peak."""
    import torch
    c = fx.roofline512(n, seed=3)
    phases, coeffs = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in c.modes)
    M = int(phases.shape[1])
    p0 = pf.make_params((n, n, n), c.dx, c.eps, 1.0, 1.0, dtype=dtype)
    with torch.cuda.stream(st):
        u, v, w = pf.velocity_from_coeffs(p0, phases, coeffs, stream=st)
        synth = cuda_timer(st, lambda: pf.velocity_from_coeffs(p0, phases, coeffs, stream=st), reps)
        pf.velocity_coeffs_grad(p0, phases, u, v, w, stream=st)
        grad = cuda_timer(st, lambda: pf.velocity_coeffs_grad(p0, phases, u, v, w, stream=st), reps)
    cells = n ** 3
    e = 8 if dtype == "f64" else 4
    del u, v, w
    torch.cuda.empty_cache()
    return {"grid": n, "modes": M, "dtype": dtype, "synthesis_ms": round(synth, 3),
            "transpose_ms": round(grad, 3),
            "hbm_floor_ms": round(3 * e * cells / HBM_PEAK_GBS / 1e6, 3),
            "fp64_floor_ms": round(2 * 3 * M * cells / FP64_PEAK_TFLOPS / 1e9, 3)}


def deformation_timing(pf, fx, st, dtype, n=256, steps=100):
    """The 3D deformation workload (256^3, sphere in the reversing deformation field, cos(pi t/T)
    time factor, eps = dx, gamma = max|u|): throughput of the default variant over `steps` steps
    from t = 0 (the loop replayed from one captured graph)."""
    import torch
    c = fx.deformation3d(n)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    phi = torch.tensor(c.phi0, dtype=tdt, device="cuda")
    u, v, w = (torch.tensor(a, dtype=tdt, device="cuda") for a in (c.U, c.V, c.W))
    s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, c.dt, dtype=dtype, vel_mode=c.vel_mode,
                  vel_T=c.vel_T)
    with torch.cuda.stream(st):
        # the same loop once untimed (its whole-loop graph is captured there), phi restored
        keep = phi.clone()
        s.step(phi, u, v, w, t0=0.0, nsteps=steps, stream=st)
        phi.copy_(keep)
        del keep
        ms = cuda_timer(st, lambda: s.step(phi, u, v, w, t0=0.0, nsteps=steps, stream=st)) / steps
    name = s.variant_name
    s.close()
    cells = n ** 3
    e = 8 if dtype == "f64" else 4
    words = WORDS_PER_CELL_STEP[kind(name)]
    return {"grid": n, "dtype": dtype, "steps": steps, "ms_per_step": round(ms, 4),
            "gcell_s": round(cells / ms / 1e6, 2),
            "achieved_gbs": round(ALG_WORDS * e * cells / ms / 1e6, 1),
            "frac_of_8tbs": round(ALG_WORDS * e * cells / ms / 1e6 / HBM_PEAK_GBS, 4),
            "moved_words_per_cell_update": words,
            "moved_frac_of_8tbs": round(words * e * cells / ms / 1e6 / HBM_PEAK_GBS, 4),
            # phi, the accumulator, the middle stage and three face arrays: beside the 256 MB
            # last-level cache, these fractions are partly cache-resident rather than HBM figures
            "working_set_mb": round(6 * e * cells / 2 ** 20, 1),
            "kernel": name}


def vortex_timing(pf, fx, st):
    """The 2D reversing-vortex workload (64 x 64, FP64, RK4, 2556 steps to t = T): a
    launch-bound grid of 4096 cells. Times the full run as specified (time-dependent velocity,
    the whole loop replayed from one captured graph) and, for the launch overhead, the same grid
    with the velocity held steady, eager and replayed from 8-step graphs."""
    import torch
    c = fx.vortex2d(64)
    n = c.shape[2]
    phi0 = torch.tensor(c.phi0, dtype=torch.float64, device="cuda")
    u, v, w = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in (c.U, c.V, c.W))
    out = {"grid": [n, n, 1], "steps": c.nsteps, "dtype": "f64"}
    runs = (("cos_us_per_step", dict(vel_mode=1, vel_T=c.vel_T, use_graph=True)),
            ("steady_eager_us_per_step", dict(use_graph=False)),
            ("steady_graph_us_per_step", dict(use_graph=True)))
    for key, kw in runs:
        s = pf.Solver((n, n, 1), c.dx, c.eps, c.gamma, c.dt, dtype="f64", **kw)
        with torch.cuda.stream(st):
            # the same loop once untimed (graphs are captured there), phi restored in place
            phi = phi0.clone()
            s.step(phi, u, v, w, nsteps=c.nsteps, stream=st)
            phi.copy_(phi0)
            ms = cuda_timer(st, lambda: s.step(phi, u, v, w, nsteps=c.nsteps, stream=st))
        if key == "cos_us_per_step":
            out["e_shape"] = float((phi - phi0).abs().sum()) * c.dx * c.dx
        out[key] = round(1e3 * ms / c.nsteps, 2)
        out["variant"] = s.variant_name
        s.close()
    return out


def adjoint_ratio(pf, fx, dtype, st, n=128, reps=10):
    """Cost of one adjoint step (stage recompute + four reverse stages + velocity gradient) over
    one forward step, on the adjoint workload (128^3, 8-mode field, delta = 1e-3/dx)."""
    import torch
    c = fx.adjoint_case(n)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    phases, coeffs = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in c.modes)
    p0 = pf.make_params((n, n, n), c.dx, c.eps, 1.0, 1.0, dtype=dtype)
    u, v, w = pf.velocity_from_coeffs(p0, phases, coeffs, stream=st)
    torch.cuda.synchronize()
    umax = max(float(t.abs().max()) for t in (u, v, w))
    fx.set_speed(c, umax)
    s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, c.dt, dtype=dtype, delta=c.delta)
    phi = torch.tensor(c.phi0, dtype=tdt, device="cuda")
    lam = torch.randn_like(phi)
    gs = [torch.zeros_like(phi) for _ in range(3)]
    with torch.cuda.stream(st):
        s.step(phi, u, v, w, nsteps=8, stream=st)
        fwd = cuda_timer(st, lambda: s.step(phi, u, v, w, nsteps=1, stream=st), reps)
        s.adjoint_step(phi, u, v, w, 0.0, lam, *gs, stream=st)
        adj = cuda_timer(st, lambda: s.adjoint_step(phi, u, v, w, 0.0, lam, *gs, stream=st), reps)
    s.close()
    return {"fwd_ms": round(fwd, 4), "adjoint_ms": round(adj, 4), "ratio": round(adj / fwd, 3),
            "grid": n, "dtype": dtype}


def rollout_timing(pf, fx, dtype, n=128):
    """The full differentiable rollout of the adjoint workload: 400 steps with a checkpoint
    every 20, loss 0.5 ||phi_T - target||^2, gradients for phi_0 and the 8^3 x 3 velocity
    coefficients. Times the forward (velocity synthesis, steps, checkpoint copies) and the
    backward (segment re-runs, 400 adjoint steps, projection onto the coefficients), on the
    current stream: the default backward, whose re-runs keep the stage inputs for the adjoint
    steps, the one whose adjoint steps recompute them, and (keep_all) a forward that keeps every
    state and stage input so that the backward is the reverse sweep alone. Each form runs twice
    and its faster run counts."""
    import torch
    c = fx.adjoint_case(n)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    phases, coeffs = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in c.modes)
    p0 = pf.make_params((n, n, n), c.dx, c.eps, 1.0, 1.0, dtype=dtype)
    u, v, w = pf.velocity_from_coeffs(p0, phases, coeffs)
    torch.cuda.synchronize()
    fx.set_speed(c, max(float(t.abs().max()) for t in (u, v, w)))
    s = pf.Solver((n, n, n), c.dx, c.eps, c.gamma, c.dt, dtype=dtype, delta=c.delta)
    phi0 = torch.tensor(c.phi0, dtype=tdt, device="cuda").requires_grad_(True)
    cf = coeffs.clone().requires_grad_(True)
    target = torch.tensor(c.extra["target"], dtype=tdt, device="cuda")

    def run(nsteps, cache, keep_all=False):
        phi0.grad = None
        cf.grad = None
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        ev[0].record()
        phiT = pf.Rollout.apply(phi0, cf, s, phases, nsteps, 20, 0.0, cache, keep_all)
        loss = 0.5 * ((phiT - target) ** 2).sum()
        ev[1].record()
        loss.backward()
        ev[2].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])

    # warm-up: one short rollout each way (first launches of every kernel, graph capture)
    run(20, True)
    run(20, False)
    run(20, None, True)
    # each form twice: a forward whose state buffer landed at a new address re-captures its
    # step graph, so the faster run of each form counts
    rec = [run(c.nsteps, False), run(c.nsteps, None, True), run(c.nsteps, True)]
    rec += [run(c.nsteps, False), run(c.nsteps, None, True), run(c.nsteps, True)]
    # the checkpointed forward (the same in both forms): the denominator of every ratio
    fwd = min(rec[0][0], rec[2][0], rec[3][0], rec[5][0])
    bwd_r = min(rec[0][1], rec[3][1])
    fwd_k, bwd_k = min(rec[1], rec[4], key=sum)
    bwd = min(rec[2][1], rec[5][1])
    out = {"grid": n, "dtype": dtype, "steps": c.nsteps, "checkpoint_every": 20,
           "forward_ms": round(fwd, 2), "backward_ms": round(bwd, 2),
           "backward_over_forward": round(bwd / fwd, 3),
           "backward_ms_recomputing_stages": round(bwd_r, 2),
           "backward_over_forward_recomputing_stages": round(bwd_r / fwd, 3),
           # the forward keeping every state and stage input (no checkpoints, no re-run)
           "keep_all": {"forward_ms": round(fwd_k, 2), "backward_ms": round(bwd_k, 2),
                        "backward_over_checkpointed_forward": round(bwd_k / fwd, 3),
                        "total_over_checkpointed_total": round((fwd_k + bwd_k) / (fwd + bwd), 3)},
           "grad_finite": bool(torch.isfinite(phi0.grad).all() and torch.isfinite(cf.grad).all())}
    s.close()
    return out


def batch_vs_loop(pf, fx, st, count=96, nsteps=300):
    """The batched driver (default mode, both modes forced, and the autotuned shape and launch
    form, the figure of record) against a loop of single solves (each its own handle, one
    stream, no graphs), on the same uneven FP32 instances; then RK3, RK2 and Euler batches of
    the same instances against their loops."""
    import torch
    cases = fx.batch_cases(count=count, nsteps=nsteps)
    params, fields = [], []
    for c in cases:
        n = c.shape[0]
        phases, coeffs = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in c.modes)
        p0 = pf.make_params((n, n, n), c.dx, c.eps, 1.0, 1.0, dtype="f32")
        u, v, w = pf.velocity_from_coeffs(p0, phases, coeffs, stream=st)
        torch.cuda.synchronize()
        fx.set_speed(c, max(float(t.abs().max()) for t in (u, v, w)))
        params.append(pf.make_params((n, n, n), c.dx, c.eps, c.gamma, c.dt, dtype="f32"))
        fields.append([torch.tensor(c.phi0, dtype=torch.float32, device="cuda"), u, v, w])
    cells = sum(int(c.cells) for c in cases)
    # batched: default mode, then each mode forced through instance 0's variant
    names = [pf.phasefield_variant_name(pf.PF_F32, v)
             for v in range(pf.phasefield_variant_count(pf.PF_F32))]
    modes = {}
    for mode, pick, persistent in (("default", -1, False),
                                   ("fused", names.index("fused_32x16x32"), False),
                                   ("per_stage", names.index("tiled_64x8x16"), False),
                                   ("fused_persistent", names.index("fused_32x16x32"), True),
                                   ("per_stage_persistent", names.index("tiled_64x8x16"), True)):
        params[0].variant = pick
        bs = pf.BatchSolver(params)
        bs.set_persistent(persistent)
        bf = [[f[0].clone(), f[1], f[2], f[3]] for f in fields]
        with torch.cuda.stream(st):
            # 50 untimed steps: capture, and the first replays after the mode switch
            bs.step(*zip(*bf), nsteps=50, stream=st)
            modes[mode] = cuda_timer(st, lambda: bs.step(*zip(*bf), nsteps=nsteps, stream=st))
        bs.close()
    params[0].variant = -1
    # the shape and launch form the batch autotuner picks (every combination timed on private
    # fields), then timed like the modes above: the batched figure of record
    bs = pf.BatchSolver(params)
    pick_shape, pick_pers, tune_times = bs.autotune(reps=2, stream=st)
    bf = [[f[0].clone(), f[1], f[2], f[3]] for f in fields]
    with torch.cuda.stream(st):
        bs.step(*zip(*bf), nsteps=50, stream=st)
        modes["autotuned"] = cuda_timer(st, lambda: bs.step(*zip(*bf), nsteps=nsteps, stream=st))
    bs.close()
    t_batch = modes["autotuned"]
    # looped single solves, uncaptured
    solvers = [pf.Solver(tuple(p.n), p.dx, p.eps, p.gamma, p.dt, dtype="f32", use_graph=False)
               for p in params]
    lf = [[f[0].clone(), f[1], f[2], f[3]] for f in fields]

    def loop(steps):
        for s, f in zip(solvers, lf):
            s.step(*f, nsteps=steps, stream=st)

    with torch.cuda.stream(st):
        loop(2)
        t_loop = cuda_timer(st, lambda: loop(nsteps))
    # looped single solves, each replayed from its own captured graph
    gsolvers = [pf.Solver(tuple(p.n), p.dx, p.eps, p.gamma, p.dt, dtype="f32", use_graph=True)
                for p in params]
    gf = [[f[0].clone(), f[1], f[2], f[3]] for f in fields]

    def gloop(steps):
        for s, f in zip(gsolvers, gf):
            s.step(*f, nsteps=steps, stream=st)

    with torch.cuda.stream(st):
        gloop(8)
        t_gloop = cuda_timer(st, lambda: gloop(nsteps))
    for s in solvers + gsolvers:
        s.close()
    # the other schemes (per-stage sweeps, one launch per stage), 100 steps at 0.9 of each
    # instance's stability limit for that scheme, against the uncaptured loop
    other = {}
    for scheme in ("rk3", "rk2", "euler"):
        sp = []
        for c, p in zip(cases, params):
            q = pf.make_params(tuple(p.n), p.dx, p.eps, p.gamma, p.dt, dtype="f32", scheme=scheme)
            q.dt = 0.9 * min(c.dt, pf.phasefield_check_params(q, c.extra["umax"]).dt_max_scheme)
            sp.append(q)
        steps = 100
        bs = pf.BatchSolver(sp)
        bf = [[f[0].clone(), f[1], f[2], f[3]] for f in fields]
        with torch.cuda.stream(st):
            bs.step(*zip(*bf), nsteps=16, stream=st)
            tb = cuda_timer(st, lambda: bs.step(*zip(*bf), nsteps=steps, stream=st))
        bs.close()
        ss = [pf.Solver(tuple(q.n), q.dx, q.eps, q.gamma, q.dt, dtype="f32", scheme=scheme,
                        use_graph=False) for q in sp]
        sf = [[f[0].clone(), f[1], f[2], f[3]] for f in fields]

        def sloop(k):
            for s, f in zip(ss, sf):
                s.step(*f, nsteps=k, stream=st)

        with torch.cuda.stream(st):
            sloop(2)
            tl = cuda_timer(st, lambda: sloop(steps))
        for s in ss:
            s.close()
        other[scheme] = {"steps": steps, "batched_ms": round(tb, 2), "looped_ms": round(tl, 2),
                         "batched_gcell_s": round(cells * steps / tb / 1e6, 2),
                         "speedup_vs_looped": round(tl / tb, 2)}
    return {"instances": count, "cells": cells, "steps": nsteps,
            "batched_ms": round(t_batch, 2), "looped_ms": round(t_loop, 2),
            "looped_graph_ms": round(t_gloop, 2),
            "batched_gcell_s": round(cells * nsteps / t_batch / 1e6, 2),
            "batched_mode_ms": {k: round(v, 2) for k, v in modes.items()},
            "autotune": {"shape": pick_shape, "persistent": pick_pers,
                         "ms_per_step": {f"{k[0]}{'_persistent' if k[1] else ''}": round(v, 4)
                                         for k, v in tune_times.items()}},
            "looped_gcell_s": round(cells * nsteps / t_loop / 1e6, 2),
            "speedup_vs_looped": round(t_loop / t_batch, 2),
            "speedup_vs_looped_graph": round(t_gloop / t_batch, 2),
            "other_schemes": other}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(fx, n=128, budget_s=12.0, n1=64, budget1_s=8.0):
    """The FP64 oracle (FP32-storage mode, RK4) timed on the host: on every core on a 128^3
    instance of the same recipe, RK4 steps until about budget_s seconds have passed, and on one
    thread on a 64^3 instance for about budget1_s seconds."""
    import numpy as np

    import oracle

    def rate(m, threads, budget):
        c = fx.roofline512(m, seed=3)
        U, V, W = fx.fourier_faces(c.shape, c.dx, *c.modes)
        fx.set_speed(c, fx.max_face_speed(U, V, W))
        U, V, W, phi = (a.astype(np.float32).astype(np.float64) for a in (U, V, W, c.phi0))
        kw = dict(dx=c.dx, eps=c.eps, gamma=c.gamma, dt=c.dt, fp32=True)
        oracle.set_threads(threads)
        used = oracle.max_threads()
        phi = oracle.step(phi, U, V, W, nsteps=1, **kw)  # warm-up
        steps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget:
            phi = oracle.step(phi, U, V, W, nsteps=1, **kw)
            steps += 1
        el = time.perf_counter() - t0
        return c.cells * steps / el / 1e9, steps, el, used

    def thr(k):
        return f"{k} thread" + ("s" if k != 1 else "")

    def fixed(c, U, V, W, threads, nsteps, scheme=4, vel_mode=0, vel_T=1.0, fp32=False):
        oracle.set_threads(threads)
        used = oracle.max_threads()
        t0 = time.perf_counter()
        oracle.step(c.phi0, U, V, W, dx=c.dx, eps=c.eps, gamma=c.gamma, dt=c.dt, nsteps=nsteps,
                    scheme=scheme, vel_mode=vel_mode, vel_T=vel_T, fp32=fp32)
        el = time.perf_counter() - t0
        return round(c.cells * nsteps / el / 1e9, 6), round(el, 2), used

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    v_all, steps, el, used = rate(n, cores, budget_s)
    v_one, steps1, el1, _ = rate(n1, 1, budget1_s)
    # the other sizes of the same recipe, FP64 oracle arithmetic in FP32-storage mode: 64^3 on
    # every core (as many steps as the one-thread run took), 256^3 for 10 steps on every core;
    # and the 2D reversing vortex (64 x 64, FP64, RK4, its whole run) on every core and one thread
    runs = {}
    c64 = fx.roofline512(n1, seed=3)
    f64 = fx.fourier_faces(c64.shape, c64.dx, *c64.modes)
    fx.set_speed(c64, fx.max_face_speed(*f64))
    r = fixed(c64, *f64, cores, max(steps1, 1), fp32=True)
    runs[f"{n1}^3, {thr(r[2])}"] = {"gcell_s": r[0], "steps": max(steps1, 1), "seconds": r[1]}
    c256 = fx.roofline512(256, seed=3)
    f256 = fx.fourier_faces(c256.shape, c256.dx, *c256.modes)
    fx.set_speed(c256, fx.max_face_speed(*f256))
    r = fixed(c256, *f256, cores, 10, fp32=True)
    runs[f"256^3, {thr(r[2])}"] = {"gcell_s": r[0], "steps": 10, "seconds": r[1]}
    del c256, f256
    cv = fx.vortex2d(64)
    for th in (cores, 1):
        r = fixed(cv, cv.U, cv.V, cv.W, th, cv.nsteps, vel_mode=1, vel_T=cv.vel_T)
        runs[f"vortex 64^2 FP64, {thr(r[2])}"] = {"gcell_s": r[0], "steps": cv.nsteps,
                                                     "seconds": r[1]}
    oracle.set_threads(cores)
    return {"value": round(v_all, 5), "unit": "Gcell-updates/s", "cores": used, "kind": "oracle",
            "sample": f"{n}^3 instance of the same recipe (64 drops, 16 modes, eps=0.75dx, "
                      f"gamma=1.1max|u|), FP32-storage RK4, {steps} steps in {el:.1f} s on "
                      f"{used} threads",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": round(v_one, 6), "unit": "Gcell-updates/s",
                              "sample": f"{n1}^3 instance, {steps1} steps in {el1:.1f} s, "
                                        "1 thread"},
            "other_runs": runs}


def stored_traffic(khash: str, vname: str, n: int = 512, dtype: str = "f32"):
    """HBM bytes per launch from the committed counter summary, if it was taken on this exact
    kernel source and variant (else None)."""
    f = os.path.join(ROOT, "profiles", f"stage_traffic_roofline{n}_{dtype}.json")
    if not os.path.exists(f):
        return None
    d = json.load(open(f))
    if d.get("kernel_hash") != khash or d.get("kernel") != vname:
        return None
    return d["bytes_per_launch"]


def _counter_values(d: str, counter: str) -> dict:
    """Per kernel name, the values of one counter for each dispatch in dispatch order, from the
    counter_collection CSV files of a rocprofv3 --pmc run under directory d (the rows of one
    dispatch are summed)."""
    import csv
    import glob
    per = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                key = (f, int(row["Dispatch_Id"]))
                per.setdefault(key, [row["Kernel_Name"], 0.0])
                per[key][1] += float(row["Counter_Value"])
    out = {}
    for key in sorted(per):
        name, v = per[key]
        out.setdefault(name, []).append(v)
    return out


def write_traffic(args):
    """HBM bytes per launch of the stage kernel of this benchmark's workload, from FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads for the
    library copy of --traffic-copy-bytes bytes (the probe: the first copy16 dispatch of the run;
    later ones are the copy-ceiling measurement)."""
    fetch = _counter_values(args.traffic_from[0], "FETCH_SIZE")
    write = _counter_values(args.traffic_from[1], "WRITE_SIZE")
    copy_name = next(k for k in fetch if "copy16_kernel" in k)
    ffac = args.traffic_copy_bytes / (fetch[copy_name][0] * 1024.0)
    wfac = args.traffic_copy_bytes / (write[copy_name][0] * 1024.0)
    esz = 4 if args.dtype == "f32" else 8
    n = args.n
    cells = n ** 3
    # the timed steps' kernels: the plain sweeps (fused_kernel<T, TX, TY, SWEEP_B, BIG, WIDE,
    # XOUT, WALLS>; the form with the optional outputs, XOUT, only ends odd step counts) or the
    # per-stage kernel
    def plain_sweep(k):
        targs = [t.strip() for t in k.split("<", 1)[1].split(">")[0].split(",")]
        return targs[6] == "false" and targs[7] == "false"

    stage = sorted(k for k in fetch if ("fused_kernel" in k and plain_sweep(k))
                   or "stage_kernel" in k)
    sweeps = {}
    for k in stage:
        fk = sum(fetch[k]) / len(fetch[k])
        wk = sum(write.get(k, [0.0])) / len(write.get(k, [0.0]))
        sweeps[k] = {"fetch_kib_raw": fk, "write_kib_raw": wk,
                     "bytes": int(fk * 1024 * ffac + wk * 1024 * wfac)}
    per_launch = sum(v["bytes"] for v in sweeps.values()) / len(sweeps)
    fused = any("fused_kernel" in k for k in stage)
    moved = (6.5 if fused else 7.0) * esz * cells
    out = {"kernel": args.traffic_variant, "kernel_name": stage, "dtype": args.dtype,
           "grid": [n, n, n], "kernel_hash": kernel_hash(), "sweeps": sweeps,
           "fetch_calibration": {"factor": round(ffac, 4), "kernel": copy_name,
                                 "bytes": args.traffic_copy_bytes, "fetch_kib": fetch[copy_name][0]},
           "write_calibration": {"factor": round(wfac, 4), "kernel": copy_name,
                                 "bytes": args.traffic_copy_bytes, "write_kib": write[copy_name][0]},
           "bytes_per_launch": int(per_launch), "moved_bytes_per_launch": int(moved),
           "counter_over_moved": round(per_launch / moved, 4),
           "commands": [f"rocprofv3 --pmc {c} -d {d} -o bench "
                        f"--output-format csv -- python3 bench.py --steps 3 --warmup 1 --quick "
                        f"--no-cpu-baseline --no-autotune --dtype {args.dtype} "
                        f"--copy-probe {args.traffic_copy_bytes}"
                        for c, d in zip(("FETCH_SIZE", "WRITE_SIZE"), args.traffic_from)]
                       + [f"python3 bench.py --traffic-from {args.traffic_from[0]} "
                          f"{args.traffic_from[1]} --dtype {args.dtype} "
                          f"--traffic-variant {args.traffic_variant}"],
           "note": "means over the dispatches of each sweep; factors scale the raw KiB counters "
                   "to bytes by the library copy of known size"}
    path = os.path.join(ROOT, "profiles", f"stage_traffic_roofline{n}_{args.dtype}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the FP64/adjoint/batch extras")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="", metavar="PARTS",
                    help="comma-separated subset of {adjoint, batch, velocity, vortex, rollout, "
                         "deformation, nonuniform}: "
                         "run only those measurements and print their JSON (for profiling "
                         "them)")
    ap.add_argument("--batch-steps", type=int, default=300)
    ap.add_argument("--adjoint-n", type=int, default=128,
                    help="grid of the adjoint measurement in --only adjoint")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="also run one library copy of BYTES bytes (hardware-counter "
                         "calibration: its FETCH_SIZE/WRITE_SIZE should read BYTES each)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: read two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "this benchmark with --copy-probe, and write the HBM traffic per launch "
                         "of the dominant kernel to profiles/stage_traffic_<workload>.json")
    ap.add_argument("--traffic-copy-bytes", type=int, default=2 ** 30)
    ap.add_argument("--traffic-variant", default="fused_64x8",
                    help="name of the variant the --pmc runs timed (recorded in the json)")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the method runs on one device here; multi-GPU slab "
              "decomposition is a design note only. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1803_01262_amd as pf
    import pf_fixtures as fx

    st = torch.cuda.Stream()
    if args.only:
        parts = {x.strip() for x in args.only.split(",") if x.strip()}
        unknown = parts - {"adjoint", "batch", "velocity", "vortex", "rollout", "deformation",
                           "nonuniform"}
        if unknown:
            print(f"--only: unknown parts {sorted(unknown)}", file=sys.stderr)
            sys.exit(2)
        res = {}
        if "adjoint" in parts:
            na = args.adjoint_n
            for dt_ in ("f64", "f32") if args.dtype == "f32" else ("f64",):
                res[f"adjoint_{na}_{dt_}"] = adjoint_ratio(pf, fx, dt_, st, n=na,
                                                         reps=20 if na <= 256 else 5)
        if "batch" in parts:
            res["batch96_f32"] = batch_vs_loop(pf, fx, st, nsteps=args.batch_steps)
        if "deformation" in parts:
            res["deformation256_f64"] = deformation_timing(pf, fx, st, "f64")
            res["deformation256_f32"] = deformation_timing(pf, fx, st, "f32")
        if "rollout" in parts:
            res["rollout_128_f64"] = rollout_timing(pf, fx, "f64")
            res["rollout_128_f32"] = rollout_timing(pf, fx, "f32")
        if "vortex" in parts:
            res["vortex64_f64"] = vortex_timing(pf, fx, st)
        if "velocity" in parts:
            res[f"velocity_{args.n}_{args.dtype}"] = velocity_timing(pf, fx, st, n=args.n,
                                                                   dtype=args.dtype)
        if "nonuniform" in parts:
            for dt_ in ("f32", "f64"):
                res[f"nonuniform_{args.n}_{dt_}"] = nonuniform_timing(pf, fx, st, dt_, n=args.n)
        print(json.dumps(res), flush=True)
        return
    if args.copy_probe:
        # one library copy of known size (pf::copy16_kernel): BYTES read and BYTES written
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        pf.phasefield_device_copy(dst, src)
        torch.cuda.synchronize()
        del src, dst
    n = args.n
    esz = 4 if args.dtype == "f32" else 8
    log(f"setup {n}^3 {args.dtype}")
    c, phi, u, v, w = setup_roofline(pf, fx, n, args.dtype, st)
    log("timing forward")
    ms, vname, tuned, m0, m1 = time_forward(pf, c, phi, u, v, w, args.dtype, args.steps,
                                            args.warmup, st, autotune=not args.no_autotune,
                                            variant=args.variant)
    cells = c.cells
    value = cells / ms / 1e6  # Gcell-updates/s
    words, launches = WORDS_PER_CELL_STEP[kind(vname)], LAUNCHES_PER_STEP[kind(vname)]
    # every step is exactly `launches` launches of the dominant kernel (graph replays and eager
    # steps alike), so the average launch takes ms / launches; algorithmic bytes per launch are
    # the 28-word cell-update split evenly over them
    launch_ms = ms / launches
    launch_bytes = ALG_WORDS * esz * cells / launches
    achieved = launch_bytes / launch_ms / 1e6  # GB/s
    khash = kernel_hash()
    tr = stored_traffic(khash, vname, n, args.dtype)
    fused_bytes = words * esz * cells / launches
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": tr, "algorithmic_words_per_cell_update": ALG_WORDS,
            "algorithmic_bytes_per_launch": int(launch_bytes), "launches_per_step": launches,
            "avg_launch_ms": round(launch_ms, 4), "kernel": vname, "kernel_hash": khash,
            "moved_words_per_cell_update": words,
            "moved_gbs": round(fused_bytes / launch_ms / 1e6, 1),
            "moved_frac": round(fused_bytes / launch_ms / 1e6 / HBM_PEAK_GBS, 4)}
    if tr:
        roof["counter_gbs"] = round(tr / launch_ms / 1e6, 1)
        roof["counter_frac"] = round(tr / launch_ms / 1e6 / HBM_PEAK_GBS, 4)
        roof["counter_over_moved"] = round(tr / fused_bytes, 3)
    del phi, u, v, w
    torch.cuda.empty_cache()
    cc = copy_ceiling(pf, st)
    roof["copy_ceiling"] = cc
    roof["moved_frac_of_library_copy"] = round(roof["moved_gbs"] / cc["library_copy_gbs"], 4)
    extras = {"tile_autotune_ms_per_step": tuned,
              "mass_drift_timed_region": (m1[0] - m0[0]) / m0[0], "min": m1[1], "max": m1[2],
              "eq17_margin": c.eps / c.dx - (c.gamma + c.extra["umax"]) / (2 * c.gamma)}
    if not args.quick:
        log("timing FP64")
        other = "f64" if args.dtype == "f32" else "f32"
        c2, phi2, u2, v2, w2 = setup_roofline(pf, fx, n, other, st)
        ms2, vname2, _, _, _ = time_forward(pf, c2, phi2, u2, v2, w2, other, min(args.steps, 200),
                                            5, st, autotune=not args.no_autotune)
        e2 = 8 if other == "f64" else 4
        w2 = WORDS_PER_CELL_STEP[kind(vname2)]
        extras[f"{other}_{n}"] = {"ms_per_step": round(ms2, 4),
                                  "gcell_s": round(cells / ms2 / 1e6, 2),
                                  "achieved_gbs": round(ALG_WORDS * e2 * cells / ms2 / 1e6, 1),
                                  "frac_of_8tbs": round(ALG_WORDS * e2 * cells / ms2 / 1e6 / HBM_PEAK_GBS, 4),
                                  "moved_words_per_cell_update": w2,
                                  "moved_frac_of_8tbs": round(w2 * e2 * cells / ms2 / 1e6 / HBM_PEAK_GBS, 4),
                                  "kernel": vname2}
        del phi2, u2, v2, w2
        torch.cuda.empty_cache()
        log("timing RK2")
        c3, phi3, u3, v3, w3 = setup_roofline(pf, fx, n, args.dtype, st)
        # the explicit midpoint rule at 0.9 x its diffusive limit (Eq. 26, three axes)
        dt_rk2 = min(c3.dt, 0.9 * c3.dx * c3.dx / (6.0 * c3.gamma * c3.eps))
        ms3, vname3, _, _, _ = time_forward(pf, c3, phi3, u3, v3, w3, args.dtype,
                                            min(args.steps, 200), 5, st, autotune=False,
                                            scheme="rk2", dt=dt_rk2)
        e3 = 8 if args.dtype == "f64" else 4
        w3 = RK2_WORDS_PER_CELL_STEP[kind(vname3)]
        extras[f"rk2_{n}_{args.dtype}"] = {"ms_per_step": round(ms3, 4),
                                           "gcell_s": round(cells / ms3 / 1e6, 2),
                                           "achieved_gbs": round(w3 * e3 * cells / ms3 / 1e6, 1),
                                           "frac_of_8tbs": round(w3 * e3 * cells / ms3 / 1e6 / HBM_PEAK_GBS, 4),
                                           "words_per_cell_step": w3, "kernel": vname3}
        del phi3, u3, v3, w3
        torch.cuda.empty_cache()
        log("timing the 3D deformation workload")
        extras["deformation256_f64"] = deformation_timing(pf, fx, st, "f64")
        extras["deformation256_f32"] = deformation_timing(pf, fx, st, "f32")
        log("timing the 2D vortex")
        extras["vortex64_f64"] = vortex_timing(pf, fx, st)
        log("timing velocity synthesis")
        extras[f"velocity_{n}_{args.dtype}"] = velocity_timing(pf, fx, st, n=n, dtype=args.dtype)
        log("timing the non-uniform mesh")
        extras[f"nonuniform_{n}_{args.dtype}"] = nonuniform_timing(pf, fx, st, args.dtype, n=n)
        log("timing adjoint")
        extras["adjoint_128_f64"] = adjoint_ratio(pf, fx, "f64", st)
        extras["adjoint_128_f32"] = adjoint_ratio(pf, fx, "f32", st)
        log("timing the checkpointed rollout")
        extras["rollout_128_f64"] = rollout_timing(pf, fx, "f64")
        extras["rollout_128_f32"] = rollout_timing(pf, fx, "f32")
        log("timing batch vs loop")
        extras["batch96_f32"] = batch_vs_loop(pf, fx, st, nsteps=args.batch_steps)
        if args.dtype == "f32":
            extras["batch96_f32"]["best_single_grid_gcell_s"] = round(value, 2)
            extras["batch96_f32"]["batched_over_best_single_grid"] = round(
                extras["batch96_f32"]["batched_gcell_s"] / value, 3)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing CPU oracle")
        cpu = cpu_baseline(fx)
    out = {"metric": METRIC, "value": round(value, 3), "unit": "Gcell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": f"roofline{n}: {n}^3 periodic unit cube, {args.dtype} storage, "
                                  "64 drops R~U[0.03,0.08], 16-mode solenoidal Fourier velocity "
                                  "(unit RMS), eps=0.75dx, gamma=1.1max|u|, RK4",
                      "grid": [n, n, n], "cells": cells, "eps_over_dx": 0.75,
                      "gamma_over_umax": 1.1, "dt": c.dt, "parallelism": "single GPU"},
           "roofline": roof, "cpu_baseline": cpu, "extras": extras}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
