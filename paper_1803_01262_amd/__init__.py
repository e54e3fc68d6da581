"""MI355X (gfx950) library for the conservative, bounded phase-field method of
Mirjalili, Ivey & Mani (arXiv:1803.01262): the explicit flux-form step of Eq. 1 on a staggered
grid (Sec. 2.2), its discrete adjoint, a batched multi-instance driver and velocity synthesis.

Everything runs in libphasefield.so (hand-written HIP kernels, C ABI in include/phasefield.h);
this package marshals torch tensors to it. Importing the package fails if the library has not
been built — there is no fallback path.
"""
from __future__ import annotations

import ctypes

import torch

from ._capi import (EXPORTED, PF_BC_PERIODIC, PF_BC_WALL, PF_ERR_DEVICE, PF_ERR_INVALID,  # noqa: F401
                    PF_ERR_NONFINITE, PF_ERR_OOM, PF_ERR_UNSUPPORTED, PF_EULER, PF_F32, PF_F64, PF_RK2, PF_RK3,
                    PF_OK, PF_RK4, PF_VEL_COS_REVERSAL, PF_VEL_STEADY, LIB_PATH, Params,
                    PhaseFieldError, Report, cells, lib, make_params, phasefield_adjoint_step,
                    phasefield_autotune, phasefield_batch_create, phasefield_batch_destroy,
                    phasefield_batch_step, phasefield_batch_set_persistent,
                    phasefield_batch_set_shape, phasefield_batch_autotune,
                    phasefield_check_params, phasefield_create,
                    phasefield_default_params, phasefield_destroy, phasefield_last_error,
                    phasefield_reduce, phasefield_set_adjoint_form, phasefield_set_spacing,
                    phasefield_solver_variant, phasefield_step, phasefield_step_stages,
                    phasefield_adjoint_step_stages,
                    phasefield_step_noalloc, phasefield_noalloc_scratch_bytes, phasefield_device_copy,
                    phasefield_variant_count, phasefield_variant_name,
                    phasefield_velocity_coeffs_grad, phasefield_velocity_from_coeffs)

TORCH_DTYPE = {PF_F32: torch.float32, PF_F64: torch.float64}
STAGE_COUNT = {PF_RK4: 3, PF_RK3: 2, PF_RK2: 1, PF_EULER: 0}  # stage inputs kept for the adjoint


class Solver:
    """One simulation handle: grid, eps, gamma, dt, scheme, storage dtype (pf_params)."""

    def __init__(self, n, dx, eps, gamma, dt, **kw):
        self.params = make_params(n, dx, eps, gamma, dt, **kw)
        self.handle = phasefield_create(self.params)

    @property
    def shape(self):
        p = self.params
        return (int(p.n[2]), int(p.n[1]), int(p.n[0]))

    @property
    def dtype(self) -> torch.dtype:
        return TORCH_DTYPE[self.params.dtype]

    @property
    def dt(self) -> float:
        return float(self.params.dt)

    @property
    def variant(self) -> int:
        return phasefield_solver_variant(self.handle)

    def step(self, phi, u, v, w, t0=0.0, nsteps=1, stream=None):
        """Advance phi in place by nsteps steps from time t0."""
        phasefield_step(self.handle, self.params, phi, u, v, w, t0, nsteps, stream)
        return phi

    def adjoint_step(self, phi_n, u, v, w, t_n, lam, gu=None, gv=None, gw=None, stream=None):
        """lam <- dL/dphi_n given lam = dL/dphi_{n+1}; gu/gv/gw accumulate dL/du0 (in place)."""
        phasefield_adjoint_step(self.handle, self.params, phi_n, u, v, w, t_n, lam, gu, gv, gw,
                                stream)
        return lam

    @property
    def stage_count(self) -> int:
        """Stage inputs one step keeps for its adjoint (RK4 3, RK3 2, RK2 1, Euler 0)."""
        return STAGE_COUNT[self.params.scheme]

    def step_stages(self, phi, u, v, w, t, *stages, phi_next=None, stream=None):
        """One step from time t that also writes its stage inputs into the stage_count tensors
        given (y2, y3, y4 as the scheme uses them); the new phi into phi_next (None: phi in
        place). Returns the new phi."""
        ys = list(stages) + [None] * (3 - len(stages))
        phasefield_step_stages(self.handle, self.params, phi, u, v, w, t, *ys[:3], stream,
                               phi_next)
        return phi if phi_next is None else phi_next

    def adjoint_step_stages(self, phi_n, stages, u, v, w, t_n, lam, gu=None, gv=None, gw=None,
                            stream=None):
        """adjoint_step with the stage inputs kept by step_stages at (phi_n, t_n): no
        recompute, the same results bit for bit."""
        ys = list(stages) + [None] * (3 - len(stages))
        phasefield_adjoint_step_stages(self.handle, self.params, phi_n, *ys[:3], u, v, w, t_n,
                                       lam, gu, gv, gw, stream)
        return lam

    def set_spacing(self, hx=None, hy=None, hz=None, eps_mode: int = 0) -> None:
        """Non-uniform rectilinear mesh: cell widths per axis (x: nx values, ...), or all None
        for the uniform mesh; eps_mode 0 keeps eps, 1 scales it with each cell's largest width
        (relative to dx)."""
        phasefield_set_spacing(self.handle, self.params, hx, hy, hz, eps_mode)

    def set_adjoint_form(self, form: int) -> None:
        """Reverse RK4 stages of adjoint_step: -1 chosen per grid, 0 one per launch, 1 two."""
        phasefield_set_adjoint_form(self.handle, form)

    def reduce(self, phi, stream=None):
        """(mass, min, max, #non-finite); synchronises the stream."""
        return phasefield_reduce(self.handle, self.params, phi, stream)

    def autotune(self, reps=5, stream=None):
        """Time every stage-kernel variant; returns (best, {name: ms per step})."""
        best, times = phasefield_autotune(self.handle, reps, stream, self.params.dtype)
        return best, {phasefield_variant_name(self.params.dtype, k): t for k, t in enumerate(times)}

    @property
    def variant_name(self) -> str:
        return phasefield_variant_name(self.params.dtype, self.variant)

    def report(self, max_face_speed: float) -> Report:
        return phasefield_check_params(self.params, max_face_speed)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            phasefield_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """Many independent simulations (uneven grids, one storage dtype, one scheme, steady
    velocity) advanced together: one launch per sweep over a global tile list, graph-replayed
    steps (RK4 in fused or per-stage sweeps, RK3, RK2 and Euler in per-stage sweeps)."""

    def __init__(self, params_list):
        self.params = list(params_list)
        self.handle = phasefield_batch_create(self.params)

    def step(self, phis, us, vs, ws, nsteps=1, t0s=None, stream=None):
        phasefield_batch_step(self.handle, self.params, phis, us, vs, ws, t0s, nsteps, stream)

    def set_persistent(self, persistent: bool = True):
        """Launch form of the sweeps: a persistent resident grid, or one workgroup per tile."""
        phasefield_batch_set_persistent(self.handle, persistent)

    SHAPES = ("fused_32x16", "fused_64x8", "stage_32x8")

    def set_shape(self, shape):
        """Tile shape of the sweeps: index into SHAPES or its name."""
        phasefield_batch_set_shape(self.handle, self.SHAPES.index(shape) if isinstance(shape, str) else shape)

    def autotune(self, reps=2, stream=None):
        """Time every shape and launch form on private fields, keep the fastest; returns
        (shape name, persistent, {(shape name, persistent): ms per step})."""
        if stream is None:  # graphs are captured: not on the NULL stream
            stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        bs, bp, times = phasefield_batch_autotune(self.handle, reps, stream)
        table = {(self.SHAPES[k // 2], bool(k % 2)): t for k, t in enumerate(times) if t >= 0}
        return self.SHAPES[bs], bool(bp), table

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            phasefield_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def velocity_from_coeffs(params: Params, phases, coeffs, stream=None):
    """Face velocity (u, v, w) of the separable-mode potential (phases (3, M), coeffs
    (M, M, M, 3), float64 GPU tensors), in the storage dtype of params."""
    M = int(phases.shape[1])
    shape = (int(params.n[2]), int(params.n[1]), int(params.n[0]))
    dt = TORCH_DTYPE[params.dtype]
    u, v, w = (torch.empty(shape, dtype=dt, device=phases.device) for _ in range(3))
    phasefield_velocity_from_coeffs(params, M, phases.contiguous(), coeffs.contiguous(), u, v, w,
                                    stream)
    return u, v, w


def velocity_coeffs_grad(params: Params, phases, gu, gv, gw, stream=None):
    """Gradient with respect to the mode coefficients of <(u, v, w), (gu, gv, gw)>."""
    M = int(phases.shape[1])
    cg = torch.zeros((M, M, M, 3), dtype=torch.float64, device=phases.device)
    phasefield_velocity_coeffs_grad(params, M, phases.contiguous(), gu, gv, gw, cg, stream)
    return cg


class Rollout(torch.autograd.Function):
    """phi_T = (nsteps steps of the solver)(phi_0) in the velocity synthesised from coeffs.

    Backward: discrete adjoint with checkpoints every ``ckpt`` steps. Each segment is re-run
    from its checkpoint (states held on the GPU), then swept backwards step by step; the
    accumulated face-velocity gradient is projected onto the mode coefficients once. With
    ``cache_stages`` the re-run keeps every step's stage inputs as well (phasefield_step_stages;
    (2 + stage_count) fields per step, for two segments at a time: each earlier segment is re-run
    on a side stream while the later one is swept) and the sweep takes them
    (phasefield_adjoint_step_stages) instead of recomputing them; without it, each adjoint step
    recomputes its stage inputs (phasefield_adjoint_step; one field per step of one segment).
    ``cache_stages=None`` (the default) caches when that memory is below half of what the device
    has available. With ``keep_all`` the forward itself keeps every step's state and stage inputs
    ((1 + stage_count) fields per step for the whole rollout, one allocation; ckpt and
    cache_stages are then unused) and the backward is the reverse sweep alone. All forms give
    the same gradients bit for bit. Returns gradients for phi_0 and coeffs.

    Usage: Rollout.apply(phi0, coeffs, solver, phases, nsteps, ckpt, t0, cache_stages, keep_all)
    """

    @staticmethod
    def forward(ctx, phi0, coeffs, solver: Solver, phases, nsteps: int, ckpt: int = 20,
                t0: float = 0.0, cache_stages: bool | None = None, keep_all: bool = False):
        p = solver.params
        u, v, w = velocity_from_coeffs(p, phases, coeffs.detach().to(torch.float64))
        phi = phi0.detach().clone().contiguous()
        ctx.solver, ctx.phases, ctx.nsteps, ctx.ckpt, ctx.t0 = solver, phases, nsteps, ckpt, t0
        ctx.vel = (u, v, w)
        ctx.keep_all = bool(keep_all)
        if ctx.keep_all:
            # every state and stage input of the rollout, in one allocation: field k of step n at
            # row n (1 + stage_count) + k (0: the state), rows padded to 256 bytes
            ns = solver.stage_count
            esz, numel = phi.element_size(), phi.numel()
            row = -(-numel * esz // 256) * 256 // esz
            pool = torch.empty(((nsteps + 1) * (1 + ns), row), dtype=phi.dtype, device=phi.device)

            def field(n, k):
                return pool[n * (1 + ns) + k, :numel].view(phi.shape)

            field(0, 0).copy_(phi)
            for n in range(nsteps):
                solver.step_stages(field(n, 0), u, v, w, t0 + n * solver.dt,
                                   *[field(n, 1 + k) for k in range(ns)], phi_next=field(n + 1, 0))
            ctx.pool, ctx.field = pool, field
            return field(nsteps, 0).clone()
        single = p.vel_mode != PF_VEL_STEADY  # time-varying: one call per step, t = t0 + n dt
        ckpts = []
        n = 0
        while n < nsteps:
            ckpts.append(phi.clone())
            m = min(ckpt, nsteps - n)
            _advance(solver, phi, u, v, w, t0, n, m, single)
            n += m
        if cache_stages is None:
            m = min(ckpt, nsteps)
            need = 2 * m * (2 + solver.stage_count) * phi.numel() * phi.element_size()
            free, _ = torch.cuda.mem_get_info(phi.device)
            free += torch.cuda.memory_reserved(phi.device) - torch.cuda.memory_allocated(phi.device)
            cache_stages = need < free // 2
        ctx.cache_stages = bool(cache_stages)
        ctx.ckpts = ckpts
        return phi

    @staticmethod
    def backward(ctx, grad_out):
        solver, nsteps, ckpt, t0 = ctx.solver, ctx.nsteps, ctx.ckpt, ctx.t0
        p = solver.params
        u, v, w = ctx.vel
        dt = solver.dt
        single = p.vel_mode != PF_VEL_STEADY
        lam = grad_out.detach().to(solver.dtype).contiguous().clone()
        gu, gv, gw = (torch.zeros_like(u) for _ in range(3))
        ns = solver.stage_count
        if ctx.keep_all:
            f = ctx.field
            for n in reversed(range(nsteps)):
                solver.adjoint_step_stages(f(n, 0), [f(n, 1 + k) for k in range(ns)], u, v, w,
                                           t0 + n * dt, lam, gu, gv, gw)
            cg = velocity_coeffs_grad(p, ctx.phases, gu, gv, gw)
            ctx.pool = ctx.field = None
            return lam, cg, None, None, None, None, None, None, None
        nseg = len(ctx.ckpts)
        if ctx.cache_stages:
            main = torch.cuda.current_stream()
            side = torch.cuda.Stream()

            def rerun(si, st):
                """Segment si re-run on stream st, keeping phi and the stage inputs of every
                step (out of place: the checkpoint stays intact)."""
                n0, m = si * ckpt, min(ckpt, nsteps - si * ckpt)
                states, stages = [], []
                with torch.cuda.stream(st):
                    cur = ctx.ckpts[si]
                    for j in range(m):
                        states.append(cur)
                        ys = [torch.empty_like(cur) for _ in range(ns)]
                        nxt = torch.empty_like(cur)
                        solver.step_stages(cur, u, v, w, t0 + (n0 + j) * dt, *ys, phi_next=nxt,
                                           stream=st)
                        stages.append(ys)
                        cur = nxt
                    done = torch.cuda.Event()
                    done.record(st)
                if st is not main:  # consumed on the main stream
                    for t in states[1:] + [y for ys in stages for y in ys]:
                        t.record_stream(main)
                return states, stages, done

            # the last segment's re-run on the main stream; each earlier one on the side stream,
            # after the previous re-run (both use the handle's accumulator) and beside the
            # reverse sweep of the segment after it (which uses the adjoint buffers only)
            pending = rerun(nseg - 1, main)
            for si in reversed(range(nseg)):
                states, stages, done = pending
                if si > 0:
                    side.wait_event(done)
                    pending = rerun(si - 1, side)
                main.wait_event(done)
                n0 = si * ckpt
                for j in reversed(range(len(states))):
                    solver.adjoint_step_stages(states[j], stages[j], u, v, w, t0 + (n0 + j) * dt,
                                               lam, gu, gv, gw, stream=main)
                del states, stages
        else:
            for s in reversed(range(nseg)):
                n0 = s * ckpt
                m = min(ckpt, nsteps - n0)
                states = [ctx.ckpts[s]]
                phi = ctx.ckpts[s].clone()
                for j in range(m - 1):
                    _advance(solver, phi, u, v, w, t0, n0 + j, 1, single)
                    states.append(phi.clone())
                for j in reversed(range(m)):
                    solver.adjoint_step(states[j], u, v, w, t0 + (n0 + j) * dt, lam, gu, gv, gw)
        cg = velocity_coeffs_grad(p, ctx.phases, gu, gv, gw)
        ctx.ckpts = None
        return lam, cg, None, None, None, None, None, None, None


def _advance(solver, phi, u, v, w, t0, n0, m, single):
    """m steps from step index n0 (time t0 + n0 dt)."""
    dt = solver.dt
    if single:
        for j in range(m):
            solver.step(phi, u, v, w, t0 + (n0 + j) * dt, 1)
    else:
        solver.step(phi, u, v, w, t0 + n0 * dt, m)

