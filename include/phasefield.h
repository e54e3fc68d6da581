/*
 * phasefield.h — C ABI of the MI355X (gfx950) library for the conservative, bounded
 * phase-field method of Mirjalili, Ivey & Mani (arXiv:1803.01262).
 *
 * What is computed (Sec. 1, Eq. 1):
 *   d(phi)/dt + div(u phi) = div[ gamma ( eps grad(phi) - phi (1-phi) grad(phi)/|grad(phi)| ) ]
 * discretised as in Sec. 2.2 (the five-step recipe): phi at cell centres, velocity on cell
 * faces (a staggered MAC grid), unit normal and the sharpening product phi(1-phi)n at cell
 * centres averaged onto faces, diffusive and advective face fluxes from second-order central
 * differences, and the cell update as the divergence of the face fluxes. Time integration is
 * forward Euler (Sec. 2.3, Eq. 25), the explicit midpoint rule (RK2, Eq. 26), the low-storage
 * third-order Runge-Kutta the paper names (RK3, Eq. 27) or classic fourth-order Runge-Kutta
 * (Eq. 28; the scheme of every experiment in Sec. 3).
 *
 * Data layout (every array): C-contiguous [nz][ny][nx], x fastest, periodic in every axis.
 *   phi[k][j][i]  cell-centre phase field.
 *   u[k][j][i]    x-velocity on the low x-face of cell (i,j,k)  (at x = i dx);
 *   v, w          likewise on the low y- and z-faces.
 * A two-dimensional problem is n[2] = 1 (with w = 0); one-dimensional is n[1] = n[2] = 1.
 * The element type of phi, u, v, w, lam and the gradients is the handle's storage dtype
 * (float for PF_F32, double for PF_F64). Arithmetic runs in the storage precision; mass sums
 * are always accumulated in double.
 *
 * Pointers: unless stated otherwise every array argument is a DEVICE pointer on the current
 * HIP device, at least 16-byte aligned, not aliasing any other argument, owned by the caller.
 * The library never frees or retains caller memory beyond a call. Scratch (stage buffers,
 * reduction partials, captured graphs) belongs to the handle and is released by destroy.
 *
 * Streams: hip_stream is a hipStream_t (NULL = the legacy default stream). Work is enqueued
 * asynchronously on it unless a function says it synchronises. A handle serves one stream at a
 * time; calls on one handle from several host threads must be serialised by the caller. One
 * exception: phasefield_step_stages (which uses the handle's accumulator buffer alone) and
 * phasefield_adjoint_step_stages (its adjoint buffers alone) may run at the same time on two
 * streams, e.g. a checkpointed backward re-running one segment while it sweeps the next one
 * backwards; each of the two still serves one stream at a time.
 *
 * Errors: every function returns pf_status; none aborts. On failure nothing has been enqueued
 * (argument errors) or the HIP error is reported as PF_ERR_DEVICE; phasefield_last_error()
 * then describes it. Leaving the paper's bounded regime (Eq. 17) or exceeding the scheme's
 * step limit (Eqs. 25, 28) is NOT an error — the paper runs such cases on purpose (Sec. 2.2.1,
 * Table 2); phasefield_check_params reports the margins.
 */
#ifndef PHASEFIELD_H
#define PHASEFIELD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PF_OK = 0,
    PF_ERR_INVALID = 1,     /* bad argument: size, spacing, parameter, null/misaligned pointer */
    PF_ERR_UNSUPPORTED = 2, /* valid request the library does not provide (e.g. the adjoint  */
                            /* on a non-uniform mesh)                                         */
    PF_ERR_DEVICE = 3,      /* a HIP call failed                                              */
    PF_ERR_OOM = 4,         /* device allocation failed                                       */
    PF_ERR_NONFINITE = 5    /* phasefield_reduce found NaN or Inf                             */
} pf_status;

typedef enum { PF_F32 = 0, PF_F64 = 1 } pf_dtype;             /* storage precision      */
typedef enum { PF_BC_PERIODIC = 0, PF_BC_WALL = 1 } pf_bc;      /* per axis               */
typedef enum { PF_EULER = 1, PF_RK2 = 2, PF_RK3 = 3, PF_RK4 = 4 } pf_scheme;
typedef enum { PF_VEL_STEADY = 0, PF_VEL_COS_REVERSAL = 1 } pf_velmode;

/* Problem statement of one simulation (Sec. 2.2: uniform isotropic mesh dx; eps and gamma
 * the interface thickness and sharpening speed of Eq. 1; dt the explicit step). */
typedef struct {
    int32_t n[3];       /* cells along x, y, z; each >= 1                                     */
    double dx;          /* mesh spacing (> 0)                                                  */
    double eps;         /* interface thickness parameter epsilon (>= 0)                        */
    double gamma;       /* sharpening velocity scale gamma (>= 0)                              */
    double dt;          /* time step (> 0)                                                     */
    double delta;       /* |grad phi| regulariser: n = g / sqrt(|g|^2 + delta^2); 0 gives the  */
                        /* plain unit normal with n = 0 where g = 0                            */
    int32_t bc[3];      /* pf_bc per axis. PF_BC_WALL: solid walls at x_a = 0 and n dx, with   */
                        /* zero total flux through the wall faces and mirror ghosts for the   */
                        /* central gradient; the face velocity stored at index 0 of a walled  */
                        /* axis (the wall face) is ignored. Walls on any axes run on every    */
                        /* kernel (the fused sweeps included). The adjoint and the batched    */
                        /* driver take walls too.                                             */
    int32_t dtype;      /* pf_dtype                                                            */
    int32_t scheme;     /* pf_scheme                                                           */
    int32_t vel_mode;   /* pf_velmode: velocity u0(x) * s(t), s = 1 or cos(pi t / vel_T)       */
    double vel_T;       /* reversal period for PF_VEL_COS_REVERSAL (> 0)                       */
    int32_t variant;    /* stage-kernel variant: -1 = automatic (tuned), else an index below   */
                        /* phasefield_variant_count(); every variant gives identical results   */
    int32_t use_graph;  /* 1: replay steps from a captured HIP graph where possible; 0: launch  */
} pf_params;

/* Fill p with defaults: periodic, FP64, RK4, steady velocity, variant -1, graphs on,
 * delta 0. The caller then sets n, dx, eps, gamma and dt. */
void phasefield_default_params(pf_params *p);

/* Criteria of the paper for a parameter set (no device work). max_face_speed is the largest
 * |component| over the face arrays (times max|s(t)|).
 *   crossover_margin_eq17: eps/dx - (gamma/U + 1)/(2 gamma/U), U = max_face_speed (Eq. 17);
 *                          >= 0 is the bounded regime proven in Sec. 2.2.
 *   crossover_margin_eq24: the same with the relaxed line of Eqs. 23-24 (identical here,
 *                          because the face speed is already the largest component).
 *   dt_max_scheme:         Eq. 25 (Euler), 26 (RK2), 27 (RK3) or 28 (RK4) with D_f = axes
 *                          longer than 1 cell.
 *   dt_over_dtmax:         dt / dt_max_scheme. */
typedef struct {
    double crossover_margin_eq17;
    double crossover_margin_eq24;
    double dt_max_scheme;
    double dt_over_dtmax;
} pf_report;
pf_status phasefield_check_params(const pf_params *p, double max_face_speed, pf_report *out);

typedef struct pf_solver pf_solver;

/* Validate p and allocate the handle with its device scratch (three field-sized stage
 * buffers). Errors: PF_ERR_INVALID (n < 1, dx <= 0, eps < 0, gamma < 0, dt <= 0, delta < 0,
 * bad enum, vel_T <= 0 in cos mode, variant out of range, n[1] or n[2] > 65535, an xy plane of
 * 2^28 cells or more), PF_ERR_OOM, PF_ERR_DEVICE. *out is NULL on failure. */
pf_status phasefield_create(const pf_params *p, pf_solver **out);

/* Release the handle and all its device memory (NULL is accepted). Synchronises the device
 * work the handle enqueued. */
pf_status phasefield_destroy(pf_solver *s);

/* Advance phi IN PLACE by nsteps steps of the handle's scheme (Sec. 2.3), starting at time
 * t0; step m runs from t0 + m dt. u, v, w: face velocity u0 (the time factor s(t) is applied
 * by the library at the stage times: RK4 t, t+dt/2, t+dt/2, t+dt; RK3 t, t+8dt/15, t+2dt/3;
 * RK2 t, t+dt/2; Euler t). RK3 runs on the per-stage kernels (a fused variant falls back).
 * nsteps = 0 is a no-op.
 * The handle's stage buffers are overwritten (and, with a fused variant, one of them holds phi
 * between steps); phi holds the result when the enqueued work completes.
 * Errors: PF_ERR_INVALID (null/misaligned pointer, nsteps < 0), PF_ERR_DEVICE. */
pf_status phasefield_step(pf_solver *s, void *phi, const void *u, const void *v, const void *w,
                          double t0, int32_t nsteps, void *hip_stream);

/* phasefield_step for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same steps, kernels and
 * results as phasefield_step on a handle created from *p, but with no handle and no allocating
 * call. The three stage buffers live in one fixed device array of the library
 * (phasefield_noalloc_scratch_bytes() bytes, 64 MiB, held by each GPU the library runs on until
 * the process ends), so 3 * round_up_256(cells * element size) must fit in it: up to about
 * 5.59M cells in FP32 (e.g. 176^3) and 2.79M in FP64 (e.g. 140^3); larger grids are rejected
 * with PF_ERR_INVALID before any device work. Steps are launched one by one (no captured graph,
 * p->use_graph is ignored). Every call on a GPU shares that GPU's array, and the array keeps
 * the last call's contents (the stage buffers need no clearing: every value is written before it
 * is read): calls that overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller. The first call on a device looks up that device's address of the
 * array (hipGetSymbolAddress). Errors: as phasefield_create's parameter checks and
 * phasefield_step's, PF_ERR_INVALID for a grid beyond the array, PF_ERR_DEVICE. */
pf_status phasefield_step_noalloc(const pf_params *p, void *phi, const void *u, const void *v,
                                  const void *w, double t0, int32_t nsteps, void *hip_stream);

/* Size in bytes of the fixed device array behind phasefield_step_noalloc. */
size_t phasefield_noalloc_scratch_bytes(void);

/* Discrete adjoint of ONE step (the transpose of the derivative of phasefield_step with
 * nsteps = 1, taken at phi_n and time t_n). On entry lam = dL/dphi_{n+1}; on exit
 * lam = dL/dphi_n (in place). gu, gv, gw (may each be NULL to skip) ACCUMULATE
 * dL/du0 etc. (+=); on a walled axis the wall face's entry (index 0) gets nothing, since the
 * step ignores the velocity stored there. The stage inputs of the forward step are recomputed
 * from phi_n. Allocates three more field-sized scratch buffers on first use. On a non-uniform
 * mesh (phasefield_set_spacing) it is the transpose of that mesh's step (one reverse stage per
 * launch). Errors: PF_ERR_INVALID (null phi_n/u/v/w/lam, misaligned),
 * PF_ERR_OOM, PF_ERR_DEVICE. */
pf_status phasefield_adjoint_step(pf_solver *s, const void *phi_n, const void *u, const void *v,
                                  const void *w, double t_n, void *lam, void *gu, void *gv,
                                  void *gw, void *hip_stream);

/* One step of the handle's scheme from time t (as phasefield_step with nsteps = 1) that also
 * stores the stage inputs its discrete adjoint reads (the Runge-Kutta stage values of Sec. 2.3:
 * RK4 y2 = phi + dt/2 k1, y3 = phi + dt/2 k2, y4 = phi + dt k3; RK3 the first two of its
 * low-storage stages, y2 and y3; RK2 the midpoint value y2; Euler none). The new phi goes to
 * phi_next (DEVICE, the field's size and type); phi_next NULL or equal to phi steps in place,
 * otherwise phi is left unchanged. y2, y3, y4: DEVICE arrays of the field's size and storage
 * type, owned by the caller, written completely; those the scheme does not use may be NULL and
 * are not touched; they must not coincide with phi, phi_next or each other. The new phi and the
 * stage values are bit-identical to phasefield_step's and to what phasefield_adjoint_step
 * recomputes. For checkpointed adjoints that keep the stage values of a re-run segment instead
 * of recomputing them (phasefield_adjoint_step_stages). Stream-ordered on hip_stream, no
 * synchronisation, no graph. Errors: PF_ERR_INVALID (null or misaligned phi, u, v, w or a stage
 * buffer the scheme needs, misaligned phi_next, coinciding buffers, non-finite t),
 * PF_ERR_DEVICE. */
pf_status phasefield_step_stages(pf_solver *s, void *phi, void *phi_next, const void *u,
                                 const void *v, const void *w, double t, void *y2, void *y3,
                                 void *y4, void *hip_stream);

/* phasefield_adjoint_step with the stage inputs supplied: y2, y3, y4 (DEVICE, read only; those
 * the scheme does not use may be NULL) as phasefield_step_stages stored them for the same phi_n,
 * velocity and t_n. Nothing is recomputed: the reverse stages alone run, and lam and the
 * gradients are bit-identical to phasefield_adjoint_step's. Stage values from another phi_n or
 * t_n give the adjoint of a different linearisation (not detected). Errors: as
 * phasefield_adjoint_step, PF_ERR_INVALID also for a null or misaligned stage buffer the scheme
 * needs. */
pf_status phasefield_adjoint_step_stages(pf_solver *s, const void *phi_n, const void *y2,
                                         const void *y3, const void *y4, const void *u,
                                         const void *v, const void *w, double t_n, void *lam,
                                         void *gu, void *gv, void *gw, void *hip_stream);

/* Non-uniform rectilinear mesh for a handle. The paper (Sec. 3.3.3, the list that closes the
 * comparison with Chiu and Lin) notes that the method extends to non-uniform anisotropic
 * Cartesian grids, with eps chosen for the worst case or tuned to the local mesh, and gives no
 * discrete form; this library reads it as follows. hx, hy, hz are HOST arrays of n[0], n[1],
 * n[2] cell widths (copied; each positive and finite; they need not sum to n dx). The width
 * index wraps on a periodic axis and mirrors across walls. With d(i) = (h(i-1) + h(i))/2 the
 * distance between the centres across the low face of cell i: the central gradient divides by
 * d(i) + d(i+1), the diffusive flux by d of its face, the divergence by h(i); the face values of
 * phi and of the sharpening product stay the means of the two cells. eps_mode 0: p->eps
 * everywhere (the worst-case choice: eps on the crossover line of Eq. 17 for the largest width);
 * 1: per cell p->eps * max(hx_i, hy_j, hz_k) / p->dx (p->dx the reference spacing p->eps belongs
 * to; the maximum over the axes longer than one cell), averaged onto each face. From then on
 * phasefield_step runs every scheme through the per-stage kernel in its non-uniform form (no
 * fused sweeps), phasefield_reduce returns
 * sum(phi * cell volume) (axes of one cell carry no volume), phasefield_adjoint_step (and the
 * stage-keeping pair) take the transpose of this mesh's step, and phasefield_autotune returns
 * PF_ERR_UNSUPPORTED. The velocity on the faces must be discretely
 * divergence-free on this mesh, sum_a (u_a[+] - u_a[-]) / h_a = 0. All three NULL returns the
 * handle to the uniform mesh of p->dx. Synchronises the device (queued work may still read the
 * previous tables). Errors: PF_ERR_INVALID (NULL handle, some but not all widths NULL, a width
 * that is not positive and finite, eps_mode not 0 or 1), PF_ERR_OOM, PF_ERR_DEVICE. */
pf_status phasefield_set_spacing(pf_solver *s, const double *hx, const double *hy,
                                 const double *hz, int32_t eps_mode);

/* How phasefield_adjoint_step runs the four reverse stages of RK4 (other schemes always take
 * one per launch): 0 one stage per launch; 1 two per launch (a kernel that keeps the later
 * stage's adjoint and flux-Jacobian terms in LDS and hands them to the earlier stage of the same
 * tile: fewer field passes, but more registers per thread); -1 (the default) two per launch for
 * FP64 on grids of 192^3 cells and more when the handle's variant is a fused one, else one.
 * Every form gives bit-identical results. Fields of 4 GiB or more, handles with walls and
 * handles with a non-uniform mesh always take one per launch.
 * Errors: PF_ERR_INVALID (NULL handle, form outside -1..1). */
pf_status phasefield_set_adjoint_form(pf_solver *s, int32_t form);

/* Mass and bounds of a field: out4 = {sum(phi) * dx^D, min(phi), max(phi), #non-finite},
 * D = number of axes longer than one cell; the sum is accumulated in double in a fixed order
 * (deterministic). Non-finite cells are left out of sum, min and max. SYNCHRONISES
 * hip_stream. out4 is a HOST pointer. Returns PF_ERR_NONFINITE (with out4 filled) if any cell
 * is NaN or Inf. */
pf_status phasefield_reduce(pf_solver *s, const void *phi, double out4[4], void *hip_stream);

/* Face velocity as the discrete curl of an edge vector potential built from separable
 * Fourier modes (the face field is then discretely divergence-free, as Eq. 19 requires):
 *   A_a(x) = sum_{m1,m2,m3=1..M} coeffs[m3-1][m2-1][m1-1][a]
 *            sin(2 pi m1 x/Lx + phases[0][m1-1]) sin(2 pi m2 y/Ly + phases[1][m2-1])
 *            sin(2 pi m3 z/Lz + phases[2][m3-1]),   L = n dx,
 * with A_x on x-edges ((i+1/2) dx, j dx, k dx), A_y on y-edges (i dx, (j+1/2) dx, k dx) and
 * A_z on z-edges (i dx, j dx, (k+1/2) dx); u = (A_z[j+1]-A_z[j] - A_y[k+1]+A_y[k]) / dx and
 * cyclically. p supplies n, dx and dtype. phases (double[3][M]) and coeffs (double[M][M][M][3])
 * are device pointers; u, v, w are written in the storage dtype (computed in double).
 * Errors: PF_ERR_INVALID (M < 1 or M > 64, null pointer), PF_ERR_OOM, PF_ERR_DEVICE. */
pf_status phasefield_velocity_from_coeffs(const pf_params *p, int32_t modes, const double *phases,
                                          const double *coeffs, void *u, void *v, void *w,
                                          void *hip_stream);

/* Transpose of phasefield_velocity_from_coeffs: coeff_grad (double[M][M][M][3], device)
 * ACCUMULATES d<(u,v,w),(gu,gv,gw)>/d coeffs (+=). gu, gv, gw in the storage dtype. Projects
 * a face-velocity gradient (from phasefield_adjoint_step) onto the mode coefficients. */
pf_status phasefield_velocity_coeffs_grad(const pf_params *p, int32_t modes,
                                          const double *phases, const void *gu, const void *gv,
                                          const void *gw, double *coeff_grad, void *hip_stream);

/* Number of compiled stage-kernel variants for a storage dtype. A name gives the kind
 * ("tiled": one launch per RK stage; "fused": two stages per launch; "global": one thread per
 * cell), the column tile (x by y) and, when it ends in a third number, the planes per z-chunk;
 * without one, each launch chooses the chunk length for the grid and the device's resident
 * workgroups. "_big" forces the addressing form of arrays of 4 GiB or more. */
int32_t phasefield_variant_count(int32_t dtype);

/* Short name of a variant (static string), or NULL if out of range. */
const char *phasefield_variant_name(int32_t dtype, int32_t variant);

/* Time every variant on the handle's grid (using the handle's scratch and temporary buffers
 * only; caller data is untouched), store the fastest as the handle's variant and return it in
 * *best; times_ms (HOST, may be NULL) receives phasefield_variant_count(dtype) per-step times.
 * Synchronises. The choice for a periodic grid is cached per (dtype, grid shape) for the life
 * of the process and used by later phasefield_create calls with variant -1; if the environment
 * variable PF_TUNE_CACHE names a file, the cache is also read from and written to it (one line
 * per entry: dtype nx ny nz variant-name). Without a cached choice, create picks a default from
 * the grid size and dtype (fused sweeps from about 104^3 cells in FP32 and 128^3 in FP64,
 * per-stage kernels below and on every grid of one plane; both with per-launch chunk
 * lengths); a grid with walls takes the per-stage kernel in FP64 and, in FP32, the fused 32x16
 * sweeps from about 144^3 cells (per-stage below). */
pf_status phasefield_autotune(pf_solver *s, int32_t reps, int32_t *best, double *times_ms,
                              void *hip_stream);

/* The variant a handle runs. */
int32_t phasefield_solver_variant(const pf_solver *s);

/* ----------------------------------------------------------------------------------------
 * Batched driver: many independent simulations (each its own pf_params, uneven grid sizes,
 * same dtype, same scheme, steady velocity) advanced together. Each sweep is ONE launch over a
 * global tile list that covers every instance (one workgroup per tile): for RK4 two fused
 * two-stage sweeps per step, or four single-stage sweeps; for RK3, RK2 and Euler one
 * single-stage sweep per stage (Euler then one batched copy of the accumulator into phi).
 * per_instance[0].variant selects the RK4 mode by its kind (a "fused_*" variant or a per-stage
 * one); with variant -1, FP32 runs fused and FP64 per-stage. Instances may have walls on any
 * axes (each its own), in either mode; a scheme other than RK4 puts the batch in per-stage mode
 * (the fused sweeps pair RK4's stages).
 * The step sequence
 * is replayed from a captured HIP graph. Results are bit-identical to running each instance
 * alone with phasefield_step.
 * ------------------------------------------------------------------------------------- */
typedef struct pf_batch pf_batch;

/* per_instance: HOST array of count parameter sets (all with the same dtype).
 * Errors: PF_ERR_INVALID (count < 1, any invalid set, mixed dtypes), PF_ERR_UNSUPPORTED (mixed
 * schemes, a time-varying velocity, or a field of 4 GiB or more: such grids take a single-grid
 * solver), PF_ERR_OOM, PF_ERR_DEVICE. */
pf_status phasefield_batch_create(const pf_params *per_instance, int32_t count, pf_batch **out);

/* Advance every instance b by nsteps steps: phi[b], u[b], v[b], w[b] are HOST arrays of count
 * device pointers; t0 is a HOST array of count start times (NULL = all zero). The pointer set
 * may change between calls (a changed set is re-captured). */
pf_status phasefield_batch_step(pf_batch *b, void *const *phi, const void *const *u,
                                const void *const *v, const void *const *w, const double *t0,
                                int32_t nsteps, void *hip_stream);

/* Launch form of the batched sweeps: 0 (the default) launches one workgroup per tile-list entry
 * and lets the hardware dispatcher hand out the entries; 1 launches a persistent grid (the
 * sweep kernel's resident workgroups, a multiple of 8) whose workgroups each walk their XCD's
 * share of the list. Results are identical either way. Synchronises work queued on the batch's
 * last stream when the form changes; the next step re-captures its graph. Errors: PF_ERR_INVALID
 * (NULL), PF_ERR_DEVICE. */
pf_status phasefield_batch_set_persistent(pf_batch *b, int32_t persistent);

/* Tile shape of the batched sweeps: 0 fused two-stage sweeps on 32x16 tiles (the fused mode's
 * default), 1 fused sweeps on 64x8 tiles (fewer halo columns; instances whose rows are not a
 * multiple of 64 pad their last tile column), 2 one launch per RK stage on 32x8 tiles (the
 * per-stage mode). Every shape gives bit-identical results. The tile list is rebuilt; the next
 * step re-uploads the per-instance tables and re-captures its graph (work queued on the batch's
 * last stream is synchronised first). Errors: PF_ERR_INVALID (NULL, shape outside 0..2),
 * PF_ERR_UNSUPPORTED (a fused shape for a scheme other than RK4), PF_ERR_OOM,
 * PF_ERR_DEVICE. */
pf_status phasefield_batch_set_shape(pf_batch *b, int32_t shape);

/* Time every tile shape (phasefield_batch_set_shape) in both launch forms
 * (phasefield_batch_set_persistent) on private fields of the batch's instances (a uniform field
 * and velocity; caller data is untouched), reps x 8 graph-replayed steps each after one
 * untimed 8-step run, and leave the batch in the fastest combination, returned in *best_shape
 * and *best_persistent (HOST, may be NULL). times_ms (HOST, may be NULL) receives 6 per-step
 * times, index 2 * shape + persistent (-1 for a combination that does not apply). Allocates
 * 4 fields per instance for the duration of the call; synchronises hip_stream, which must not be
 * the NULL stream. Errors: PF_ERR_INVALID (NULL batch or stream, reps < 1), PF_ERR_OOM,
 * PF_ERR_DEVICE. */
pf_status phasefield_batch_autotune(pf_batch *b, int32_t reps, int32_t *best_shape,
                                    int32_t *best_persistent, double *times_ms, void *hip_stream);

pf_status phasefield_batch_destroy(pf_batch *b);

/* Copy `bytes` bytes (a multiple of 4) from src to dst, both device pointers, asynchronously
 * on hip_stream: the library's streaming copy (16-byte pieces, four in flight per thread, when
 * both pointers are 16-byte aligned), which also ends odd step counts of the alternating
 * schedules. It serves as the measured bandwidth reference of a plain read-plus-write stream.
 * The ranges must not overlap. Errors: PF_ERR_INVALID (null pointer, size), PF_ERR_DEVICE. */
pf_status phasefield_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Description of the last error on the calling thread (empty string if none); valid until
 * the next library call on that thread. */
const char *phasefield_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PHASEFIELD_H */
