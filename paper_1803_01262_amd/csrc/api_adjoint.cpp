// C ABI: discrete adjoint of one step, velocity synthesis from modes and its transpose.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>

#include "pf_api_internal.h"

using namespace pf;

template <typename T>
static AdjArgs<T> make_adj(const pf_params& p, double svel, const T* y, const T* kap_in,
                           double kap_scale, const T* lam_base, T* lam_out, const T* lamp,
                           T* kap_out, double kb, double ka, T* gU, T* gV, T* gW, const T* U,
                           const T* V, const T* W, const NuMesh* nu)
{
    AdjArgs<T> a;
    a.y = y;
    a.kap_in = kap_in;
    a.kap_scale = (T)kap_scale;
    a.lam_base = lam_base;
    a.lam_out = lam_out;
    a.lamp = lamp;
    a.kap_out = kap_out;
    a.kb = (T)kb;
    a.ka = (T)ka;
    a.gU = gU;
    a.gV = gV;
    a.gW = gW;
    a.U = U;
    a.V = V;
    a.W = W;
    a.nx = p.n[0];
    a.ny = p.n[1];
    a.nz = p.n[2];
    a.walls = wall_mask(p);
    a.inv_dx = (T)(1.0 / p.dx);
    a.inv_2dx = (T)(1.0 / (2.0 * p.dx));
    a.ge = (T)(p.gamma * p.eps / p.dx);
    a.hg = (T)(0.5 * p.gamma);
    a.hs = (T)(0.5 * svel);
    a.delta2 = (T)(p.delta * p.delta);
    if (nu) {  // the forward's coefficients of the mesh (make_stage)
        for (int ax = 0; ax < 3; ++ax) a.nu[ax] = (const T*)nu->tab[ax];
        a.nu_ge = (T)(nu->eps_mode == 1 ? p.gamma * p.eps / p.dx : p.gamma * p.eps);
        a.nu_hg = (T)(0.5 * p.gamma);
        a.nu_eps_mode = nu->eps_mode;
    }
    return a;
}

template <typename T>
static AdjPairArgs<T> make_pair(const pf_params& p, double svelH, double svelL, const T* yH,
                                const T* srcH, double kscaleH, const T* yL, const T* lamp,
                                const T* base, T* L_out, T* kout, T* lam_copy, double kaL,
                                double kbL, double kaO, double kbO, T* gU, T* gV, T* gW,
                                const T* U, const T* V, const T* W)
{
    AdjPairArgs<T> a;
    a.yH = yH;
    a.srcH = srcH;
    a.kscaleH = (T)kscaleH;
    a.yL = yL;
    a.lamp = lamp;
    a.base = base;
    a.L_out = L_out;
    a.kout = kout;
    a.lam_copy = lam_copy;
    a.kaL = (T)kaL;
    a.kbL = (T)kbL;
    a.kaO = (T)kaO;
    a.kbO = (T)kbO;
    a.gU = gU;
    a.gV = gV;
    a.gW = gW;
    a.U = U;
    a.V = V;
    a.W = W;
    a.nx = p.n[0];
    a.ny = p.n[1];
    a.nz = p.n[2];
    a.inv_dx = (T)(1.0 / p.dx);
    a.inv_2dx = (T)(1.0 / (2.0 * p.dx));
    a.ge = (T)(p.gamma * p.eps / p.dx);
    a.hg = (T)(0.5 * p.gamma);
    a.hsH = (T)(0.5 * svelH);
    a.hsL = (T)(0.5 * svelL);
    a.delta2 = (T)(p.delta * p.delta);
    return a;
}

// Reverse sweep of one classic RK4 step  phi' = phi + dt/6 (k1 + 2k2 + 2k3 + k4),
// y1 = phi, y2 = phi + dt/2 k1, y3 = phi + dt/2 k2, y4 = phi + dt k3, k_s = f(y_s, t_s):
//   kap4 = dt/6 lam'                       lam_n = lam' + sum_s ybar_s,
//   kap3 = dt/3 lam' + dt   ybar4          ybar_s = (df/dy at y_s)^T kap_s,
//   kap2 = dt/3 lam' + dt/2 ybar3          gU += sum_s (df/dU at y_s)^T kap_s.
//   kap1 = dt/6 lam' + dt/2 ybar2
// Buffers: y2, y3, y4 reuse the forward stage buffers; Ka/Kb ping-pong the stage cotangent
// (it is read with a stencil), L accumulates lam' + sum ybar. With stages (the caller's copies of
// the stage inputs, from phasefield_step_stages) nothing is recomputed: y2, y3, y4 are read from
// there (RK3: y2, y3; RK2: y2).
template <typename T>
static pf_status adjoint_impl(pf_solver* s, const T* phi, const T* U, const T* V, const T* W,
                              double t, T* lam, T* gU, T* gV, T* gW, hipStream_t st,
                              const T* const* stages = nullptr)
{
    const pf_params& p = s->p;
    for (int b = 0; b < 3; ++b)
        if (!s->adj[b]) {
            hipError_t e = hipMalloc(&s->adj[b], s->N * sizeof(T));
            if (e != hipSuccess) return hip_fail(e, "phasefield_adjoint_step: allocation");
        }
    T* Ka = (T*)s->adj[0];
    T* Kb = (T*)s->adj[1];
    T* L = (T*)s->adj[2];
    const double dt = p.dt;
    // The plain forward variant pairs with the plain adjoint kernel (both one thread per cell).
    // A per-stage tiled variant lends its tile shape, chunk length (none: chosen per launch) and
    // large-array form to the tiled adjoint when that shape has an adjoint kernel; otherwise the
    // tile is chosen from the grid size and the chunk per launch.
    const char* vname = stage_variant(p.dtype, s->variant).name;
    const bool plain = std::strcmp(vname, "global") == 0;
    int tile = -1, tx = 0, ty = 0, kz = 0;
    const int got = std::sscanf(vname, "tiled_%dx%dx%d", &tx, &ty, &kz);
    if (got >= 2) tile = adjoint_tile_index(tx, ty);
    if (got < 3 || tile < 0) kz = 0;
    if (tile < 0) tile = adjoint_default_tile(p.n[0], p.n[1], p.n[2]);
    const size_t vlen = std::strlen(vname);
    const bool big = vlen > 4 && std::strcmp(vname + vlen - 4, "_big") == 0;
    // a non-uniform mesh: the forward's per-stage NU kernel for the recompute, the NU forms of the
    // plain and tiled adjoint kernels for the reverse stages
    const NuMesh* nu = s->nu.on() ? &s->nu : nullptr;
    auto adj = [&](const AdjArgs<T>& a, hipStream_t hs) {
        if (plain) return nu ? launch_adjoint_stage_nu<T>(a, hs) : launch_adjoint_stage_global<T>(a, hs);
        return launch_adjoint_stage<T>(a, tile, kz, big, hs);
    };
    hipError_t e;
    if (p.scheme == PF_EULER) {
        // phi' = phi + dt f(phi):  lam_n = lam' + (df/dphi)^T (dt lam')
        e = adj(make_adj<T>(p, time_factor(p, t), phi, lam, dt, lam, L, nullptr,
                                                nullptr, 0.0, 0.0, gU, gV, gW, U, V, W, nu), st);
        if (e == hipSuccess) e = launch_copy<T>(lam, L, s->N, st);
        return e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_adjoint_step");
    }
    if (p.scheme == PF_RK3) {
        // Butcher form of the low-storage RK3: a21 = 8/15, a31 = 1/4, a32 = 5/12, b = (1/4, 0, 3/4),
        // stage times t, t + 8/15 dt, t + 2/3 dt. Reverse:
        //   kap3 = dt 3/4 lam';  L = lam' + ybar3;  kap2 = dt a32 ybar3 (b2 = 0);
        //   kap1 = dt (b1 lam' + a21 ybar2 + a31 ybar3) = dt/4 L + dt 8/15 ybar2   (a31 = b1);
        //   L += ybar2;  lam_n = L + ybar1
        constexpr double g1 = 8.0 / 15.0, g2 = 5.0 / 12.0, z2 = -17.0 / 60.0;
        static_assert(g1 + z2 == 0.25, "a31 must equal b1 for the folded kap1");
        const T* y2 = (T*)s->ya;
        const T* y3 = (T*)s->yb;
        T* A = (T*)s->acc;  // u1 + dt z2 k1, the base of y3
        const double s1 = time_factor(p, t), s2 = time_factor(p, t + g1 * dt),
                     s3 = time_factor(p, t + (g1 + g2 + z2) * dt);
        if (stages) {
            y2 = stages[0];
            y3 = stages[1];
            e = hipSuccess;
        } else {
            e = run_stage<T>(s->variant, make_stage<T>(p, s1, phi, phi, phi, (T*)y2, A, dt * g1,
                                                       dt * (g1 + z2), U, V, W, nu), st);
            if (e == hipSuccess)
                e = run_stage<T>(s->variant, make_stage<T>(p, s2, y2, A, nullptr, (T*)y3, nullptr,
                                                           dt * g2, 0.0, U, V, W, nu), st);
        }
        if (e == hipSuccess)
            e = adj(make_adj<T>(p, s3, y3, lam, 0.75 * dt, lam, L, lam, Ka, 0.0, g2 * dt, gU, gV,
                                gW, U, V, W, nu), st);
        if (e == hipSuccess)
            e = adj(make_adj<T>(p, s2, y2, Ka, 1.0, L, L, L, Kb, 0.25 * dt, g1 * dt, gU, gV, gW, U,
                                V, W, nu), st);
        if (e == hipSuccess)
            e = adj(make_adj<T>(p, s1, phi, Kb, 1.0, L, lam, nullptr, nullptr, 0.0, 0.0, gU, gV,
                                gW, U, V, W, nu), st);
        return e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_adjoint_step");
    }
    if (p.scheme == PF_RK2) {
        // phi' = phi + dt k2,  k2 = f(y2, t + dt/2),  y2 = phi + dt/2 k1:
        //   kap2 = dt lam';  ybar2 = (df/dy at y2)^T kap2;  kap1 = dt/2 ybar2;
        //   lam_n = lam' + ybar2 + (df/dy at phi)^T kap1
        const T* y2 = stages ? stages[0] : (T*)s->ya;
        const double s1 = time_factor(p, t), s2 = time_factor(p, t + 0.5 * dt);
        e = stages ? hipSuccess
                   : run_stage<T>(s->variant, make_stage<T>(p, s1, phi, phi, nullptr, (T*)y2, nullptr,
                                                            0.5 * dt, 0.0, U, V, W, nu), st);
        if (e == hipSuccess)
            e = adj(make_adj<T>(p, s2, y2, lam, dt, lam, L, lam, Ka, 0.0, 0.5 * dt, gU, gV, gW, U,
                                V, W, nu), st);
        if (e == hipSuccess)
            e = adj(make_adj<T>(p, s1, phi, Ka, 1.0, L, lam, nullptr, nullptr, 0.0, 0.0, gU, gV,
                                gW, U, V, W, nu), st);
        return e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_adjoint_step");
    }
    T* y2 = (T*)s->ya;
    T* y3 = (T*)s->yb;
    T* y4 = (T*)s->acc;
    const double s1 = time_factor(p, t), s2 = time_factor(p, t + 0.5 * dt),
                 s4 = time_factor(p, t + dt);
    const int v = s->variant;
    // recompute the stage inputs exactly as the forward step stores them (every variant rounds
    // alike). A fused variant produces y2 and y3 in one sweep (sweep A with its y_mid output and
    // no accumulator output; FP64 adjoint step against three per-stage launches on 64x8 tiles:
    // 128^3 0.259 / 0.259 ms, 256^3 1.90 / 1.95, 512^3 14.98 / 15.38); on walled grids three
    // per-stage launches.
    const bool fused_rc = !nu && variant_is_fused(p.dtype, v) && wall_mask(p) == 0;
    const int vs = variant_is_fused(p.dtype, v) && !fused_rc ? stage_variant_index(p.dtype, "tiled_64x8") : v;
    if (stages) {
        y2 = (T*)stages[0];
        y3 = (T*)stages[1];
        y4 = (T*)stages[2];
        e = hipSuccess;
    } else if (fused_rc) {
        FusedArgs<T> a = make_fused<T>(p, false, t, phi, y4, U, V, W, y3);
        a.out_mid = y2;
        a.out_acc = nullptr;
        e = run_fused_sweep<T>(v, a, false, st);
    } else {
        e = run_stage<T>(vs, make_stage<T>(p, s1, phi, phi, nullptr, y2, nullptr, 0.5 * dt, 0.0, U, V, W, nu), st);
        if (e == hipSuccess)
            e = run_stage<T>(vs, make_stage<T>(p, s2, y2, phi, nullptr, y3, nullptr, 0.5 * dt, 0.0, U, V, W, nu), st);
    }
    if (e == hipSuccess && !stages)
        e = run_stage<T>(vs, make_stage<T>(p, s2, y3, phi, nullptr, y4, nullptr, dt, 0.0, U, V, W, nu), st);
    // reverse stages: one per launch, or two per launch (adjoint_fused.hip, the same
    // arithmetic as the single stages below, bit for bit): (4, 3) writes L = lam' + ybar4 +
    // ybar3, kap2 into Kb and a copy of lam' into Ka (so that (2, 1) can write lam in place while
    // it still reads lam' around its tile); (2, 1) writes lam = L + ybar2 + ybar1.
    // Chosen per grid: FP64 with a fused forward variant on grids of 192^3 cells and more
    // (measured 0.92-0.99 of the single-stage time from 192^3 to 512^3, 1.13 at 128^3); never in
    // FP32, where the pair kernel needs about 170 registers (two waves per SIMD) and measured
    // 1.08-1.44 times slower from 128^3 to 512^3.
    const size_t cells = (size_t)p.n[0] * p.n[1] * p.n[2];
    const bool pair_auto = variant_is_fused(p.dtype, v) && p.dtype == PF_F64 &&
                           cells >= (size_t)192 * 192 * 192;
    const bool pair = (s->adjoint_form == 1 || (s->adjoint_form < 0 && pair_auto)) &&
                      !field_needs_big(p.n[0], p.n[1], p.n[2], sizeof(T)) && wall_mask(p) == 0 &&
                      !nu;
    if (pair) {
        // a fused forward variant lends its tile shape (64x8 or 32x16) and fixed chunk length, if
        // it names one; otherwise 64x8 unless 64-wide tiles pad more columns, chunks per launch
        int ftx = 0, fty = 0, fkz = 0;
        const int fgot = std::sscanf(vname, "fused_%dx%dx%d", &ftx, &fty, &fkz);
        int pt = adjoint_default_tile(p.n[0], p.n[1], p.n[2]) == 0 ? 0 : 1;
        if (fgot >= 2 && ftx == 64 && fty == 8) pt = 0;
        if (fgot >= 2 && ftx == 32 && fty == 16) pt = 1;
        const int pkz = fgot >= 3 ? fkz : 0;
        if (e == hipSuccess)
            e = launch_adjoint_pair<T>(make_pair<T>(p, s4, s2, y4, lam, dt / 6.0, y3, lam, lam, L,
                                                    Kb, Ka, dt, dt / 3.0, 0.5 * dt, dt / 3.0, gU,
                                                    gV, gW, U, V, W), pt, pkz, st);
        if (e == hipSuccess)
            e = launch_adjoint_pair<T>(make_pair<T>(p, s2, s1, y2, Kb, 1.0, phi, Ka, L, lam,
                                                    nullptr, nullptr, 0.5 * dt, dt / 6.0, 0.0, 0.0,
                                                    gU, gV, gW, U, V, W), pt, pkz, st);
        return e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_adjoint_step");
    }
    if (e == hipSuccess)
        e = adj(make_adj<T>(p, s4, y4, lam, dt / 6.0, lam, L, lam, Ka, dt / 3.0,
                                                dt, gU, gV, gW, U, V, W, nu), st);
    if (e == hipSuccess)
        e = adj(make_adj<T>(p, s2, y3, Ka, 1.0, L, L, lam, Kb, dt / 3.0,
                                                0.5 * dt, gU, gV, gW, U, V, W, nu), st);
    if (e == hipSuccess)
        e = adj(make_adj<T>(p, s2, y2, Kb, 1.0, L, L, lam, Ka, dt / 6.0,
                                                0.5 * dt, gU, gV, gW, U, V, W, nu), st);
    if (e == hipSuccess)
        e = adj(make_adj<T>(p, s1, phi, Ka, 1.0, L, lam, nullptr, nullptr, 0.0,
                                                0.0, gU, gV, gW, U, V, W, nu), st);
    // the forward graph (if any) captured the stage buffers' old contents only; nothing to redo
    return e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_adjoint_step");
}

// Stage inputs an RK step keeps for its adjoint: RK4 y2, y3, y4; RK3 y2, y3; RK2 y2; Euler none.
int pf::scheme_stage_count(int scheme)
{
    return scheme == PF_RK4 ? 3 : scheme == PF_RK3 ? 2 : scheme == PF_RK2 ? 1 : 0;
}

static pf_status adjoint_checks(pf_solver* s, const void* phi_n, const void* u, const void* v,
                                const void* w, double t_n, const void* lam, const void* gu,
                                const void* gv, const void* gw)
{
    if (!s) return fail(PF_ERR_INVALID, "solver is NULL");
    pf_status st;
    if ((st = check_field_ptr(phi_n, "phi_n")) != PF_OK) return st;
    if ((st = check_field_ptr(u, "u")) != PF_OK) return st;
    if ((st = check_field_ptr(v, "v")) != PF_OK) return st;
    if ((st = check_field_ptr(w, "w")) != PF_OK) return st;
    if ((st = check_field_ptr(lam, "lam")) != PF_OK) return st;
    for (const void* g : {gu, gv, gw})
        if (g && (((uintptr_t)g) & 15)) return fail(PF_ERR_INVALID, "gradient not 16-byte aligned");
    if (!std::isfinite(t_n)) return fail(PF_ERR_INVALID, "t_n is not finite");
    return PF_OK;
}

static pf_status adjoint_dispatch(pf_solver* s, const void* phi_n, const void* u, const void* v,
                                  const void* w, double t_n, void* lam, void* gu, void* gv,
                                  void* gw, void* hip_stream, const void* const* stages)
{
    hipStream_t hs = (hipStream_t)hip_stream;
    if (s->p.dtype == PF_F32)
        return adjoint_impl<float>(s, (const float*)phi_n, (const float*)u, (const float*)v,
                                   (const float*)w, t_n, (float*)lam, (float*)gu, (float*)gv,
                                   (float*)gw, hs, (const float* const*)stages);
    return adjoint_impl<double>(s, (const double*)phi_n, (const double*)u, (const double*)v,
                                (const double*)w, t_n, (double*)lam, (double*)gu, (double*)gv,
                                (double*)gw, hs, (const double* const*)stages);
}

extern "C" pf_status phasefield_adjoint_step(pf_solver* s, const void* phi_n, const void* u,
                                             const void* v, const void* w, double t_n, void* lam,
                                             void* gu, void* gv, void* gw, void* hip_stream)
{
    pf_status st = adjoint_checks(s, phi_n, u, v, w, t_n, lam, gu, gv, gw);
    if (st != PF_OK) return st;
    return adjoint_dispatch(s, phi_n, u, v, w, t_n, lam, gu, gv, gw, hip_stream, nullptr);
}

extern "C" pf_status phasefield_adjoint_step_stages(pf_solver* s, const void* phi_n,
                                                    const void* y2, const void* y3,
                                                    const void* y4, const void* u, const void* v,
                                                    const void* w, double t_n, void* lam,
                                                    void* gu, void* gv, void* gw, void* hip_stream)
{
    pf_status st = adjoint_checks(s, phi_n, u, v, w, t_n, lam, gu, gv, gw);
    if (st != PF_OK) return st;
    const void* stages[3] = {y2, y3, y4};
    const int ns = scheme_stage_count(s->p.scheme);
    for (int k = 0; k < ns; ++k)
        if ((st = check_field_ptr(stages[k], k == 0 ? "y2" : k == 1 ? "y3" : "y4")) != PF_OK)
            return st;
    return adjoint_dispatch(s, phi_n, u, v, w, t_n, lam, gu, gv, gw, hip_stream, stages);
}

// ------------------------------------------------------------------------------ velocity
static pf_status velocity_common(const pf_params* p, int32_t modes, const double* phases)
{
    pf_status st = validate_params(p);
    if (st != PF_OK) return st;
    if (modes < 1 || modes > 64) return fail(PF_ERR_INVALID, "modes = %d out of [1, 64]", modes);
    if (!phases) return fail(PF_ERR_INVALID, "phases is NULL");
    return PF_OK;
}

extern "C" pf_status phasefield_velocity_from_coeffs(const pf_params* p, int32_t modes,
                                                     const double* phases, const double* coeffs,
                                                     void* u, void* v, void* w, void* hip_stream)
{
    pf_status st = velocity_common(p, modes, phases);
    if (st != PF_OK) return st;
    if (!coeffs) return fail(PF_ERR_INVALID, "coeffs is NULL");
    if ((st = check_field_ptr(u, "u")) != PF_OK) return st;
    if ((st = check_field_ptr(v, "v")) != PF_OK) return st;
    if ((st = check_field_ptr(w, "w")) != PF_OK) return st;
    hipStream_t hs = (hipStream_t)hip_stream;
    double* scratch = nullptr;
    const size_t nd = velocity_scratch_doubles(p->n[0], p->n[1], p->n[2], modes);
    hipError_t e = hipMalloc((void**)&scratch, nd * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "phasefield_velocity_from_coeffs: allocation");
    if (p->dtype == PF_F32)
        e = launch_velocity<float>(p->n[0], p->n[1], p->n[2], p->dx, modes, phases, coeffs,
                                   (float*)u, (float*)v, (float*)w, scratch, hs);
    else
        e = launch_velocity<double>(p->n[0], p->n[1], p->n[2], p->dx, modes, phases, coeffs,
                                    (double*)u, (double*)v, (double*)w, scratch, hs);
    hipError_t e2 = hipStreamSynchronize(hs);
    (void)hipFree(scratch);
    if (e == hipSuccess) e = e2;
    return e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_velocity_from_coeffs");
}

extern "C" pf_status phasefield_velocity_coeffs_grad(const pf_params* p, int32_t modes,
                                                     const double* phases, const void* gu,
                                                     const void* gv, const void* gw,
                                                     double* coeff_grad, void* hip_stream)
{
    pf_status st = velocity_common(p, modes, phases);
    if (st != PF_OK) return st;
    if (!coeff_grad) return fail(PF_ERR_INVALID, "coeff_grad is NULL");
    if ((st = check_field_ptr(gu, "gu")) != PF_OK) return st;
    if ((st = check_field_ptr(gv, "gv")) != PF_OK) return st;
    if ((st = check_field_ptr(gw, "gw")) != PF_OK) return st;
    hipStream_t hs = (hipStream_t)hip_stream;
    double* scratch = nullptr;
    const size_t nd = velocity_scratch_doubles(p->n[0], p->n[1], p->n[2], modes);
    hipError_t e = hipMalloc((void**)&scratch, nd * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "phasefield_velocity_coeffs_grad: allocation");
    if (p->dtype == PF_F32)
        e = launch_velocity_grad<float>(p->n[0], p->n[1], p->n[2], p->dx, modes, phases,
                                        (const float*)gu, (const float*)gv, (const float*)gw,
                                        coeff_grad, scratch, hs);
    else
        e = launch_velocity_grad<double>(p->n[0], p->n[1], p->n[2], p->dx, modes, phases,
                                         (const double*)gu, (const double*)gv, (const double*)gw,
                                         coeff_grad, scratch, hs);
    hipError_t e2 = hipStreamSynchronize(hs);
    (void)hipFree(scratch);
    if (e == hipSuccess) e = e2;
    return e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_velocity_coeffs_grad");
}

extern "C" pf_status phasefield_set_adjoint_form(pf_solver* s, int32_t form)
{
    if (!s) return fail(PF_ERR_INVALID, "solver is NULL");
    if (form < -1 || form > 1) return fail(PF_ERR_INVALID, "adjoint form %d is not -1, 0 or 1", (int)form);
    s->adjoint_form = form;
    return PF_OK;
}
