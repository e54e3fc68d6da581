// C ABI of the phase-field library: handles, validation, stage schedules, graph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pf_api_internal.h"

using namespace pf;

// ------------------------------------------------------------------------------ errors
static thread_local std::string g_err;

pf_status pf::fail(pf_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

pf_status pf::hip_fail(hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(PF_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
    return fail(PF_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char* phasefield_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------------------ params
extern "C" void phasefield_default_params(pf_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->n[0] = p->n[1] = p->n[2] = 1;
    p->dx = 1.0;
    p->bc[0] = p->bc[1] = p->bc[2] = PF_BC_PERIODIC;
    p->dtype = PF_F64;
    p->scheme = PF_RK4;
    p->vel_mode = PF_VEL_STEADY;
    p->vel_T = 1.0;
    p->variant = -1;
    p->use_graph = 1;
}

int pf::wall_mask(const pf_params& p)
{
    return (p.bc[0] == PF_BC_WALL ? 1 : 0) | (p.bc[1] == PF_BC_WALL ? 2 : 0) |
           (p.bc[2] == PF_BC_WALL ? 4 : 0);
}

pf_status pf::validate_params(const pf_params* p)
{
    if (!p) return fail(PF_ERR_INVALID, "params is NULL");
    for (int a = 0; a < 3; ++a) {
        if (p->n[a] < 1 || p->n[a] > (1 << 20))
            return fail(PF_ERR_INVALID, "n[%d] = %d out of range [1, 2^20]", a, p->n[a]);
        if (p->bc[a] != PF_BC_PERIODIC && p->bc[a] != PF_BC_WALL)
            return fail(PF_ERR_INVALID, "bc[%d] = %d", a, p->bc[a]);
    }
    const double cells = (double)p->n[0] * p->n[1] * p->n[2];
    if (cells > 4.0e9) return fail(PF_ERR_INVALID, "grid of %.3g cells is too large", cells);
    if (p->n[2] > 65535 || p->n[1] > 65535)
        return fail(PF_ERR_INVALID, "n[1] and n[2] must be <= 65535");
    if ((double)p->n[0] * p->n[1] * 8.0 >= 2147483648.0)
        return fail(PF_ERR_INVALID, "an xy plane must hold fewer than 2^28 cells");
    if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return fail(PF_ERR_INVALID, "dx must be > 0");
    if (!(p->eps >= 0.0) || !std::isfinite(p->eps)) return fail(PF_ERR_INVALID, "eps must be >= 0");
    if (!(p->gamma >= 0.0) || !std::isfinite(p->gamma))
        return fail(PF_ERR_INVALID, "gamma must be >= 0");
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(PF_ERR_INVALID, "dt must be > 0");
    if (!(p->delta >= 0.0) || !std::isfinite(p->delta))
        return fail(PF_ERR_INVALID, "delta must be >= 0");
    if (p->dtype != PF_F32 && p->dtype != PF_F64) return fail(PF_ERR_INVALID, "dtype = %d", p->dtype);
    if (p->scheme != PF_EULER && p->scheme != PF_RK2 && p->scheme != PF_RK3 && p->scheme != PF_RK4)
        return fail(PF_ERR_INVALID, "scheme = %d", p->scheme);
    if (p->vel_mode != PF_VEL_STEADY && p->vel_mode != PF_VEL_COS_REVERSAL)
        return fail(PF_ERR_INVALID, "vel_mode = %d", p->vel_mode);
    if (p->vel_mode == PF_VEL_COS_REVERSAL && !(p->vel_T > 0.0))
        return fail(PF_ERR_INVALID, "vel_T must be > 0 with the cos reversal");
    if (p->variant < -1 || p->variant >= stage_variant_count(p->dtype))
        return fail(PF_ERR_INVALID, "variant %d out of range for this dtype", p->variant);
    return PF_OK;
}

static int active_dims(const int32_t n[3])
{
    const int d = (n[0] > 1) + (n[1] > 1) + (n[2] > 1);
    return d > 0 ? d : 1;
}

extern "C" pf_status phasefield_check_params(const pf_params* p, double max_face_speed,
                                             pf_report* out)
{
    pf_status st = validate_params(p);
    if (st != PF_OK) return st;
    if (!out) return fail(PF_ERR_INVALID, "out is NULL");
    if (!(max_face_speed >= 0.0)) return fail(PF_ERR_INVALID, "max_face_speed must be >= 0");
    // Eq. 17: eps/dx >= (gamma/U + 1) / (2 gamma/U) = (gamma + U) / (2 gamma)
    double thr;
    if (p->gamma > 0.0)
        thr = (p->gamma + max_face_speed) / (2.0 * p->gamma);
    else
        thr = max_face_speed > 0.0 ? INFINITY : 0.5;
    out->crossover_margin_eq17 = p->eps / p->dx - thr;
    out->crossover_margin_eq24 = out->crossover_margin_eq17;
    const int D = active_dims(p->n);
    const double ge = p->gamma * p->eps;
    const double base = ge > 0.0 ? p->dx * p->dx / ge : INFINITY;
    // Eq. 25 (Euler) and Eq. 26 (RK2) coincide; Eq. 27 (RK3), Eq. 28 (RK4)
    out->dt_max_scheme = p->scheme == PF_RK4   ? 2.79 * base / (4.0 * D)
                         : p->scheme == PF_RK3 ? 2.51 * base / (4.0 * D)
                                               : base / (2.0 * D);
    out->dt_over_dtmax = p->dt / out->dt_max_scheme;
    return PF_OK;
}

// ------------------------------------------------------------------------------ tuning cache
// Tuned variants per (dtype, grid), kept for the process and, when the environment variable
// PF_TUNE_CACHE names a file, persisted there as lines "dtype nx ny nz variant_name" (names,
// not indices, so a cache survives a rebuild that reorders the table; unknown names are
// ignored).
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int>, int> g_tuned;
static std::string g_tune_path;  // cache file the in-process table was last read from

static int variant_by_name(int dtype, const char* name)
{
    for (int v = 0; v < stage_variant_count(dtype); ++v)
        if (std::strcmp(stage_variant(dtype, v).name, name) == 0) return v;
    return -1;
}

static void load_tune_cache_locked()
{
    const char* path = std::getenv("PF_TUNE_CACHE");
    if (!path || !*path || g_tune_path == path) return;
    g_tune_path = path;  // (re)read whenever the variable names a different file
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    int d, nx, ny, nz;
    char name[128];
    while (std::fscanf(f, "%d %d %d %d %127s", &d, &nx, &ny, &nz, name) == 5) {
        if (d != PF_F32 && d != PF_F64) continue;
        const int v = variant_by_name(d, name);
        if (v >= 0) g_tuned[std::make_tuple(d, nx, ny, nz)] = v;
    }
    std::fclose(f);
}

static void save_tune_cache_locked()
{
    const char* path = std::getenv("PF_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto& kv : g_tuned)
        std::fprintf(f, "%d %d %d %d %s\n", std::get<0>(kv.first), std::get<1>(kv.first),
                     std::get<2>(kv.first), std::get<3>(kv.first),
                     stage_variant(std::get<0>(kv.first), kv.second).name);
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

int pf::tuned_variant(int dtype, const int32_t n[3])
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    auto it = g_tuned.find(std::make_tuple(dtype, n[0], n[1], n[2]));
    if (it != g_tuned.end()) return it->second;
    return default_stage_variant(n[0], n[1], n[2], dtype);
}

// Default variant of a grid with walls (the tuning cache is kept for periodic grids). Walls cost
// the fused sweeps their 16-byte plane loads and scalar registers (walls on x and z, per step:
// FP64 512^3 fused_32x16 7.08 ms against tiled_64x8 6.09, 128^3 0.162 against 0.105 on
// tiled_32x4; FP32 512^3 fused_32x16 2.78 against fused_64x8 3.04 and tiled_64x8 3.29, 256^3
// 0.352 against 0.436, 160^3 0.106 against 0.124, 128^3 0.082 against 0.077 on tiled_32x4):
// FP64 takes the per-stage kernel, FP32 the fused 32x16 sweeps from 144^3 cells and per-stage
// 64x8 tiles below (32x4 where 64-wide tiles pad more columns).
static int walled_default_variant(int dtype, const int32_t n[3])
{
    if (dtype == PF_F64) return per_stage_variant(n[0], n[1], n[2], dtype);
    const long long cells = (long long)n[0] * n[1] * n[2];
    if (cells >= 144LL * 144 * 144) return stage_variant_index(dtype, "fused_32x16");
    const bool x64 = (n[0] + 63) / 64 * 64 <= (n[0] + 31) / 32 * 32;
    return stage_variant_index(dtype, x64 ? "tiled_64x8" : "tiled_32x4");
}

int pf::default_variant(const pf_params& p)
{
    return wall_mask(p) != 0 ? walled_default_variant(p.dtype, p.n) : tuned_variant(p.dtype, p.n);
}

static void store_tuned(int dtype, const int32_t n[3], int v)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    g_tuned[std::make_tuple(dtype, n[0], n[1], n[2])] = v;
    save_tune_cache_locked();
}

extern "C" int32_t phasefield_variant_count(int32_t dtype)
{
    if (dtype != PF_F32 && dtype != PF_F64) return 0;
    return stage_variant_count(dtype);
}

extern "C" const char* phasefield_variant_name(int32_t dtype, int32_t v)
{
    if (dtype != PF_F32 && dtype != PF_F64) return nullptr;
    if (v < 0 || v >= stage_variant_count(dtype)) return nullptr;
    return stage_variant(dtype, v).name;
}

// ------------------------------------------------------------------------------ solver
static void free_dev(void*& ptr)
{
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
}

void pf::release_graph(StepGraph& g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = StepGraph{};
}

extern "C" pf_status phasefield_create(const pf_params* p, pf_solver** out)
{
    if (!out) return fail(PF_ERR_INVALID, "out is NULL");
    *out = nullptr;
    pf_status st = validate_params(p);
    if (st != PF_OK) return st;
    auto* s = new pf_solver();
    s->p = *p;
    s->N = (size_t)p->n[0] * p->n[1] * p->n[2];
    s->esz = p->dtype == PF_F32 ? sizeof(float) : sizeof(double);
    s->variant = p->variant >= 0 ? p->variant : default_variant(*p);
    hipError_t e = hipSuccess;
    for (void** b : {&s->ya, &s->yb, &s->acc}) {
        e = hipMalloc(b, s->N * s->esz);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipMalloc((void**)&s->red_part, sizeof(double) * 4 * kReduceBlocks);
    if (e == hipSuccess) e = hipMalloc((void**)&s->red_out, sizeof(double) * 4);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->red_host, sizeof(double) * 4);
    if (e != hipSuccess) {
        phasefield_destroy(s);
        return hip_fail(e, "phasefield_create: allocation");
    }
    *out = s;
    return PF_OK;
}

static void free_mesh(NuMesh& m);

extern "C" pf_status phasefield_destroy(pf_solver* s)
{
    if (!s) return PF_OK;
    (void)hipDeviceSynchronize();
    release_graph(s->graph);
    for (void** b : {&s->ya, &s->yb, &s->acc}) free_dev(*b);
    for (auto& b : s->adj) free_dev(b);
    void* rp = s->red_part;
    void* ro = s->red_out;
    free_dev(rp);
    free_dev(ro);
    if (s->red_host) (void)hipHostFree(s->red_host);
    free_dev(s->vel_scratch);
    free_mesh(s->nu);
    delete s;
    return PF_OK;
}

// ------------------------------------------------------------------ non-uniform meshes
static void free_mesh(NuMesh& m)
{
    for (int a = 0; a < 3; ++a) {
        free_dev(m.tab[a]);
        void* w = m.width[a];
        free_dev(w);
        m.width[a] = nullptr;
    }
    m.eps_mode = 0;
}

// One axis: the kNuCols columns per cell index (NuCol) in the storage dtype, and the widths for
// the volume weights. The width index wraps on a periodic axis and mirrors across walls.
template <typename T>
static hipError_t upload_axis(const double* h, int n, bool walled, void** tab, double** width)
{
    auto wid = [&](long idx) {
        long m;
        if (walled) {
            const long p2 = 2L * n;
            long r = idx % p2;
            if (r < 0) r += p2;
            m = r < n ? r : p2 - 1 - r;
        } else {
            m = idx % n;
            if (m < 0) m += n;
        }
        return h[m];
    };
    auto dist = [&](long idx) { return 0.5 * (wid(idx - 1) + wid(idx)); };
    std::vector<T> t((size_t)n * kNuCols);
    for (long i = 0; i < n; ++i) {
        T* r = t.data() + (size_t)i * kNuCols;
        r[kNuInvW] = (T)(1.0 / h[i]);
        r[kNuInvSpan] = (T)(1.0 / (dist(i) + dist(i + 1)));
        r[kNuInvDist] = (T)(1.0 / dist(i));
        r[kNuWidth] = n == 1 ? T(0) : (T)h[i];  // a one-cell axis is left out of the local eps
    }
    // an axis of one cell carries no volume
    std::vector<double> w(h, h + n);
    if (n == 1) w[0] = 1.0;
    hipError_t e = hipMalloc(tab, t.size() * sizeof(T));
    if (e == hipSuccess) e = hipMemcpy(*tab, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)width, w.size() * sizeof(double));
    if (e == hipSuccess)
        e = hipMemcpy(*width, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice);
    return e;
}

extern "C" pf_status phasefield_set_spacing(pf_solver* s, const double* hx, const double* hy,
                                            const double* hz, int32_t eps_mode)
{
    if (!s) return fail(PF_ERR_INVALID, "solver is NULL");
    const double* h[3] = {hx, hy, hz};
    const int given = (hx != nullptr) + (hy != nullptr) + (hz != nullptr);
    if (given != 0 && given != 3) return fail(PF_ERR_INVALID, "give hx, hy and hz, or none");
    if (eps_mode != 0 && eps_mode != 1) return fail(PF_ERR_INVALID, "eps_mode %d is not 0 or 1", (int)eps_mode);
    if (given == 3)
        for (int a = 0; a < 3; ++a)
            for (int i = 0; i < s->p.n[a]; ++i)
                if (!(std::isfinite(h[a][i]) && h[a][i] > 0.0))
                    return fail(PF_ERR_INVALID, "width %d of axis %c is not positive and finite", i,
                                "xyz"[a]);
    // queued work may still read the old tables
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "phasefield_set_spacing: synchronize");
    release_graph(s->graph);
    free_mesh(s->nu);
    if (given == 0) return PF_OK;
    const int wm = wall_mask(s->p);
    for (int a = 0; a < 3 && e == hipSuccess; ++a)
        e = s->p.dtype == PF_F32
                ? upload_axis<float>(h[a], s->p.n[a], (wm >> a) & 1, &s->nu.tab[a], &s->nu.width[a])
                : upload_axis<double>(h[a], s->p.n[a], (wm >> a) & 1, &s->nu.tab[a], &s->nu.width[a]);
    if (e != hipSuccess) {
        free_mesh(s->nu);
        return e == hipErrorOutOfMemory ? fail(PF_ERR_OOM, "phasefield_set_spacing: out of memory")
                                        : hip_fail(e, "phasefield_set_spacing: upload");
    }
    s->nu.eps_mode = eps_mode;
    return PF_OK;
}

extern "C" int32_t phasefield_solver_variant(const pf_solver* s) { return s ? s->variant : -1; }

pf_status pf::check_field_ptr(const void* ptr, const char* name)
{
    if (!ptr) return fail(PF_ERR_INVALID, "%s is NULL", name);
    if (((uintptr_t)ptr) & 15) return fail(PF_ERR_INVALID, "%s is not 16-byte aligned", name);
    return PF_OK;
}

double pf::time_factor(const pf_params& p, double t)
{
    return p.vel_mode == PF_VEL_COS_REVERSAL ? std::cos(M_PI * t / p.vel_T) : 1.0;
}

template <typename T>
StageArgs<T> pf::make_stage(const pf_params& p, double svel, const T* y, const T* base1,
                            const T* base2, T* out1, T* out2, double c1, double c2, const T* U,
                            const T* V, const T* W, const NuMesh* nu)
{
    StageArgs<T> a;
    a.y = y;
    a.base1 = base1;
    a.base2 = base2;
    a.out1 = out1;
    a.out2 = out2;
    a.U = U;
    a.V = V;
    a.W = W;
    a.nx = p.n[0];
    a.ny = p.n[1];
    a.nz = p.n[2];
    a.inv_2dx = (T)(1.0 / (2.0 * p.dx));
    a.ge = (T)(p.gamma * p.eps / (p.dx * p.dx));
    a.hg = (T)(0.5 * p.gamma / p.dx);
    a.nhs = (T)(-0.5 * svel / p.dx);
    a.delta2 = (T)(p.delta * p.delta);
    a.c1 = (T)c1;
    a.c2 = (T)c2;
    a.walls = wall_mask(p);
    if (nu && nu->on()) {
        for (int ax = 0; ax < 3; ++ax) a.nu[ax] = (const T*)nu->tab[ax];
        a.nu_ge = (T)(nu->eps_mode == 1 ? p.gamma * p.eps / p.dx : p.gamma * p.eps);
        a.nu_hg = (T)(0.5 * p.gamma);
        a.nu_nhs = (T)(-0.5 * svel);
        a.nu_eps_mode = nu->eps_mode;
    }
    return a;
}
template StageArgs<float> pf::make_stage<float>(const pf_params&, double, const float*,
                                                const float*, const float*, float*, float*,
                                                double, double, const float*, const float*,
                                                const float*, const NuMesh*);
template StageArgs<double> pf::make_stage<double>(const pf_params&, double, const double*,
                                                  const double*, const double*, double*,
                                                  double*, double, double, const double*,
                                                  const double*, const double*, const NuMesh*);

template <typename T>
hipError_t pf::run_stage(int variant, const StageArgs<T>& a, hipStream_t st)
{
    constexpr int dtype = sizeof(T) == 4 ? PF_F32 : PF_F64;
    if (a.nu[0]) return launch_stage_nu<T>(a, st);
    const int v = variant_is_fused(dtype, variant) ? per_stage_variant(a.nx, a.ny, a.nz, dtype) : variant;
    const StageVariant& sv = stage_variant(dtype, v);
    if constexpr (sizeof(T) == 4)
        return sv.launch_f32(a, st);
    else
        return sv.launch_f64(a, st);
}
template hipError_t pf::run_stage<float>(int, const StageArgs<float>&, hipStream_t);
template hipError_t pf::run_stage<double>(int, const StageArgs<double>&, hipStream_t);

// One explicit step from time t on the given buffers (phi updated in place).
//   RK4 (classic; Sec. 2.3, Eq. 28), fixed buffers, no pointer swaps:
//     S1: ya = phi + dt/2 k1,  acc = phi + dt/6 k1          (k1 = f(phi, t))
//     S2: yb = phi + dt/2 k2,  acc += dt/3 k2               (k2 = f(ya, t + dt/2))
//     S3: ya = phi + dt k3,    acc += dt/3 k3               (k3 = f(yb, t + dt/2))
//     S4: phi = acc + dt/6 k4                               (k4 = f(ya, t + dt))
//   Euler (Eq. 25): acc = phi + dt f(phi, t); phi = acc (a run of steps alternates phi and acc
//   instead, enqueue_steps).
//   RK2, the explicit midpoint rule (Eq. 26):
//     S1: ya = phi + dt/2 k1;  S2: phi = phi + dt k2   (k2 = f(ya, t + dt/2))
//   RK3, low storage (Eq. 27), u1 = u0 + dt g1 k1, u2 = u1 + dt (g2 k2 + z2 k1),
//   u3 = u2 + dt (g3 k3 + z3 k2), with acc carrying the part of the next stage known so far:
//     S1: ya = phi + dt g1 k1,  acc = phi + dt (g1 + z2) k1             (k1 = f(phi, t))
//     S2: yb = acc + dt g2 k2  (acc += dt (g2 + z3) k2 is a no-op: g2 + z3 = 0)
//     S3: phi = acc + dt g3 k3                            (k2, k3 at t + g1 dt, t + (g1 + g2 + z2) dt)
// S4 writes phi in place: it reads phi nowhere (its stencil input is ya, acc is read only at
// the cell being written). RK2's S2 likewise reads phi only at the cell it writes.
template <typename T>
hipError_t pf::enqueue_step(const pf_params& p, int variant, T* phi, const T* U, const T* V,
                            const T* W, T* ya, T* yb, T* acc, double t, hipStream_t st,
                            const NuMesh* nu)
{
    const double dt = p.dt;
    hipError_t e;
    if (p.scheme == PF_EULER) {
        e = run_stage<T>(variant, make_stage<T>(p, time_factor(p, t), phi, nullptr, phi, nullptr,
                                                acc, 0.0, dt, U, V, W, nu), st);
        if (e != hipSuccess) return e;
        return launch_copy<T>(phi, acc, (size_t)p.n[0] * p.n[1] * p.n[2], st);
    }
    const double sh = time_factor(p, t + 0.5 * dt);
    if (p.scheme == PF_RK3) {
        constexpr double g1 = 8.0 / 15.0, g2 = 5.0 / 12.0, g3 = 0.75, z2 = -17.0 / 60.0,
                         z3 = -5.0 / 12.0;
        e = run_stage<T>(variant, make_stage<T>(p, time_factor(p, t), phi, phi, phi, ya, acc,
                                                dt * g1, dt * (g1 + z2), U, V, W, nu), st);
        if (e != hipSuccess) return e;
        static_assert(g2 + z3 == 0.0, "acc already holds u2 + dt z3 k2 after S2");
        e = run_stage<T>(variant, make_stage<T>(p, time_factor(p, t + g1 * dt), ya, acc, nullptr,
                                                yb, nullptr, dt * g2, 0.0, U, V, W, nu), st);
        if (e != hipSuccess) return e;
        return run_stage<T>(variant, make_stage<T>(p, time_factor(p, t + (g1 + g2 + z2) * dt), yb,
                                                   nullptr, acc, nullptr, phi, 0.0, dt * g3, U, V, W, nu),
                            st);
    }
    if (p.scheme == PF_RK2) {
        e = run_stage<T>(variant, make_stage<T>(p, time_factor(p, t), phi, phi, nullptr, ya,
                                                nullptr, 0.5 * dt, 0.0, U, V, W, nu), st);
        if (e != hipSuccess) return e;
        return run_stage<T>(variant, make_stage<T>(p, sh, ya, nullptr, phi, nullptr, phi, 0.0, dt,
                                                   U, V, W, nu), st);
    }
    e = run_stage<T>(variant, make_stage<T>(p, time_factor(p, t), phi, phi, phi, ya, acc,
                                            0.5 * dt, dt / 6.0, U, V, W, nu), st);
    if (e != hipSuccess) return e;
    e = run_stage<T>(variant, make_stage<T>(p, sh, ya, phi, acc, yb, acc, 0.5 * dt, dt / 3.0, U, V, W, nu), st);
    if (e != hipSuccess) return e;
    e = run_stage<T>(variant, make_stage<T>(p, sh, yb, phi, acc, ya, acc, dt, dt / 3.0, U, V, W, nu),
                     st);
    if (e != hipSuccess) return e;
    return run_stage<T>(variant, make_stage<T>(p, time_factor(p, t + dt), ya, nullptr, acc,
                                               nullptr, phi, 0.0, dt / 6.0, U, V, W, nu), st);
}
template hipError_t pf::enqueue_step<float>(const pf_params&, int, float*, const float*,
                                            const float*, const float*, float*, float*, float*,
                                            double, hipStream_t, const NuMesh*);
template hipError_t pf::enqueue_step<double>(const pf_params&, int, double*, const double*,
                                             const double*, const double*, double*, double*,
                                             double*, double, hipStream_t, const NuMesh*);

// Arguments of one fused sweep of the RK4 step at time t (pf_fused_body.h): sweep A runs stages
// 1-2 from phi_cur (writing yb and the accumulator into phi_next), sweep B runs stages 3-4 from
// yb (writing the new phi over the accumulator in phi_next). RK2 is sweep A alone: the midpoint
// value in LDS, the new phi into phi_next, no accumulator.
template <typename T>
FusedArgs<T> pf::make_fused(const pf_params& p, bool sweep_b, double t, const T* phi_cur,
                            T* phi_next, const T* U, const T* V, const T* W, T* yb)
{
    const double dt = p.dt;
    FusedArgs<T> a;
    a.U = U;
    a.V = V;
    a.W = W;
    a.nx = p.n[0];
    a.ny = p.n[1];
    a.nz = p.n[2];
    a.inv_2dx = (T)(1.0 / (2.0 * p.dx));
    a.ge = (T)(p.gamma * p.eps / (p.dx * p.dx));
    a.hg = (T)(0.5 * p.gamma / p.dx);
    a.delta2 = (T)(p.delta * p.delta);
    a.walls = wall_mask(p);
    a.phi = phi_cur;
    a.out_acc = phi_next;
    a.out_mid = nullptr;
    a.out_phi = nullptr;
    if (p.scheme == PF_RK2) {
        a.y = phi_cur;
        a.acc_in = nullptr;
        a.out_y = phi_next;
        a.out_acc = nullptr;
        a.nhs1 = (T)(-0.5 * time_factor(p, t) / p.dx);
        a.nhs2 = (T)(-0.5 * time_factor(p, t + 0.5 * dt) / p.dx);
        a.c_mid = (T)(0.5 * dt);
        a.c_acc1 = (T)0;
        a.c_y2 = (T)dt;
        a.c_acc2 = (T)0;
    } else if (!sweep_b) {
        a.y = phi_cur;
        a.acc_in = nullptr;
        a.out_y = yb;
        a.nhs1 = (T)(-0.5 * time_factor(p, t) / p.dx);
        a.nhs2 = (T)(-0.5 * time_factor(p, t + 0.5 * dt) / p.dx);
        a.c_mid = (T)(0.5 * dt);
        a.c_acc1 = (T)(dt / 6.0);
        a.c_y2 = (T)(0.5 * dt);
        a.c_acc2 = (T)(dt / 3.0);
    } else {
        a.y = yb;
        a.acc_in = phi_next;
        a.out_y = nullptr;
        a.nhs1 = (T)(-0.5 * time_factor(p, t + 0.5 * dt) / p.dx);
        a.nhs2 = (T)(-0.5 * time_factor(p, t + dt) / p.dx);
        a.c_mid = (T)dt;
        a.c_acc1 = (T)(dt / 3.0);
        a.c_y2 = (T)0;
        a.c_acc2 = (T)(dt / 6.0);
    }
    return a;
}
template FusedArgs<float> pf::make_fused<float>(const pf_params&, bool, double, const float*,
                                                float*, const float*, const float*, const float*,
                                                float*);
template FusedArgs<double> pf::make_fused<double>(const pf_params&, bool, double, const double*,
                                                  double*, const double*, const double*,
                                                  const double*, double*);

template <typename T>
hipError_t pf::run_fused_sweep(int variant, const FusedArgs<T>& a, bool sweep_b, hipStream_t st)
{
    constexpr int dtype = sizeof(T) == 4 ? PF_F32 : PF_F64;
    const StageVariant& sv = stage_variant(dtype, variant);
    if constexpr (sizeof(T) == 4)
        return sv.fused_f32 ? sv.fused_f32(a, sweep_b, st) : hipErrorInvalidValue;
    else
        return sv.fused_f64 ? sv.fused_f64(a, sweep_b, st) : hipErrorInvalidValue;
}
template hipError_t pf::run_fused_sweep<float>(int, const FusedArgs<float>&, bool, hipStream_t);
template hipError_t pf::run_fused_sweep<double>(int, const FusedArgs<double>&, bool, hipStream_t);

// One RK4 step as two fused sweeps (RK2: sweep A alone); the new phi lands in phi_next. Sweep A
// writes the accumulator into acc_buf (for the plain form, phi_next itself). With phi_copy (RK4
// only), sweep A also copies phi_cur there and sweep B takes its phi from that copy, so nothing
// reads phi_cur during sweep B and phi_next may be phi_cur: the step runs in place.
template <typename T>
static hipError_t enqueue_step_fused(const pf_params& p, int variant, const T* phi_cur,
                                     T* phi_next, T* acc_buf, T* phi_copy, const T* U,
                                     const T* V, const T* W, T* yb, double t, hipStream_t st)
{
    FusedArgs<T> a = make_fused<T>(p, false, t, phi_cur, p.scheme == PF_RK2 ? phi_next : acc_buf,
                                   U, V, W, yb);
    if (phi_copy) a.out_phi = phi_copy;
    hipError_t e = run_fused_sweep<T>(variant, a, false, st);
    if (e != hipSuccess || p.scheme == PF_RK2) return e;
    FusedArgs<T> b = make_fused<T>(p, true, t, phi_copy ? phi_copy : phi_cur, acc_buf, U, V, W, yb);
    b.out_acc = phi_next;
    return run_fused_sweep<T>(variant, b, true, st);
}

// nsteps steps from t0 (step m at t0 + m dt), phi updated in place. A fused variant alternates
// phi between the caller's buffer and acc; after an odd count RK4 runs its last step in place
// (through a copy of phi in ya), RK2 copies back.
template <typename T>
hipError_t pf::enqueue_steps(const pf_params& p, int variant, T* phi, const T* U, const T* V,
                             const T* W, T* ya, T* yb, T* acc, double t0, int nsteps,
                             hipStream_t st, const NuMesh* nu)
{
    constexpr int dtype = sizeof(T) == 4 ? PF_F32 : PF_F64;
    // the fused sweeps run RK4 and RK2 on uniform meshes with periodic or walled axes (arrays
    // below 4 GiB when walled); otherwise their variants run the per-stage kernel
    const int wm = wall_mask(p);
    const bool fused = (p.scheme == PF_RK4 || p.scheme == PF_RK2) && variant_is_fused(dtype, variant) &&
                       !(wm != 0 && field_needs_big(p.n[0], p.n[1], p.n[2], sizeof(T))) &&
                       !(nu && nu->on());
    T* cur = phi;
    for (int m = 0; m < nsteps; ++m) {
        const double t = t0 + (double)m * p.dt;
        hipError_t e;
        if (p.scheme == PF_EULER) {
            // the Euler stage reads cur with its stencil and writes the other buffer of the pair
            // (phi, acc); no copy per step
            T* next = cur == phi ? acc : phi;
            e = run_stage<T>(variant, make_stage<T>(p, time_factor(p, t), cur, nullptr, cur, nullptr,
                                                    next, 0.0, p.dt, U, V, W, nu), st);
            cur = next;
        } else if (fused) {
            if (m == nsteps - 1 && cur == phi && p.scheme == PF_RK4) {
                e = enqueue_step_fused<T>(p, variant, phi, phi, acc, ya, U, V, W, yb, t, st);
            } else {
                T* next = cur == phi ? acc : phi;
                e = enqueue_step_fused<T>(p, variant, cur, next, next, nullptr, U, V, W, yb, t, st);
                cur = next;
            }
        } else {
            e = enqueue_step<T>(p, variant, phi, U, V, W, ya, yb, acc, t, st, nu);
        }
        if (e != hipSuccess) return e;
    }
    if (cur != phi) return launch_copy<T>(phi, cur, (size_t)p.n[0] * p.n[1] * p.n[2], st);
    return hipSuccess;
}
template hipError_t pf::enqueue_steps<float>(const pf_params&, int, float*, const float*,
                                             const float*, const float*, float*, float*, float*,
                                             double, int, hipStream_t, const NuMesh*);
template hipError_t pf::enqueue_steps<double>(const pf_params&, int, double*, const double*,
                                              const double*, const double*, double*, double*,
                                              double*, double, int, hipStream_t, const NuMesh*);

// Capture `nsteps` steps from t0 on stream st into the handle's graph (replacing what it held)
// and instantiate it.
template <typename T>
static pf_status capture_steps(pf_solver* s, T* phi, const T* U, const T* V, const T* W,
                               double t0, int32_t nsteps, hipStream_t st)
{
    StepGraph& g = s->graph;
    release_graph(g);
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "phasefield_step: begin capture");
    const hipError_t le = enqueue_steps<T>(s->p, s->variant, phi, U, V, W, (T*)s->ya, (T*)s->yb,
                                           (T*)s->acc, t0, nsteps, st, &s->nu);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le, "phasefield_step: launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "phasefield_step: end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "phasefield_step: instantiate");
    }
    g.graph = graph;
    g.exec = exec;
    g.phi = phi;
    g.U = U;
    g.V = V;
    g.W = W;
    g.stream = st;
    g.variant = s->variant;
    g.t0 = t0;
    g.nsteps = nsteps;
    return PF_OK;
}

template <typename T>
static pf_status step_impl(pf_solver* s, T* phi, const T* U, const T* V, const T* W, double t0,
                           int32_t nsteps, hipStream_t st)
{
    const pf_params& p = s->p;
    StepGraph& g = s->graph;
    // (capture is not possible on the legacy NULL stream)
    const bool graphs = p.use_graph && st != nullptr;
    auto same_operands = [&]() {
        return g.exec && g.phi == phi && g.U == U && g.V == V && g.W == W && g.stream == st &&
               g.variant == s->variant;
    };
    if (graphs && p.vel_mode != PF_VEL_STEADY && nsteps >= kLoopGraphMin &&
        nsteps <= kLoopGraphMax) {
        // time-varying velocity: the whole loop is one graph
        if (!(same_operands() && g.t0 == t0 && g.nsteps == nsteps)) {
            const pf_status cs = capture_steps<T>(s, phi, U, V, W, t0, nsteps, st);
            if (cs != PF_OK) return cs;
        }
        const hipError_t e = hipGraphLaunch(g.exec, st);
        return e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_step: graph launch");
    }
    // Steady velocity: every step is the same launch sequence, replayed from a captured graph
    // of kGraphSteps steps.
    int32_t done = 0;
    if (graphs && p.vel_mode == PF_VEL_STEADY && nsteps >= kGraphSteps) {
        if (!(same_operands() && g.nsteps == kGraphSteps)) {
            const pf_status cs = capture_steps<T>(s, phi, U, V, W, 0.0, kGraphSteps, st);
            if (cs != PF_OK) return cs;
        }
        for (; done + kGraphSteps <= nsteps; done += kGraphSteps) {
            hipError_t e = hipGraphLaunch(g.exec, st);
            if (e != hipSuccess) return hip_fail(e, "phasefield_step: graph launch");
        }
    }
    if (done < nsteps) {
        hipError_t e = enqueue_steps<T>(p, s->variant, phi, U, V, W, (T*)s->ya, (T*)s->yb,
                                        (T*)s->acc, t0 + (double)done * p.dt, nsteps - done, st,
                                        &s->nu);
        if (e != hipSuccess) return hip_fail(e, "phasefield_step: launch");
    }
    return PF_OK;
}

extern "C" pf_status phasefield_step(pf_solver* s, void* phi, const void* u, const void* v,
                                     const void* w, double t0, int32_t nsteps, void* hip_stream)
{
    if (!s) return fail(PF_ERR_INVALID, "solver is NULL");
    pf_status st;
    if ((st = check_field_ptr(phi, "phi")) != PF_OK) return st;
    if ((st = check_field_ptr(u, "u")) != PF_OK) return st;
    if ((st = check_field_ptr(v, "v")) != PF_OK) return st;
    if ((st = check_field_ptr(w, "w")) != PF_OK) return st;
    if (nsteps < 0) return fail(PF_ERR_INVALID, "nsteps < 0");
    if (!std::isfinite(t0)) return fail(PF_ERR_INVALID, "t0 is not finite");
    if (nsteps == 0) return PF_OK;
    hipStream_t hs = (hipStream_t)hip_stream;
    if (s->p.dtype == PF_F32)
        return step_impl<float>(s, (float*)phi, (const float*)u, (const float*)v, (const float*)w,
                                t0, nsteps, hs);
    return step_impl<double>(s, (double*)phi, (const double*)u, (const double*)v,
                             (const double*)w, t0, nsteps, hs);
}

// One step of the handle's scheme from time t that also stores the stage inputs the adjoint step
// reads (scheme_stage_count), the new phi into phi_next (phi itself: in place): the per-stage
// launches with the stage outputs directed into the caller's buffers; an RK4 step of a fused
// variant (no walls; FP64 from 176^3 cells, where the fused sweeps overtake the per-stage
// launches) runs its two sweeps, each storing its middle value (y2, y4; sweep A also writes y3),
// when out of place, and in place sweep A then two per-stage launches for y4 and the new phi;
// on a non-uniform mesh the per-stage launches of that mesh's kernel. Every form rounds alike, so the new phi and the stages are bit-identical to those of
// phasefield_step and of the adjoint's own recompute.
template <typename T>
static hipError_t step_stages_impl(pf_solver* s, const T* phi, T* phi_next, const T* U,
                                   const T* V, const T* W, double t, T* y2, T* y3, T* y4,
                                   hipStream_t st)
{
    const pf_params& p = s->p;
    const double dt = p.dt;
    T* acc = (T*)s->acc;
    const int v = s->variant;
    const double sh = time_factor(p, t + 0.5 * dt);
    const NuMesh* nu = s->nu.on() ? &s->nu : nullptr;
    hipError_t e;
    if (p.scheme == PF_EULER) {
        if (phi_next == phi)  // in place: through the accumulator, as the step does
            return enqueue_step<T>(p, v, phi_next, U, V, W, (T*)s->ya, (T*)s->yb, acc, t, st,
                                   nu);
        return run_stage<T>(v, make_stage<T>(p, time_factor(p, t), phi, nullptr, phi, nullptr,
                                             phi_next, 0.0, dt, U, V, W, nu), st);
    }
    if (p.scheme == PF_RK2) {
        e = run_stage<T>(v, make_stage<T>(p, time_factor(p, t), phi, phi, nullptr, y2, nullptr,
                                          0.5 * dt, 0.0, U, V, W, nu), st);
        if (e != hipSuccess) return e;
        return run_stage<T>(v, make_stage<T>(p, sh, y2, nullptr, phi, nullptr, phi_next, 0.0, dt,
                                             U, V, W, nu), st);
    }
    if (p.scheme == PF_RK3) {
        constexpr double g1 = 8.0 / 15.0, g2 = 5.0 / 12.0, g3 = 0.75, z2 = -17.0 / 60.0;
        e = run_stage<T>(v, make_stage<T>(p, time_factor(p, t), phi, phi, phi, y2, acc, dt * g1,
                                          dt * (g1 + z2), U, V, W, nu), st);
        if (e != hipSuccess) return e;
        e = run_stage<T>(v, make_stage<T>(p, time_factor(p, t + g1 * dt), y2, acc, nullptr, y3,
                                          nullptr, dt * g2, 0.0, U, V, W, nu), st);
        if (e != hipSuccess) return e;
        return run_stage<T>(v, make_stage<T>(p, time_factor(p, t + (g1 + g2 + z2) * dt), y3,
                                             nullptr, acc, nullptr, phi_next, 0.0, dt * g3, U, V, W, nu),
                            st);
    }
    const long long cells = (long long)p.n[0] * p.n[1] * p.n[2];
    const bool fused = !nu && variant_is_fused(p.dtype, v) && wall_mask(p) == 0 &&
                       (p.dtype == PF_F32 || cells >= 176LL * 176 * 176);
    if (fused && phi_next != phi) {
        // out of place: the two sweeps of the step, the accumulator in phi_next (sweep B writes
        // the new phi over it at the cell), sweep A storing y2, sweep B y4
        FusedArgs<T> a = make_fused<T>(p, false, t, phi, phi_next, U, V, W, y3);
        a.out_mid = y2;
        e = run_fused_sweep<T>(v, a, false, st);
        if (e != hipSuccess) return e;
        FusedArgs<T> b = make_fused<T>(p, true, t, phi, phi_next, U, V, W, y3);
        b.out_mid = y4;
        return run_fused_sweep<T>(v, b, true, st);
    }
    if (fused) {
        FusedArgs<T> a = make_fused<T>(p, false, t, phi, acc, U, V, W, y3);
        a.out_mid = y2;
        e = run_fused_sweep<T>(v, a, false, st);
    } else {
        e = run_stage<T>(v, make_stage<T>(p, time_factor(p, t), phi, phi, phi, y2, acc, 0.5 * dt,
                                          dt / 6.0, U, V, W, nu), st);
        if (e == hipSuccess)
            e = run_stage<T>(v, make_stage<T>(p, sh, y2, phi, acc, y3, acc, 0.5 * dt, dt / 3.0, U, V,
                                              W, nu), st);
    }
    if (e == hipSuccess)
        e = run_stage<T>(v, make_stage<T>(p, sh, y3, phi, acc, y4, acc, dt, dt / 3.0, U, V, W, nu), st);
    if (e == hipSuccess)
        e = run_stage<T>(v, make_stage<T>(p, time_factor(p, t + dt), y4, nullptr, acc, nullptr,
                                          phi_next, 0.0, dt / 6.0, U, V, W, nu), st);
    return e;
}

extern "C" pf_status phasefield_step_stages(pf_solver* s, void* phi, void* phi_next, const void* u,
                                            const void* v, const void* w, double t, void* y2,
                                            void* y3, void* y4, void* hip_stream)
{
    if (!s) return fail(PF_ERR_INVALID, "solver is NULL");
    pf_status st;
    if ((st = check_field_ptr(phi, "phi")) != PF_OK) return st;
    if ((st = check_field_ptr(u, "u")) != PF_OK) return st;
    if ((st = check_field_ptr(v, "v")) != PF_OK) return st;
    if ((st = check_field_ptr(w, "w")) != PF_OK) return st;
    if (!phi_next) phi_next = phi;
    if ((st = check_field_ptr(phi_next, "phi_next")) != PF_OK) return st;
    if (!std::isfinite(t)) return fail(PF_ERR_INVALID, "t is not finite");
    void* stages[3] = {y2, y3, y4};
    const int ns = scheme_stage_count(s->p.scheme);
    for (int k = 0; k < ns; ++k) {
        if ((st = check_field_ptr(stages[k], k == 0 ? "y2" : k == 1 ? "y3" : "y4")) != PF_OK)
            return st;
        if (stages[k] == phi || stages[k] == phi_next)
            return fail(PF_ERR_INVALID, "a stage buffer is phi or phi_next");
        for (int j = 0; j < k; ++j)
            if (stages[j] == stages[k]) return fail(PF_ERR_INVALID, "stage buffers coincide");
    }
    hipStream_t hs = (hipStream_t)hip_stream;
    hipError_t e =
        s->p.dtype == PF_F32
            ? step_stages_impl<float>(s, (const float*)phi, (float*)phi_next, (const float*)u,
                                      (const float*)v, (const float*)w, t,
                                      (float*)(ns > 0 ? y2 : nullptr), (float*)(ns > 1 ? y3 : nullptr),
                                      (float*)(ns > 2 ? y4 : nullptr), hs)
            : step_stages_impl<double>(s, (const double*)phi, (double*)phi_next, (const double*)u,
                                       (const double*)v, (const double*)w, t,
                                       (double*)(ns > 0 ? y2 : nullptr),
                                       (double*)(ns > 1 ? y3 : nullptr),
                                       (double*)(ns > 2 ? y4 : nullptr), hs);
    return e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_step_stages");
}

extern "C" pf_status phasefield_reduce(pf_solver* s, const void* phi, double out4[4],
                                       void* hip_stream)
{
    if (!s) return fail(PF_ERR_INVALID, "solver is NULL");
    pf_status st = check_field_ptr(phi, "phi");
    if (st != PF_OK) return st;
    if (!out4) return fail(PF_ERR_INVALID, "out4 is NULL");
    hipStream_t hs = (hipStream_t)hip_stream;
    const NuMesh& m = s->nu;
    const int* n = s->p.n;
    hipError_t e;
    if (m.on())
        e = s->p.dtype == PF_F32
                ? launch_reduce_weighted<float>((const float*)phi, n[0], n[1], n[2], m.width[0],
                                                m.width[1], m.width[2], s->red_part, s->red_out, hs)
                : launch_reduce_weighted<double>((const double*)phi, n[0], n[1], n[2], m.width[0],
                                                 m.width[1], m.width[2], s->red_part, s->red_out, hs);
    else
        e = s->p.dtype == PF_F32
                ? launch_reduce<float>((const float*)phi, s->N, s->red_part, s->red_out, hs)
                : launch_reduce<double>((const double*)phi, s->N, s->red_part, s->red_out, hs);
    if (e != hipSuccess) return hip_fail(e, "phasefield_reduce: launch");
    e = hipMemcpyAsync(s->red_host, s->red_out, 4 * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e != hipSuccess) return hip_fail(e, "phasefield_reduce: copy");
    e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_fail(e, "phasefield_reduce: synchronize");
    const int D = active_dims(s->p.n);
    double dV = 1.0;
    for (int d = 0; d < D && !m.on(); ++d) dV *= s->p.dx;  // the weighted sum holds the volumes
    out4[0] = s->red_host[0] * dV;
    out4[1] = s->red_host[1];
    out4[2] = s->red_host[2];
    out4[3] = s->red_host[3];
    if (out4[3] > 0.0) return fail(PF_ERR_NONFINITE, "%.0f non-finite cells", out4[3]);
    return PF_OK;
}

extern "C" pf_status phasefield_device_copy(void* dst, const void* src, size_t bytes,
                                           void* hip_stream)
{
    if (!dst || !src) return fail(PF_ERR_INVALID, "dst or src is NULL");
    if (bytes % 4) return fail(PF_ERR_INVALID, "bytes must be a multiple of 4");
    if (bytes == 0) return PF_OK;
    hipError_t e = launch_copy<float>((float*)dst, (const float*)src, bytes / 4,
                                      (hipStream_t)hip_stream);
    return e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_device_copy");
}

// ------------------------------------------------------------------------------ autotune
template <typename T>
static pf_status autotune_impl(pf_solver* s, int reps, int32_t* best, double* times_ms,
                               hipStream_t st)
{
    const pf_params& p = s->p;
    // private operands: phi and velocity live in adjoint-scratch-sized temporaries
    T *phi = nullptr, *U = nullptr, *V = nullptr, *W = nullptr;
    hipError_t e = hipMalloc((void**)&phi, s->N * sizeof(T));
    if (e == hipSuccess) e = hipMalloc((void**)&U, s->N * sizeof(T));
    if (e == hipSuccess) e = hipMalloc((void**)&V, s->N * sizeof(T));
    if (e == hipSuccess) e = hipMalloc((void**)&W, s->N * sizeof(T));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    pf_status ret = PF_OK;
    if (e == hipSuccess) {
        // a smooth bounded field and a uniform velocity: timing does not depend on the values
        e = launch_fill<T>(phi, (T)0.5, s->N, st);
        if (e == hipSuccess) e = launch_fill<T>(U, (T)0.1, s->N, st);
        if (e == hipSuccess) e = launch_fill<T>(V, (T)0.1, s->N, st);
        if (e == hipSuccess) e = launch_fill<T>(W, (T)0.1, s->N, st);
    }
    double best_t = INFINITY;
    int best_v = s->variant;
    const int nv = stage_variant_count(p.dtype);
    for (int v = 0; v < nv && e == hipSuccess; ++v) {
        e = enqueue_steps<T>(p, v, phi, U, V, W, (T*)s->ya, (T*)s->yb, (T*)s->acc, 0.0, 2, st);
        if (e != hipSuccess) break;
        e = hipEventRecord(ev0, st);
        if (e == hipSuccess)
            e = enqueue_steps<T>(p, v, phi, U, V, W, (T*)s->ya, (T*)s->yb, (T*)s->acc, 0.0,
                                 2 * reps, st);
        if (e == hipSuccess) e = hipEventRecord(ev1, st);
        if (e == hipSuccess) e = hipEventSynchronize(ev1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
        const double per = ms / (2.0 * std::max(reps, 1));
        if (times_ms) times_ms[v] = per;
        if (e == hipSuccess && per < best_t) {
            best_t = per;
            best_v = v;
        }
    }
    if (e != hipSuccess) ret = hip_fail(e, "phasefield_autotune");
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    (void)hipStreamSynchronize(st);
    for (T* b : {phi, U, V, W})
        if (b) (void)hipFree(b);
    if (ret == PF_OK) {
        s->variant = best_v;
        if (wall_mask(p) == 0) store_tuned(p.dtype, p.n, best_v);  // the cache is for periodic grids
        release_graph(s->graph);
        if (best) *best = best_v;
    }
    return ret;
}

extern "C" pf_status phasefield_autotune(pf_solver* s, int32_t reps, int32_t* best,
                                         double* times_ms, void* hip_stream)
{
    if (!s) return fail(PF_ERR_INVALID, "solver is NULL");
    if (reps < 1) return fail(PF_ERR_INVALID, "reps < 1");
    if (s->nu.on())
        return fail(PF_ERR_UNSUPPORTED, "a non-uniform mesh runs one kernel form: nothing to tune");
    hipStream_t hs = (hipStream_t)hip_stream;
    return s->p.dtype == PF_F32 ? autotune_impl<float>(s, reps, best, times_ms, hs)
                                : autotune_impl<double>(s, reps, best, times_ms, hs);
}
