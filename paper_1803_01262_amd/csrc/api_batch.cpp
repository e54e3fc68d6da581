// C ABI: batched driver. Every instance of the batch advances together: each sweep is ONE
// launch over a global tile list that covers all instances (one workgroup per tile), and the
// step sequence is captured once into a HIP graph and replayed.
//
// Two modes. The kind of the variant that instance 0 names (variant >= 0) selects one; with
// variant -1 FP32 runs fused and FP64 per-stage:
//   fused:     two-stage sweeps (two launches per step). phi alternates with the accumulator
//              buffer from step to step; tables for even and odd steps are kept, and after an
//              odd step count one batched copy returns phi to the caller's buffers.
//   per-stage: one launch per RK stage (RK4 four, RK3 three, RK2 two, Euler one and a batched
//              copy of the accumulator into phi), fixed buffers; the only mode of the schemes
//              other than RK4 (the fused sweeps pair RK4's stages).
// Every instance of a batch runs the same scheme. Either way every instance is bit-identical to
// its own single solve. The tile shape (fused
// 32x16 or 64x8, per-stage 32x8) and the launch form can be set, or chosen by timing them all
// (phasefield_batch_autotune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "pf_api_internal.h"

using namespace pf;

struct pf_batch {
    int count = 0;
    int dtype = PF_F64;
    int scheme = PF_RK4;  // every instance's
    bool fused = false;
    std::vector<pf_params> p;
    std::vector<size_t> N;
    void* pool = nullptr;          // stage buffers of every instance (ya, yb, acc each)
    std::vector<size_t> pool_off;  // element offset of instance b's first buffer
    int num_tiles = 0;
    bool persistent = false;  // launch form: resident-slot grid looping over the list
    bool wide = false;  // every instance's nx allows 16-byte plane loads
    bool walls = false;  // some instance has walls
    int shape = kBatchStage32x8;  // BatchShape of the tile list
    BatchTile* tiles = nullptr;  // device: the global tile list (8 equal per-XCD ranges)
    // device per-instance argument arrays: per-stage mode S1..S4 (StageArgs; RK3 S1..S3, RK2
    // S1..S2, Euler S1);
    // fused mode A_even, B_even, A_odd, B_odd (FusedArgs)
    void* tables[4] = {nullptr, nullptr, nullptr, nullptr};
    void* copies = nullptr;        // device BatchCopy<T>[count]: acc -> phi after an odd count
    std::vector<const void*> key;  // pointer set the tables and graph were built for
    hipStream_t key_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void batch_release_graph(pf_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

extern "C" pf_status phasefield_batch_destroy(pf_batch* b)
{
    if (!b) return PF_OK;
    (void)hipDeviceSynchronize();
    batch_release_graph(b);
    if (b->pool) (void)hipFree(b->pool);
    if (b->tiles) (void)hipFree(b->tiles);
    if (b->copies) (void)hipFree(b->copies);
    for (void* t : b->tables)
        if (t) (void)hipFree(t);
    delete b;
    return PF_OK;
}

static size_t padded(size_t n) { return (n + 63) / 64 * 64; }  // keeps buffers 256-byte aligned

// Whether the fused shapes apply: RK4 (the fused sweeps pair RK4's stages); 0 if they do, else
// the first instance that stops them.
static int B_stage_only(const pf_params* per_instance, int count)
{
    for (int b = 0; b < count; ++b)
        if (per_instance[b].scheme != PF_RK4) return b + 1;
    return 0;
}

// Mode: the kind (fused or per-stage) of the variant named by instance 0, else by dtype.
// Per-stage whenever the fused shapes do not apply (B_stage_only).
static bool B_mode_fused(const pf_params* per_instance, int count)
{
    if (B_stage_only(per_instance, count)) return false;
    const int dtype = per_instance[0].dtype, v0 = per_instance[0].variant;
    if (v0 >= 0 && v0 < stage_variant_count(dtype)) return variant_is_fused(dtype, v0);
    return dtype == PF_F32;
}

// The global tile list. Instances are packed onto the 8 XCDs by longest processing time (largest
// first, each onto the least-loaded XCD), so the tiles of one instance share one L2; within an
// XCD's range the tiles run longest z-chunk first, so short tiles fill the end; the ranges are
// padded to one length with empty entries (the launch maps workgroup ids onto the ranges).
static bool build_tile_list(const pf_params* p, int count, int shape, std::vector<BatchTile>& out)
{
    int TX, TY, KZ;
    batch_tile_shape(shape, &TX, &TY, &KZ);
    const int warm = shape != kBatchStage32x8 ? 6 : 2;  // warm-up planes per z-chunk
    std::vector<double> work(count);
    std::vector<int> order(count);
    for (int b = 0; b < count; ++b) {
        const double tx = (p[b].n[0] + TX - 1) / TX, ty = (p[b].n[1] + TY - 1) / TY;
        const double cz = (p[b].n[2] + KZ - 1) / KZ;
        work[b] = tx * ty * ((double)p[b].n[2] + cz * warm);
        order[b] = b;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    constexpr int kXcd = 8;
    std::vector<BatchTile> bins[kXcd];
    double load[kXcd] = {0};
    for (int b : order) {
        const int x = (int)(std::min_element(load, load + kXcd) - load);
        load[x] += work[b];
        const int tx = (p[b].n[0] + TX - 1) / TX, ty = (p[b].n[1] + TY - 1) / TY;
        const int cz = (p[b].n[2] + KZ - 1) / KZ;
        for (int k = 0; k < cz; ++k)
            for (int j = 0; j < ty; ++j)
                for (int i = 0; i < tx; ++i) bins[x].push_back({b, i, j, k});
    }
    size_t len = 0;
    for (auto& bin : bins) {
        std::stable_sort(bin.begin(), bin.end(), [&](const BatchTile& u, const BatchTile& v) {
            return std::min(KZ, p[u.b].n[2] - u.tk * KZ) > std::min(KZ, p[v.b].n[2] - v.tk * KZ);
        });
        len = std::max(len, bin.size());
    }
    if (len * kXcd > 0x7fffffffull) return false;
    out.assign(len * kXcd, BatchTile{-1, 0, 0, 0});
    for (int x = 0; x < kXcd; ++x) std::copy(bins[x].begin(), bins[x].end(), out.begin() + x * len);
    return true;
}

extern "C" pf_status phasefield_batch_create(const pf_params* per_instance, int32_t count,
                                             pf_batch** out)
{
    if (!out) return fail(PF_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (count < 1 || !per_instance) return fail(PF_ERR_INVALID, "count < 1 or params NULL");
    for (int b = 0; b < count; ++b) {
        pf_status st = validate_params(&per_instance[b]);
        if (st != PF_OK) return fail(st, "instance %d: %s", b, phasefield_last_error());
        if (per_instance[b].dtype != per_instance[0].dtype)
            return fail(PF_ERR_INVALID, "instance %d: mixed dtypes", b);
        if (per_instance[b].scheme != per_instance[0].scheme)
            return fail(PF_ERR_UNSUPPORTED, "instance %d: mixed schemes in one batch", b);
        if (per_instance[b].vel_mode != PF_VEL_STEADY)
            return fail(PF_ERR_UNSUPPORTED, "instance %d: the batched driver needs a steady velocity", b);
        const pf_params& q = per_instance[b];
        if (field_needs_big(q.n[0], q.n[1], q.n[2], q.dtype == PF_F32 ? 4 : 8))
            return fail(PF_ERR_UNSUPPORTED,
                        "instance %d: a field of 4 GiB or more; use a single-grid solver", b);
    }
    std::vector<BatchTile> list;
    const int shape = B_mode_fused(per_instance, count) ? kBatchFused32x16 : kBatchStage32x8;
    if (!build_tile_list(per_instance, count, shape, list))
        return fail(PF_ERR_INVALID, "the batch has too many tiles for one launch");
    auto* B = new pf_batch();
    B->count = count;
    B->dtype = per_instance[0].dtype;
    B->scheme = per_instance[0].scheme;
    B->shape = shape;
    B->fused = shape != kBatchStage32x8;
    B->p.assign(per_instance, per_instance + count);
    const size_t esz = B->dtype == PF_F32 ? sizeof(float) : sizeof(double);
    size_t total = 0;
    for (int b = 0; b < count; ++b) {
        const size_t n = (size_t)B->p[b].n[0] * B->p[b].n[1] * B->p[b].n[2];
        B->N.push_back(n);
        B->pool_off.push_back(total);
        total += 3 * padded(n);
    }
    B->num_tiles = (int)list.size();
    B->walls = false;
    for (int b = 0; b < count; ++b) B->walls = B->walls || wall_mask(B->p[b]) != 0;
    B->wide = !B->walls;  // mirror reads are element-wise
    for (int b = 0; b < count; ++b)
        B->wide = B->wide && B->p[b].n[0] % (int)(16 / esz) == 0;
    hipError_t e = hipMalloc(&B->pool, total * esz);
    if (e == hipSuccess) e = hipMalloc((void**)&B->tiles, list.size() * sizeof(BatchTile));
    if (e == hipSuccess)
        e = hipMemcpy(B->tiles, list.data(), list.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
    // room for either mode's per-instance arguments (the shape can change later)
    const size_t tsz = B->dtype == PF_F32
                           ? std::max(sizeof(FusedArgs<float>), sizeof(StageArgs<float>))
                           : std::max(sizeof(FusedArgs<double>), sizeof(StageArgs<double>));
    for (int s = 0; s < 4 && e == hipSuccess; ++s) e = hipMalloc(&B->tables[s], tsz * count);
    if (e == hipSuccess)
        e = hipMalloc(&B->copies, (B->dtype == PF_F32 ? sizeof(BatchCopy<float>) : sizeof(BatchCopy<double>)) * count);
    if (e != hipSuccess) {
        phasefield_batch_destroy(B);
        return hip_fail(e, "phasefield_batch_create: allocation");
    }
    *out = B;
    return PF_OK;
}

// Stage launches per step in per-stage mode.
static int batch_stage_count(int scheme)
{
    return scheme == PF_RK4 ? 4 : scheme == PF_RK3 ? 3 : scheme == PF_RK2 ? 2 : 1;
}

// Build the device tables for one pointer set. Per-stage mode, the single-grid step's stages:
//   RK4:   S1 ya = phi + dt/2 k1, acc = phi + dt/6 k1;  S2 yb = phi + dt/2 k2, acc += dt/3 k2;
//          S3 ya = phi + dt k3, acc += dt/3 k3;        S4 phi = acc + dt/6 k4.
//   RK3:   S1 ya = phi + dt g1 k1, acc = phi + dt (g1 + z2) k1;  S2 yb = acc + dt g2 k2;
//          S3 phi = acc + dt g3 k3.
//   RK2:   S1 ya = phi + dt/2 k1;  S2 phi = phi + dt k2.
//   Euler: S1 acc = phi + dt k1, then the batched copy acc -> phi.
//   fused:     even steps run from phi into acc, odd steps from acc back into phi.
template <typename T>
static pf_status upload_tables(pf_batch* B, void* const* phi, const void* const* u,
                               const void* const* v, const void* const* w)
{
    std::vector<StageArgs<T>> st_tab[4];
    std::vector<FusedArgs<T>> fu_tab[4];
    std::vector<BatchCopy<T>> copies;
    for (int b = 0; b < B->count; ++b) {
        const pf_params& p = B->p[b];
        T* ph = (T*)phi[b];
        const T *U = (const T*)u[b], *V = (const T*)v[b], *W = (const T*)w[b];
        T* base = (T*)B->pool + B->pool_off[b];
        const size_t stride = padded(B->N[b]);
        T *ya = base, *yb = base + stride, *acc = base + 2 * stride;
        if (B->fused) {
            const FusedArgs<T> f[4] = {make_fused<T>(p, false, 0.0, ph, acc, U, V, W, yb),
                                       make_fused<T>(p, true, 0.0, ph, acc, U, V, W, yb),
                                       make_fused<T>(p, false, 0.0, acc, ph, U, V, W, yb),
                                       make_fused<T>(p, true, 0.0, acc, ph, U, V, W, yb)};
            for (int s = 0; s < 4; ++s) fu_tab[s].push_back(f[s]);
        } else {
            const double dt = p.dt;
            constexpr double g1 = 8.0 / 15.0, g2 = 5.0 / 12.0, g3 = 0.75, z2 = -17.0 / 60.0;
            StageArgs<T> sa[4] = {};
            if (p.scheme == PF_RK4) {
                sa[0] = make_stage<T>(p, 1.0, ph, ph, ph, ya, acc, 0.5 * dt, dt / 6.0, U, V, W);
                sa[1] = make_stage<T>(p, 1.0, ya, ph, acc, yb, acc, 0.5 * dt, dt / 3.0, U, V, W);
                sa[2] = make_stage<T>(p, 1.0, yb, ph, acc, ya, acc, dt, dt / 3.0, U, V, W);
                sa[3] = make_stage<T>(p, 1.0, ya, nullptr, acc, nullptr, ph, 0.0, dt / 6.0, U, V, W);
            } else if (p.scheme == PF_RK3) {
                sa[0] = make_stage<T>(p, 1.0, ph, ph, ph, ya, acc, dt * g1, dt * (g1 + z2), U, V, W);
                sa[1] = make_stage<T>(p, 1.0, ya, acc, nullptr, yb, nullptr, dt * g2, 0.0, U, V, W);
                sa[2] = make_stage<T>(p, 1.0, yb, nullptr, acc, nullptr, ph, 0.0, dt * g3, U, V, W);
            } else if (p.scheme == PF_RK2) {
                sa[0] = make_stage<T>(p, 1.0, ph, ph, nullptr, ya, nullptr, 0.5 * dt, 0.0, U, V, W);
                sa[1] = make_stage<T>(p, 1.0, ya, nullptr, ph, nullptr, ph, 0.0, dt, U, V, W);
            } else {
                sa[0] = make_stage<T>(p, 1.0, ph, nullptr, ph, nullptr, acc, 0.0, dt, U, V, W);
            }
            for (int s = 0; s < batch_stage_count(p.scheme); ++s) st_tab[s].push_back(sa[s]);
        }
        copies.push_back({acc, ph, B->N[b]});
    }
    for (int s = 0; s < (B->fused ? 4 : batch_stage_count(B->scheme)); ++s) {
        hipError_t e = B->fused ? hipMemcpy(B->tables[s], fu_tab[s].data(),
                                            sizeof(FusedArgs<T>) * B->count, hipMemcpyHostToDevice)
                                : hipMemcpy(B->tables[s], st_tab[s].data(),
                                            sizeof(StageArgs<T>) * B->count, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "phasefield_batch_step: table upload");
    }
    hipError_t e = hipMemcpy(B->copies, copies.data(), sizeof(BatchCopy<T>) * B->count,
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "phasefield_batch_step: table upload");
    return PF_OK;
}

// One step; `odd` selects the fused tables of an odd step within a call.
template <typename T>
static hipError_t enqueue_batch_step(pf_batch* B, bool odd, hipStream_t st)
{
    if (B->fused) {
        for (int s = 0; s < 2; ++s) {
            hipError_t e = launch_batch_fused<T>((const FusedArgs<T>*)B->tables[(odd ? 2 : 0) + s],
                                                 s == 1, B->wide, B->tiles, B->num_tiles,
                                                 B->persistent, B->walls, B->shape, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    for (int s = 0; s < batch_stage_count(B->scheme); ++s) {
        hipError_t e = launch_batch_stage<T>((const StageArgs<T>*)B->tables[s], B->tiles,
                                             B->num_tiles, B->persistent, B->walls, st);
        if (e != hipSuccess) return e;
    }
    if (B->scheme == PF_EULER)  // the step's new phi is in the accumulator
        return launch_batch_copy<T>((const BatchCopy<T>*)B->copies, B->count, st);
    return hipSuccess;
}

template <typename T>
static pf_status batch_step_impl(pf_batch* B, void* const* phi, const void* const* u,
                                 const void* const* v, const void* const* w, int32_t nsteps,
                                 hipStream_t st)
{
    std::vector<const void*> key;
    for (int b = 0; b < B->count; ++b) {
        key.push_back(phi[b]);
        key.push_back(u[b]);
        key.push_back(v[b]);
        key.push_back(w[b]);
    }
    if (key != B->key) {
        // tables may be in use by queued work on the previous stream
        hipError_t e = B->key_stream ? hipStreamSynchronize(B->key_stream) : hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "phasefield_batch_step: synchronize");
        pf_status ps = upload_tables<T>(B, phi, u, v, w);
        if (ps != PF_OK) return ps;
        batch_release_graph(B);
        B->key = key;
    }
    int32_t done = 0;
    // the captured sequence has an even number of steps, so phi is back in place after each replay
    if (st != nullptr && nsteps >= kGraphSteps) {
        if (!B->exec || B->key_stream != st) {
            batch_release_graph(B);
            hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "phasefield_batch_step: begin capture");
            hipError_t le = hipSuccess;
            for (int m = 0; m < kGraphSteps && le == hipSuccess; ++m)
                le = enqueue_batch_step<T>(B, (m & 1) != 0, st);
            e = hipStreamEndCapture(st, &B->graph);
            if (le != hipSuccess) return hip_fail(le, "phasefield_batch_step: launch during capture");
            if (e != hipSuccess) return hip_fail(e, "phasefield_batch_step: end capture");
            e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return hip_fail(e, "phasefield_batch_step: instantiate");
        }
        for (; done + kGraphSteps <= nsteps; done += kGraphSteps) {
            hipError_t e = hipGraphLaunch(B->exec, st);
            if (e != hipSuccess) return hip_fail(e, "phasefield_batch_step: graph launch");
        }
    }
    B->key_stream = st;
    const int32_t rest = nsteps - done;
    for (int32_t m = 0; m < rest; ++m) {
        hipError_t e = enqueue_batch_step<T>(B, (m & 1) != 0, st);
        if (e != hipSuccess) return hip_fail(e, "phasefield_batch_step: launch");
    }
    if (B->fused && (rest & 1)) {
        hipError_t e = launch_batch_copy<T>((const BatchCopy<T>*)B->copies, B->count, st);
        if (e != hipSuccess) return hip_fail(e, "phasefield_batch_step: copy back");
    }
    return PF_OK;
}

extern "C" pf_status phasefield_batch_set_persistent(pf_batch* b, int32_t persistent)
{
    if (!b) return fail(PF_ERR_INVALID, "batch is NULL");
    if (b->persistent != (persistent != 0)) {
        // queued replays of the old graph may still run; the new form is captured on next use
        hipError_t e = b->key_stream ? hipStreamSynchronize(b->key_stream) : hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "phasefield_batch_set_persistent: synchronize");
        batch_release_graph(b);
        b->persistent = persistent != 0;
    }
    return PF_OK;
}

extern "C" pf_status phasefield_batch_step(pf_batch* b, void* const* phi, const void* const* u,
                                           const void* const* v, const void* const* w,
                                           const double* t0, int32_t nsteps, void* hip_stream)
{
    (void)t0;  // steady velocity: the step does not depend on the start time
    if (!b) return fail(PF_ERR_INVALID, "batch is NULL");
    if (!phi || !u || !v || !w) return fail(PF_ERR_INVALID, "pointer array is NULL");
    if (nsteps < 0) return fail(PF_ERR_INVALID, "nsteps < 0");
    for (int i = 0; i < b->count; ++i) {
        pf_status st;
        if ((st = check_field_ptr(phi[i], "phi[b]")) != PF_OK) return st;
        if ((st = check_field_ptr(u[i], "u[b]")) != PF_OK) return st;
        if ((st = check_field_ptr(v[i], "v[b]")) != PF_OK) return st;
        if ((st = check_field_ptr(w[i], "w[b]")) != PF_OK) return st;
    }
    if (nsteps == 0) return PF_OK;
    hipStream_t hs = (hipStream_t)hip_stream;
    return b->dtype == PF_F32 ? batch_step_impl<float>(b, phi, u, v, w, nsteps, hs)
                              : batch_step_impl<double>(b, phi, u, v, w, nsteps, hs);
}

// Rebuild the tile list for another shape. Queued work on the batch's last stream may still read
// the old list and tables, so that stream is synchronised first; the next step re-uploads the
// tables and re-captures the graph.
static pf_status batch_apply_shape(pf_batch* b, int shape)
{
    if (shape == b->shape) return PF_OK;
    std::vector<BatchTile> list;
    if (!build_tile_list(b->p.data(), b->count, shape, list))
        return fail(PF_ERR_INVALID, "the batch has too many tiles for one launch");
    hipError_t e = b->key_stream ? hipStreamSynchronize(b->key_stream) : hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "phasefield_batch_set_shape: synchronize");
    batch_release_graph(b);
    BatchTile* tiles = nullptr;
    e = hipMalloc((void**)&tiles, list.size() * sizeof(BatchTile));
    if (e == hipSuccess)
        e = hipMemcpy(tiles, list.data(), list.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (tiles) (void)hipFree(tiles);
        return e == hipErrorOutOfMemory ? fail(PF_ERR_OOM, "phasefield_batch_set_shape: out of memory")
                                        : hip_fail(e, "phasefield_batch_set_shape: tile list");
    }
    if (b->tiles) (void)hipFree(b->tiles);
    b->tiles = tiles;
    b->num_tiles = (int)list.size();
    b->shape = shape;
    b->fused = shape != kBatchStage32x8;
    b->key.clear();  // the tables of the new mode are uploaded by the next step
    return PF_OK;
}

extern "C" pf_status phasefield_batch_set_shape(pf_batch* b, int32_t shape)
{
    if (!b) return fail(PF_ERR_INVALID, "batch is NULL");
    if (shape < 0 || shape >= kNumBatchShapes)
        return fail(PF_ERR_INVALID, "batch shape %d is not 0, 1 or 2", (int)shape);
    if (shape != kBatchStage32x8) {
        const int i = B_stage_only(b->p.data(), b->count) - 1;
        if (i >= 0)
            return fail(PF_ERR_UNSUPPORTED,
                        "instance %d runs a scheme other than RK4: per-stage shape only", i);
    }
    return batch_apply_shape(b, shape);
}

template <typename T>
static pf_status batch_autotune_impl(pf_batch* B, int reps, int32_t* best_shape,
                                     int32_t* best_persistent, double* times_ms, hipStream_t st)
{
    // private operands for every instance: a smooth bounded field and a uniform velocity (the
    // timing does not depend on the values)
    size_t total = 0;
    for (int b = 0; b < B->count; ++b) total += 4 * padded(B->N[b]);
    T* pool = nullptr;
    hipError_t e = hipMalloc((void**)&pool, total * sizeof(T));
    if (e != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(PF_ERR_OOM, "phasefield_batch_autotune: out of memory")
                                        : hip_fail(e, "phasefield_batch_autotune: allocation");
    std::vector<void*> phi(B->count);
    std::vector<const void*> u(B->count), v(B->count), w(B->count);
    size_t off = 0;
    for (int b = 0; b < B->count && e == hipSuccess; ++b) {
        const size_t n = B->N[b], pn = padded(n);
        T* base = pool + off;
        off += 4 * pn;
        phi[b] = base;
        u[b] = base + pn;
        v[b] = base + 2 * pn;
        w[b] = base + 3 * pn;
        e = launch_fill<T>(base, (T)0.5, n, st);
        for (int k = 1; k < 4 && e == hipSuccess; ++k) e = launch_fill<T>(base + k * pn, (T)0.1, n, st);
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    pf_status ret = e == hipSuccess ? PF_OK : hip_fail(e, "phasefield_batch_autotune: set-up");
    const int start_shape = B->shape;
    const bool start_persistent = B->persistent;
    double best_t = INFINITY;
    int bs = start_shape, bp = start_persistent ? 1 : 0;
    const bool stage_only = B_stage_only(B->p.data(), B->count) != 0;
    const int steps = kGraphSteps * std::max(reps, 1);
    for (int shape = 0; shape < kNumBatchShapes && ret == PF_OK; ++shape) {
        for (int pers = 0; pers < 2 && ret == PF_OK; ++pers) {
            const int slot = 2 * shape + pers;
            if (times_ms) times_ms[slot] = -1.0;
            if (stage_only && shape != kBatchStage32x8) continue;  // fused shapes do not apply
            ret = batch_apply_shape(B, shape);
            if (ret != PF_OK) break;
            if (B->persistent != (pers != 0)) {
                batch_release_graph(B);
                B->persistent = pers != 0;
            }
            // one graph-length run first: table upload and capture stay out of the timing
            ret = batch_step_impl<T>(B, phi.data(), u.data(), v.data(), w.data(), kGraphSteps, st);
            if (ret != PF_OK) break;
            e = hipEventRecord(ev0, st);
            if (e == hipSuccess) {
                ret = batch_step_impl<T>(B, phi.data(), u.data(), v.data(), w.data(), steps, st);
                if (ret != PF_OK) break;
                e = hipEventRecord(ev1, st);
            }
            if (e == hipSuccess) e = hipEventSynchronize(ev1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
            if (e != hipSuccess) {
                ret = hip_fail(e, "phasefield_batch_autotune: timing");
                break;
            }
            const double per = ms / steps;
            if (times_ms) times_ms[slot] = per;
            if (per < best_t) {
                best_t = per;
                bs = shape;
                bp = pers;
            }
        }
    }
    (void)hipStreamSynchronize(st);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    // the private pointers must not be mistaken for a caller's set later
    batch_release_graph(B);
    B->key.clear();
    (void)hipFree(pool);
    if (ret != PF_OK) {
        (void)batch_apply_shape(B, start_shape);
        B->persistent = start_persistent;
        return ret;
    }
    ret = batch_apply_shape(B, bs);
    if (ret != PF_OK) return ret;
    B->persistent = bp != 0;
    if (best_shape) *best_shape = bs;
    if (best_persistent) *best_persistent = bp;
    return PF_OK;
}

extern "C" pf_status phasefield_batch_autotune(pf_batch* b, int32_t reps, int32_t* best_shape,
                                               int32_t* best_persistent, double* times_ms,
                                               void* hip_stream)
{
    if (!b) return fail(PF_ERR_INVALID, "batch is NULL");
    if (reps < 1) return fail(PF_ERR_INVALID, "reps < 1");
    hipStream_t hs = (hipStream_t)hip_stream;
    if (!hs) return fail(PF_ERR_INVALID, "the batch autotuner needs a stream (graphs are captured)");
    return b->dtype == PF_F32 ? batch_autotune_impl<float>(b, reps, best_shape, best_persistent, times_ms, hs)
                              : batch_autotune_impl<double>(b, reps, best_shape, best_persistent, times_ms, hs);
}
