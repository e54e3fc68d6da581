// Internal declarations of the gfx950 phase-field library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

#include "phasefield.h"

namespace pf {

// One explicit stage of the flux-form update (Sec. 2.2 recipe): evaluate f = d(phi)/dt of
// Eq. 1 from the stage input y, then write out1 = base1 + c1 f and out2 = base2 + c2 f
// (either output may be null). base2 and out2 may be the same array (in-place accumulator);
// y is never written by the stage.
template <typename T>
struct StageArgs {
    const T* y;
    const T* base1;
    const T* base2;
    T* out1;
    T* out2;
    const T* U;
    const T* V;
    const T* W;
    int nx, ny, nz;
    // Flux coefficients carry the 1/dx of the divergence, so face fluxes are summed directly.
    T inv_2dx;  // 1 / (2 dx), central gradient
    T ge;       // gamma eps / dx^2, diffusive flux
    T hg;       // gamma / (2 dx), sharpening flux (face mean of q), folded into q
    T nhs;      // -s(t) / (2 dx), advective flux (face mean of phi)
    T delta2;   // delta^2, |grad phi| regulariser
    T c1, c2;
    // Walls (bit 0: x, 1: y, 2: z): on a walled axis the stage input is read through mirror
    // indices (reflectn) and the face velocity stored at index 0 (the wall faces, low and, by
    // periodic storage, high) counts as zero, which makes every flux through a wall face zero.
    int walls;
    // Non-uniform rectilinear mesh (null: the uniform mesh above). Per axis a table of kNuCols
    // values per cell index (see NuCol); the kernel reads it at the wrapped index on a periodic
    // axis and at the mirrored one on a walled axis. The uniform coefficients above are then
    // unused.
    const T* nu[3] = {nullptr, nullptr, nullptr};
    T nu_ge = T(0);   // gamma eps (eps mode 0) or gamma eps / dx (mode 1: times the face's mean
                      // of its two cells' largest widths)
    T nu_hg = T(0);   // gamma / 2, the face mean of q, folded into q
    T nu_nhs = T(0);  // -s(t) / 2, the face mean of phi
    int nu_eps_mode = 0;
};

// Columns of a non-uniform mesh table, per cell index along one axis: 1/h (divergence),
// 1/(distance between the centres of the two neighbours) (central gradient), 1/(distance
// between the centres across the cell's low face) (diffusive flux), h (local eps; 0 on an axis of
// one cell, which the local eps leaves out).
enum NuCol { kNuInvW = 0, kNuInvSpan = 1, kNuInvDist = 2, kNuWidth = 3, kNuCols = 4 };

// Adjoint of one stage: given the cotangent kap of the stage's f (a field), accumulate
//   lam_out = lam_base + a_lam * ybar        (ybar = (df/dy)^T kap at y)
//   kap_out = kap_lam_coef * lamp + a_kap * ybar   (next stage's cotangent), if kap_out
// and gU/gV/gW += (df/dU)^T kap (if non-null). kap is read through kap_scale * kap_in.
template <typename T>
struct AdjArgs {
    const T* y;        // stage input (forward)
    const T* kap_in;   // cotangent source read with a stencil
    T kap_scale;       // kap = kap_scale * kap_in
    const T* lam_base; // lam_out = lam_base + ybar
    T* lam_out;
    const T* lamp;     // lambda' (cotangent of the step output), centre only; may alias lam_out
    T* kap_out;        // = kb * lamp + ka * ybar (nullable)
    T kb, ka;
    T* gU;
    T* gV;
    T* gW;
    const T* U;
    const T* V;
    const T* W;
    int nx, ny, nz;
    T inv_dx, inv_2dx, ge, hg, hs, delta2;
    // Walls (bit 0: x, 1: y, 2: z): the stage input and the cotangent are read through mirror
    // indices on a walled axis. The cotangent of a wall face's flux is then exactly zero, and a
    // mirror ghost's gradient cotangent the exact negative of its partner's along the wall
    // normal, which is what the gather needs for the gradient's mirror read of the cell itself.
    int walls = 0;
    // Non-uniform mesh (nu[0] set; the per-axis coefficient tables of the forward's NU form,
    // NuCol columns per cell index): nu_ge = gamma eps (eps mode 0) or gamma eps / dx (mode 1,
    // eps of a cell ~ its largest width), nu_hg = gamma / 2.
    const T* nu[3] = {nullptr, nullptr, nullptr};
    T nu_ge = 0, nu_hg = 0;
    int nu_eps_mode = 0;
};

// Two reverse RK4 stages in one sweep (adjoint_fused.hip): stage H then stage L.
//   kap_H = kscaleH * srcH (read with a stencil); ybar_H = (df/dy at yH)^T kap_H;
//   kap_L = kaL ybar_H + kbL lamp (on the tile plus a halo, in LDS);  ybar_L at yL;
//   L_out = (base + ybar_H) + ybar_L;  kout = kaO ybar_L + kbO lamp (nullable);
//   lam_copy = lamp (nullable);  gU/gV/gW += both stages' velocity gradients (nullable).
template <typename T>
struct AdjPairArgs {
    const T* yH;
    const T* srcH;
    T kscaleH;
    const T* yL;
    const T* lamp;   // lambda' (read on the tile plus a two-cell halo)
    const T* base;   // at the cell
    T* L_out;
    T* kout;
    T* lam_copy;
    T kaL, kbL, kaO, kbO;
    T* gU;
    T* gV;
    T* gW;
    const T* U;
    const T* V;
    const T* W;
    int nx, ny, nz;
    T inv_dx, inv_2dx, ge, hg, hsH, hsL, delta2;
};

// Two RK4 stages in one sweep (pf_fused_body.h): E1 evaluates f on the stage input y over the
// tile plus a two-cell halo and keeps y_mid = base + c_mid f1 in LDS; E2 evaluates f on y_mid.
//   sweep A: y = phi;  writes out_y = phi + c_y2 f2 and out_acc = (phi + c_acc1 f1) + c_acc2 f2
//            (out_acc may be null: RK2 is sweep A alone, its out_y the new phi)
//   sweep B: y = yb, base of y_mid = phi;  writes out_acc = (acc_in + c_acc1 f1) + c_acc2 f2
template <typename T>
struct FusedArgs {
    const T* y;       // E1 stencil input: phi (sweep A) or yb (sweep B)
    const T* phi;     // phi: base of y_mid and (sweep A) of the outputs
    const T* acc_in;  // sweep B: accumulator after stage 2 (read at the cell only)
    T* out_y;         // sweep A: yb
    T* out_acc;       // sweep A: accumulator (nullable);  sweep B: phi' (may alias acc_in)
    T* out_mid;       // sweep A, nullable: y_mid = phi + c_mid f1 at the tile (the adjoint's y2)
    T* out_phi;       // sweep A, nullable: a copy of phi (so that sweep B can write phi in place)
    const T* U;
    const T* V;
    const T* W;
    int nx, ny, nz;
    T inv_2dx, ge, hg, delta2;  // as in StageArgs
    T nhs1, nhs2;               // -s / (2 dx) at the stage time of E1 and of E2
    T c_mid, c_acc1, c_y2, c_acc2;
    int walls;                  // bit a: axis a walled
};

// An array of nx*ny*nz elements of `es` bytes needs the per-plane buffer descriptors of the
// z-marches (buffer offsets are 32-bit) when it spans 4 GiB or more.
inline bool field_needs_big(int nx, int ny, int nz, size_t es)
{
    return (size_t)nx * (size_t)ny * (size_t)nz * es > 0xffffffffull;
}

// ------------------------------------------------------------------ z-chunks of the marches
// Every tiled kernel (per-stage, fused, adjoint) gives each workgroup a column tile and a chunk of
// consecutive planes, marched in whole groups of six iterations after a warm-up. The chunk
// length is a launch-time choice: the number of chunks c minimises
//   rounds x (6 ceil((kz + 2) / 6) + extra),   kz = ceil(nz / c),
// where a round is one workgroup per resident slot and the second factor is the iterations one
// workgroup runs (extra: warm-up beyond the two planes every march needs, plus start-up; about 5
// for the fused sweeps, 1 for the per-stage and adjoint kernels, as measured on MI355X). Longer
// chunks repeat less warm-up and re-read fewer halo planes; more chunks fill the device. Ties go
// to the longer chunk.
inline int march_chunk_planes(long long tiles, int nz, long long slots, int extra)
{
    int best_kz = nz;
    long long best = -1;
    // far past the chunks that fill the slots, more chunks only add warm-up
    const long long cmax = std::min<long long>(nz, std::max<long long>(64, 4 * ((slots + tiles - 1) / tiles)));
    for (int c = 1; c <= cmax; ++c) {
        const int kz = (nz + c - 1) / c;
        if (c > 1 && kz == (nz + c - 2) / (c - 1)) continue;  // same chunks as c - 1
        const long long rounds = (tiles * ((nz + kz - 1) / kz) + slots - 1) / slots;
        const long long cost = rounds * (6 * ((kz + 7) / 6) + extra);
        if (best < 0 || cost < best) {
            best = cost;
            best_kz = kz;
        }
    }
    return best_kz;
}

// Workgroups of `kernel` (launched with `threads` threads, no dynamic LDS) resident on one compute
// unit, from the HIP occupancy calculator; cached per kernel. 0 on error.
int resident_groups_per_cu(const void* kernel, int threads);
// Chunk length for a launch of `kernel` over `tiles` column tiles of an nz-plane grid on the
// current device (march_chunk_planes with the device's resident slots); 0 on error.
int launch_chunk_planes(const void* kernel, int threads, long long tiles, int nz, int extra);

// ------------------------------------------------------------------ stage-kernel variants
// Either a per-stage kernel (four launches per RK4 step) or a fused pair of sweeps (two
// launches per RK4 step). Every variant produces bit-identical results.
struct StageVariant {
    const char* name;
    hipError_t (*launch_f32)(const StageArgs<float>&, hipStream_t);    // per-stage
    hipError_t (*launch_f64)(const StageArgs<double>&, hipStream_t);
    hipError_t (*fused_f32)(const FusedArgs<float>&, bool sweep_b, hipStream_t);  // fused
    hipError_t (*fused_f64)(const FusedArgs<double>&, bool sweep_b, hipStream_t);
};
// Variants available for a storage dtype, indexed 0..count-1 (per dtype).
int stage_variant_count(int dtype);
const StageVariant& stage_variant(int dtype, int v);
bool variant_is_fused(int dtype, int v);
int default_stage_variant(int nx, int ny, int nz, int dtype);
// The per-stage variant that single stages of a fused solver run on (adjoint recompute, Euler).
int per_stage_variant(int nx, int ny, int nz, int dtype);
// Index of the variant of that name (0 if there is none).
int stage_variant_index(int dtype, const char* name);

// ------------------------------------------------------------------ batched stages (batch.hip)
// Per-instance arguments of one sweep (per-stage mode: StageArgs, fused mode: FusedArgs), and the
// global tile list: one entry {instance, ti, tj, tk} per workgroup, instance < 0 for the padding
// entries that even out the per-XCD ranges (they do nothing).
struct BatchTile {
    int b, ti, tj, tk;
};
template <typename T>
struct BatchCopy {
    const T* src;
    T* dst;
    size_t n;
};
// The list holds 8 equal per-XCD ranges (num_tiles a multiple of 8). persistent: a grid of the
// kernel's resident slots whose workgroups loop over their XCD's range, instead of one workgroup
// per entry.
// walls: some instance has walls (the form that reads through mirror indices where an
// instance's args flag them; periodic instances read as before).
template <typename T>
hipError_t launch_batch_stage(const StageArgs<T>* args_dev, const BatchTile* tiles_dev,
                              int num_tiles, bool persistent, bool walls, hipStream_t st);
// wide: every instance's nx is a multiple of 16 bytes' worth of elements (16-byte plane loads;
// never with walls, whose mirror reads are element-wise)
template <typename T>
hipError_t launch_batch_fused(const FusedArgs<T>* args_dev, bool sweep_b, bool wide,
                              const BatchTile* tiles_dev, int num_tiles, bool persistent,
                              bool walls, int shape, hipStream_t st);
template <typename T>
hipError_t launch_batch_copy(const BatchCopy<T>* table_dev, int count, hipStream_t st);
// Tile shapes of the batched sweeps (the values of phasefield_batch_set_shape).
enum BatchShape { kBatchFused32x16 = 0, kBatchFused64x8 = 1, kBatchStage32x8 = 2, kNumBatchShapes = 3 };
// Tile of a batch shape: x, y extent and z-chunk.
void batch_tile_shape(int shape, int* tx, int* ty, int* kz);

// ------------------------------------------------------------------ adjoint (adjoint.hip)
// Tiled z-march with tile shape `tile` (an index from adjoint_tile_index or
// adjoint_default_tile) and z-chunks of kz planes (0: chosen per launch); big forces the
// large-array addressing form.
template <typename T>
hipError_t launch_adjoint_stage(const AdjArgs<T>& a, int tile, int kz, bool big, hipStream_t st);
int adjoint_tile_index(int tx, int ty);               // -1 if that shape has no adjoint kernel
int adjoint_default_tile(int nx, int ny, int nz);
template <typename T>
hipError_t launch_adjoint_stage_global(const AdjArgs<T>& a, hipStream_t st);  // one thread per cell
template <typename T>
hipError_t launch_adjoint_stage_nu(const AdjArgs<T>& a, hipStream_t st);  // non-uniform mesh
// Two reverse stages per launch (tile 0: 64x8, 1: 32x16; kz 0: chosen per launch). Arrays of
// 4 GiB or more are refused (hipErrorInvalidValue): the caller runs single stages then.
template <typename T>
hipError_t launch_adjoint_pair(const AdjPairArgs<T>& a, int tile, int kz, hipStream_t st);

// ------------------------------------------------------------------ reduction (reduce.hip)
constexpr int kReduceBlocks = 2048;
template <typename T>
hipError_t launch_reduce(const T* phi, size_t n, double* partial /*4*kReduceBlocks*/,
                         double* out4 /*device, 4*/, hipStream_t st);

// The same on a non-uniform mesh: the sum weights cell (i, j, k) by wx[i] wy[j] wz[k] (device).
template <typename T>
hipError_t launch_reduce_weighted(const T* phi, int nx, int ny, int nz, const double* wx,
                                  const double* wy, const double* wz, double* partial,
                                  double* out4, hipStream_t st);

// ------------------------------------------------------------------ velocity (velocity.hip)
// Scratch needs (doubles) for synthesis / projection of an n grid with M modes.
size_t velocity_scratch_doubles(int nx, int ny, int nz, int M);
template <typename T>
hipError_t launch_velocity(int nx, int ny, int nz, double dx, int M, const double* phases,
                           const double* coeffs, T* U, T* V, T* W, double* scratch,
                           hipStream_t st);
template <typename T>
hipError_t launch_velocity_grad(int nx, int ny, int nz, double dx, int M, const double* phases,
                                const T* gU, const T* gV, const T* gW, double* coeff_grad,
                                double* scratch, hipStream_t st);

// ------------------------------------------------------------------ small utilities
int device_compute_units();  // of the current device; 0 on error (cached per device)
template <typename T>
hipError_t launch_copy(T* dst, const T* src, size_t n, hipStream_t st);

// One stage on a non-uniform mesh (a.nu set): stage_tiled.hip.
template <typename T>
hipError_t launch_stage_nu(const StageArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_fill(T* dst, T value, size_t n, hipStream_t st);

}  // namespace pf
