// Batched sweeps: one launch advances one RK stage (per-stage mode) or one two-stage sweep
// (fused mode) of many independent simulations. The tiles of all instances form one global list,
// one workgroup per entry, and each runs the same per-tile body as the single-grid kernels, so
// every instance's result is bit-identical to its own single solve.
#include "pf_fused_body.h"
#include "pf_tiled_body.h"

namespace pf {

// Tile shapes (BatchShape): fused 32x16 (instances down to 32 cells wide), fused 64x8 (fewer
// halo columns where rows are whole multiples of 64), per-stage 32x8; 64-plane z-chunks (little
// warm-up per chunk; 96 and 128 planes measured no faster).
constexpr int kBTX = 32, kBTY = 8, kBKZ = 64;   // per-stage tile
constexpr int kFKZ = 64;                        // fused tiles' z-chunk

// Workgroup -> tile-list entry: the list holds 8 equal ranges of `len` entries, one per XCD.
// One workgroup per entry: xcd_tile_order lets each XCD walk its own range in order.
// Persistent form (PERSIST, a grid of G workgroups, G a multiple of 8 and at most the resident
// slots): workgroup w stays on XCD w mod 8 and takes entries r, r + G/8, r + 2G/8, ... of that
// XCD's range (r = w / 8), in the range's longest-first order; every workgroup leaves the loop
// when it runs past the range end.
template <bool PERSIST, typename Body>
__device__ __forceinline__ void for_batch_tiles(const BatchTile* __restrict__ tiles, int len,
                                                Body body)
{
    if constexpr (!PERSIST) {
        const BatchTile tl = tiles[xcd_tile_order(blockIdx.x, gridDim.x)];
        if (tl.b >= 0) body(tl);
    } else {
        const int x = blockIdx.x & 7, r = blockIdx.x >> 3, step = gridDim.x >> 3;
        for (int e = r; e < len; e += step) {
            __syncthreads();  // the previous tile's LDS reads have completed
            const BatchTile tl = tiles[x * len + e];
            if (tl.b >= 0) body(tl);
        }
    }
}

template <typename T, bool PERSIST, bool WALLS>
__global__ void __launch_bounds__(kBTX* kBTY) batch_stage_kernel(const StageArgs<T>* __restrict__ args,
                                                                  const BatchTile* __restrict__ tiles,
                                                                  int len)
{
    for_batch_tiles<PERSIST>(tiles, len, [&](const BatchTile& tl) {
        const int k0 = tl.tk * kBKZ;
        // 64-plane chunks: the form that loads per-cell operands one iteration ahead (1.6-1.8 %
        // faster)
        tiled_stage_body<T, kBTX, kBTY, false, WALLS, true>(args[tl.b], tl.ti, tl.tj, k0,
                                                            min(k0 + kBKZ, args[tl.b].nz));
    });
}

// Fused mode: one launch per two-stage sweep, with the register budget of the single-grid fused
// kernel (FP32: four waves per SIMD).
// WIDE: every instance's rows are a whole number of 16-byte pieces (16-byte plane loads).
// WALLS: walls in some instance, on any axes (element-wise loads, WIDE off).
template <typename T, int TX, int TY, bool SWEEP_B, bool WIDE, bool PERSIST, bool WALLS = false>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
batch_fused_kernel(const FusedArgs<T>* __restrict__ args, const BatchTile* __restrict__ tiles, int len)
{
    for_batch_tiles<PERSIST>(tiles, len, [&](const BatchTile& tl) {
        const int k0 = tl.tk * kFKZ;
        fused_body<T, TX, TY, SWEEP_B, false, WIDE, false, WALLS, fused_lag<T, TX, TY>()>(
            args[tl.b], tl.ti, tl.tj, k0, min(k0 + kFKZ, args[tl.b].nz));
    });
}

// dst[b] = src[b] for every instance b (blockIdx.y), grid-stride within the instance.
template <typename T>
__global__ void batch_copy_kernel(const BatchCopy<T>* __restrict__ e)
{
    const BatchCopy<T> c = e[blockIdx.y];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < c.n; i += (size_t)gridDim.x * blockDim.x)
        c.dst[i] = c.src[i];
}

void batch_tile_shape(int shape, int* tx, int* ty, int* kz)
{
    *tx = shape == kBatchFused64x8 ? 64 : 32;
    *ty = shape == kBatchFused32x16 ? 16 : 8;
    *kz = shape == kBatchStage32x8 ? kBKZ : kFKZ;
}

// Grid of the persistent form: the resident slots of the kernel (compute units x workgroups per
// compute unit), rounded down to a multiple of 8 and capped at the list length; 0 on error.
static int persistent_grid(const void* kernel, int threads, int num_tiles)
{
    const int cus = device_compute_units();
    const int groups = resident_groups_per_cu(kernel, threads);
    if (cus <= 0 || groups <= 0) return 0;
    int g = (cus * groups) / 8 * 8;
    return g > num_tiles ? num_tiles : g;
}

template <typename T, int TX, int TY, bool SWEEP_B, bool WIDE, bool WALLS = false>
static hipError_t launch_batch_fused_form(const FusedArgs<T>* args_dev, const BatchTile* tiles_dev,
                                          int num_tiles, bool persistent, hipStream_t st)
{
    const int len = num_tiles / 8;
    if (persistent) {
        const void* k = (const void*)batch_fused_kernel<T, TX, TY, SWEEP_B, WIDE, true, WALLS>;
        const int g = persistent_grid(k, TX * TY, num_tiles);
        if (g < 8) return hipErrorInvalidDevice;
        hipLaunchKernelGGL((batch_fused_kernel<T, TX, TY, SWEEP_B, WIDE, true, WALLS>), dim3(g),
                           dim3(TX * TY), 0, st, args_dev, tiles_dev, len);
    } else {
        hipLaunchKernelGGL((batch_fused_kernel<T, TX, TY, SWEEP_B, WIDE, false, WALLS>),
                           dim3(num_tiles), dim3(TX * TY), 0, st, args_dev, tiles_dev, len);
    }
    return hipGetLastError();
}

template <typename T, int TX, int TY>
static hipError_t launch_batch_fused_shape(const FusedArgs<T>* args_dev, bool sweep_b, bool wide,
                                           const BatchTile* tiles_dev, int num_tiles,
                                           bool persistent, bool walls, hipStream_t st)
{
    if (walls) {
        if (wide) return hipErrorInvalidValue;
        return sweep_b ? launch_batch_fused_form<T, TX, TY, true, false, true>(args_dev, tiles_dev, num_tiles, persistent, st)
                       : launch_batch_fused_form<T, TX, TY, false, false, true>(args_dev, tiles_dev, num_tiles, persistent, st);
    }
    if (wide)
        return sweep_b ? launch_batch_fused_form<T, TX, TY, true, true>(args_dev, tiles_dev, num_tiles, persistent, st)
                       : launch_batch_fused_form<T, TX, TY, false, true>(args_dev, tiles_dev, num_tiles, persistent, st);
    return sweep_b ? launch_batch_fused_form<T, TX, TY, true, false>(args_dev, tiles_dev, num_tiles, persistent, st)
                   : launch_batch_fused_form<T, TX, TY, false, false>(args_dev, tiles_dev, num_tiles, persistent, st);
}

template <typename T>
hipError_t launch_batch_fused(const FusedArgs<T>* args_dev, bool sweep_b, bool wide,
                              const BatchTile* tiles_dev, int num_tiles, bool persistent,
                              bool walls, int shape, hipStream_t st)
{
    if (num_tiles <= 0 || num_tiles % 8) return hipErrorInvalidValue;
    if (shape == kBatchFused32x16)
        return launch_batch_fused_shape<T, 32, 16>(args_dev, sweep_b, wide, tiles_dev, num_tiles,
                                                   persistent, walls, st);
    if (shape == kBatchFused64x8)
        return launch_batch_fused_shape<T, 64, 8>(args_dev, sweep_b, wide, tiles_dev, num_tiles,
                                                  persistent, walls, st);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_batch_copy(const BatchCopy<T>* table_dev, int count, hipStream_t st)
{
    hipLaunchKernelGGL(batch_copy_kernel<T>, dim3(256, count), dim3(256), 0, st, table_dev);
    return hipGetLastError();
}

template hipError_t launch_batch_fused<float>(const FusedArgs<float>*, bool, bool, const BatchTile*, int, bool, bool, int, hipStream_t);
template hipError_t launch_batch_fused<double>(const FusedArgs<double>*, bool, bool, const BatchTile*, int, bool, bool, int, hipStream_t);
template hipError_t launch_batch_copy<float>(const BatchCopy<float>*, int, hipStream_t);
template hipError_t launch_batch_copy<double>(const BatchCopy<double>*, int, hipStream_t);

template <typename T, bool WALLS>
static hipError_t launch_batch_stage_form(const StageArgs<T>* args_dev, const BatchTile* tiles_dev,
                                          int num_tiles, bool persistent, hipStream_t st)
{
    const int len = num_tiles / 8;
    if (persistent) {
        const int g = persistent_grid((const void*)batch_stage_kernel<T, true, WALLS>, kBTX * kBTY,
                                      num_tiles);
        if (g < 8) return hipErrorInvalidDevice;
        hipLaunchKernelGGL((batch_stage_kernel<T, true, WALLS>), dim3(g), dim3(kBTX * kBTY), 0, st,
                           args_dev, tiles_dev, len);
    } else {
        hipLaunchKernelGGL((batch_stage_kernel<T, false, WALLS>), dim3(num_tiles), dim3(kBTX * kBTY),
                           0, st, args_dev, tiles_dev, len);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_stage(const StageArgs<T>* args_dev, const BatchTile* tiles_dev, int num_tiles,
                              bool persistent, bool walls, hipStream_t st)
{
    if (num_tiles <= 0 || num_tiles % 8) return hipErrorInvalidValue;
    return walls ? launch_batch_stage_form<T, true>(args_dev, tiles_dev, num_tiles, persistent, st)
                 : launch_batch_stage_form<T, false>(args_dev, tiles_dev, num_tiles, persistent, st);
}

template hipError_t launch_batch_stage<float>(const StageArgs<float>*, const BatchTile*, int, bool, bool, hipStream_t);
template hipError_t launch_batch_stage<double>(const StageArgs<double>*, const BatchTile*, int, bool, bool, hipStream_t);

}  // namespace pf
