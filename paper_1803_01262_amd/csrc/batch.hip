// Batched stage kernel: one persistent launch advances one RK stage of many independent
// simulations. The tiles of all instances form one global list; each workgroup strides over it
// and runs the same per-tile body as the single-grid tiled kernel, so every instance's result
// is bit-identical to its own single solve.
#include "pf_fused_body.h"
#include "pf_tiled_body.h"

namespace pf {

constexpr int kBTX = 32, kBTY = 8, kBKZ = 32;   // per-stage mode tile shape
constexpr int kFTX = 32, kFTY = 16, kFKZ = 32;  // fused mode tile shape

template <typename T>
__global__ void __launch_bounds__(kBTX* kBTY) batch_stage_kernel(const BatchEntry<T>* __restrict__ table,
                                                                  const int* __restrict__ owner,
                                                                  int total_tiles)
{
    for (int t = blockIdx.x; t < total_tiles; t += gridDim.x) {
        const int b = owner[t];
        const StageArgs<T> a = table[b].a;
        int local = t - table[b].tile_begin;
        const int tiles_x = table[b].tiles_x, tiles_y = table[b].tiles_y;
        const int ti = local % tiles_x;
        local /= tiles_x;
        const int tj = local % tiles_y;
        const int tk = local / tiles_y;
        __syncthreads();  // the previous tile's LDS reads are complete
        tiled_stage_body<T, kBTX, kBTY, kBKZ, false>(a, ti, tj, tk);
    }
}

// Fused mode: the same persistent walk over the tile list, one launch per two-stage sweep.
template <typename T, bool SWEEP_B>
__global__ void __launch_bounds__(kFTX* kFTY) batch_fused_kernel(const FusedBatchEntry<T>* __restrict__ table,
                                                                  const int* __restrict__ owner,
                                                                  int total_tiles)
{
    for (int t = blockIdx.x; t < total_tiles; t += gridDim.x) {
        const int b = owner[t];
        const FusedArgs<T> a = table[b].a;
        int local = t - table[b].tile_begin;
        const int tiles_x = table[b].tiles_x, tiles_y = table[b].tiles_y;
        const int ti = local % tiles_x;
        local /= tiles_x;
        const int tj = local % tiles_y;
        const int tk = local / tiles_y;
        __syncthreads();  // the previous tile's LDS reads are complete
        fused_body<T, kFTX, kFTY, kFKZ, SWEEP_B, false>(a, ti, tj, tk);
    }
}

// dst[b] = src[b] for every instance b (blockIdx.y), grid-stride within the instance.
template <typename T>
__global__ void batch_copy_kernel(const BatchCopy<T>* __restrict__ e)
{
    const BatchCopy<T> c = e[blockIdx.y];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < c.n; i += (size_t)gridDim.x * blockDim.x)
        c.dst[i] = c.src[i];
}

void batch_tile_counts(bool fused, int nx, int ny, int nz, int* tx, int* ty, int* cz)
{
    const int TX = fused ? kFTX : kBTX, TY = fused ? kFTY : kBTY, KZ = fused ? kFKZ : kBKZ;
    *tx = (nx + TX - 1) / TX;
    *ty = (ny + TY - 1) / TY;
    *cz = (nz + KZ - 1) / KZ;
}

template <typename T>
hipError_t launch_batch_fused(const FusedBatchEntry<T>* table_dev, bool sweep_b, const int* owner_dev,
                              int total_tiles, int grid_blocks, hipStream_t st)
{
    if (sweep_b)
        hipLaunchKernelGGL((batch_fused_kernel<T, true>), dim3(grid_blocks), dim3(kFTX * kFTY), 0,
                           st, table_dev, owner_dev, total_tiles);
    else
        hipLaunchKernelGGL((batch_fused_kernel<T, false>), dim3(grid_blocks), dim3(kFTX * kFTY), 0,
                           st, table_dev, owner_dev, total_tiles);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_copy(const BatchCopy<T>* table_dev, int count, hipStream_t st)
{
    hipLaunchKernelGGL(batch_copy_kernel<T>, dim3(256, count), dim3(256), 0, st, table_dev);
    return hipGetLastError();
}

template hipError_t launch_batch_fused<float>(const FusedBatchEntry<float>*, bool, const int*, int, int, hipStream_t);
template hipError_t launch_batch_fused<double>(const FusedBatchEntry<double>*, bool, const int*, int, int, hipStream_t);
template hipError_t launch_batch_copy<float>(const BatchCopy<float>*, int, hipStream_t);
template hipError_t launch_batch_copy<double>(const BatchCopy<double>*, int, hipStream_t);

template <typename T>
hipError_t launch_batch_stage(const BatchEntry<T>* table_dev, const int* owner_dev, int total_tiles,
                              int grid_blocks, hipStream_t st)
{
    hipLaunchKernelGGL(batch_stage_kernel<T>, dim3(grid_blocks), dim3(kBTX * kBTY), 0, st,
                       table_dev, owner_dev, total_tiles);
    return hipGetLastError();
}

template hipError_t launch_batch_stage<float>(const BatchEntry<float>*, const int*, int, int, hipStream_t);
template hipError_t launch_batch_stage<double>(const BatchEntry<double>*, const int*, int, int, hipStream_t);

}  // namespace pf
