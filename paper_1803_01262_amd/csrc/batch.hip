// Batched stage kernel: one persistent launch advances one RK stage of many independent
// simulations. The tiles of all instances form one global list; each workgroup strides over it
// and runs the same per-tile body as the single-grid tiled kernel, so every instance's result
// is bit-identical to its own single solve.
#include "pf_tiled_body.h"

namespace pf {

constexpr int kBTX = 32, kBTY = 8, kBKZ = 32;  // tile shape of the batched launch

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
        tiled_stage_body<T, kBTX, kBTY, kBKZ>(a, ti, tj, tk);
    }
}

void batch_tile_counts(int nx, int ny, int nz, int* tx, int* ty, int* cz)
{
    *tx = (nx + kBTX - 1) / kBTX;
    *ty = (ny + kBTY - 1) / kBTY;
    *cz = (nz + kBKZ - 1) / kBKZ;
}

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
