// Fused two-stage sweeps (see pf_fused_body.h): the single-grid kernel and its launcher,
// instantiated per storage type in stage_fused_f32.hip / stage_fused_f64.hip. Tile order is
// XCD-aware as in the per-stage kernels.
#pragma once

#include "pf_fused_body.h"

namespace pf {

// FP32: at least four waves per SIMD (at most 128 VGPRs), two workgroups of eight waves per CU.
// FP64 needs more registers than that and runs at two waves per SIMD.
template <typename T, int TX, int TY, int KZ, bool SWEEP_B, bool BIG, bool WIDE>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
fused_kernel(FusedArgs<T> a, int tiles_x, int tiles_y)
{
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int ti = b % tiles_x;
    b /= tiles_x;
    const int tj = b % tiles_y;
    const int tk = b / tiles_y;
    fused_body<T, TX, TY, KZ, SWEEP_B, BIG, WIDE>(a, ti, tj, tk);
}

template <typename T, int TX, int TY, int KZ, bool BIG, bool WIDE>
static hipError_t launch_fused_sweep(const FusedArgs<T>& a, bool sweep_b, unsigned blocks,
                                     int tiles_x, int tiles_y, hipStream_t st)
{
    if (sweep_b)
        hipLaunchKernelGGL((fused_kernel<T, TX, TY, KZ, true, BIG, WIDE>), dim3(blocks),
                           dim3(TX * TY), 0, st, a, tiles_x, tiles_y);
    else
        hipLaunchKernelGGL((fused_kernel<T, TX, TY, KZ, false, BIG, WIDE>), dim3(blocks),
                           dim3(TX * TY), 0, st, a, tiles_x, tiles_y);
    return hipGetLastError();
}

// FORCE_BIG selects the per-plane descriptor form even for small arrays (see the tiled launcher).
template <typename T, int TX, int TY, int KZ, bool FORCE_BIG>
hipError_t launch_fused(const FusedArgs<T>& a, bool sweep_b, hipStream_t st)
{
    const int tiles_x = (a.nx + TX - 1) / TX;
    const int tiles_y = (a.ny + TY - 1) / TY;
    const int chunks = (a.nz + KZ - 1) / KZ;
    const long long blocks = (long long)tiles_x * tiles_y * chunks;
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    // 16-byte plane loads need rows that are a whole number of 16-byte pieces
    const bool wide = a.nx % (16 / (int)sizeof(T)) == 0;
    const unsigned nb = (unsigned)blocks;
    if (FORCE_BIG || field_needs_big(a.nx, a.ny, a.nz, sizeof(T)))
        return wide ? launch_fused_sweep<T, TX, TY, KZ, true, true>(a, sweep_b, nb, tiles_x, tiles_y, st)
                    : launch_fused_sweep<T, TX, TY, KZ, true, false>(a, sweep_b, nb, tiles_x, tiles_y, st);
    return wide ? launch_fused_sweep<T, TX, TY, KZ, false, true>(a, sweep_b, nb, tiles_x, tiles_y, st)
                : launch_fused_sweep<T, TX, TY, KZ, false, false>(a, sweep_b, nb, tiles_x, tiles_y, st);
}

}  // namespace pf

#define PF_FUSED_INST(T, TX, TY, KZ, FB)                                                 \
    template hipError_t pf::launch_fused<T, TX, TY, KZ, FB>(const pf::FusedArgs<T>&, bool, \
                                                            hipStream_t);
