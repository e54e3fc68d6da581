// Fused two-stage sweeps (see pf_fused_body.h): the single-grid kernel and its launcher,
// instantiated per storage type in stage_fused_f32.hip / stage_fused_f64.hip. Tile order is
// XCD-aware as in the per-stage kernels.
#pragma once

#include "pf_fused_body.h"

namespace pf {

// One workgroup per (tile, z-chunk of kz planes); the chunk length is a launch argument.
// FP32: at least four waves per SIMD (at most 128 VGPRs), two workgroups of eight waves per CU.
// FP64 needs more registers than that and runs at two waves per SIMD.
// XOUT: the optional outputs (out_mid; sweep A also out_phi). WALLS: x and/or y walled (a.walls),
// element-wise plane loads, single-descriptor addressing.
template <typename T, int TX, int TY, bool SWEEP_B, bool BIG, bool WIDE, bool XOUT, bool WALLS = false>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
fused_kernel(FusedArgs<T> a, int tiles_x, int tiles_y, int kz)
{
    int b = xcd_tile_order(blockIdx.x, gridDim.x);
    const int ti = b % tiles_x;
    b /= tiles_x;
    const int tj = b % tiles_y;
    const int k0 = (b / tiles_y) * kz;
    fused_body<T, TX, TY, SWEEP_B, BIG, WIDE, XOUT, WALLS, fused_lag<T, TX, TY>()>(a, ti, tj, k0,
                                                                            min(k0 + kz, a.nz));
}

template <typename T, int TX, int TY, bool BIG, bool WIDE, bool WALLS = false>
hipError_t launch_fused_sweep(const FusedArgs<T>& a, bool sweep_b, unsigned blocks, int tiles_x,
                              int tiles_y, int kz, hipStream_t st)
{
    if (sweep_b) {
        if constexpr (!WALLS) {  // sweep B with out_mid: periodic x and y only
            if (a.out_mid) {
                hipLaunchKernelGGL((fused_kernel<T, TX, TY, true, BIG, WIDE, true, false>),
                                   dim3(blocks), dim3(TX * TY), 0, st, a, tiles_x, tiles_y, kz);
                return hipGetLastError();
            }
        }
        if (a.out_mid || a.out_phi) return hipErrorInvalidValue;
        hipLaunchKernelGGL((fused_kernel<T, TX, TY, true, BIG, WIDE, false, WALLS>), dim3(blocks),
                           dim3(TX * TY), 0, st, a, tiles_x, tiles_y, kz);
    } else if (a.out_mid || a.out_phi)
        hipLaunchKernelGGL((fused_kernel<T, TX, TY, false, BIG, WIDE, true, WALLS>), dim3(blocks),
                           dim3(TX * TY), 0, st, a, tiles_x, tiles_y, kz);
    else
        hipLaunchKernelGGL((fused_kernel<T, TX, TY, false, BIG, WIDE, false, WALLS>), dim3(blocks),
                           dim3(TX * TY), 0, st, a, tiles_x, tiles_y, kz);
    return hipGetLastError();
}

// KZ: planes per z-chunk, a host-side choice (every KZ shares the kernels of its tile shape);
// KZ = 0 chooses it per launch (launch_chunk_planes) for the grid and the current device.
// FORCE_BIG selects the per-plane descriptor form even for small arrays (see the tiled launcher).
template <typename T, int TX, int TY, int KZ, bool FORCE_BIG>
hipError_t launch_fused(const FusedArgs<T>& a, bool sweep_b, hipStream_t st)
{
    const int tiles_x = (a.nx + TX - 1) / TX;
    const int tiles_y = (a.ny + TY - 1) / TY;
    if (a.nz <= 0 || tiles_x <= 0 || tiles_y <= 0) return hipErrorInvalidValue;
    // 16-byte plane loads need rows that are a whole number of 16-byte pieces
    const bool wide = a.nx % (16 / (int)sizeof(T)) == 0;
    const bool big = FORCE_BIG || field_needs_big(a.nx, a.ny, a.nz, sizeof(T));
    if (a.walls) {
        // walled axes: one form (mirror reads element by element, single-descriptor addressing:
        // arrays below 4 GiB, also for the variants that force the large-array form)
        if (field_needs_big(a.nx, a.ny, a.nz, sizeof(T))) return hipErrorInvalidValue;
        int kzw = KZ;
        if (KZ == 0) {
            const void* k = (const void*)fused_kernel<T, TX, TY, false, false, false, false, true>;
            kzw = launch_chunk_planes(k, TX * TY, (long long)tiles_x * tiles_y, a.nz, 5);
            if (kzw <= 0) return hipErrorInvalidDevice;
        }
        const long long wb = (long long)tiles_x * tiles_y * ((a.nz + kzw - 1) / kzw);
        if (wb <= 0 || wb > 0x7fffffffLL) return hipErrorInvalidValue;
        return launch_fused_sweep<T, TX, TY, false, false, true>(a, sweep_b, (unsigned)wb, tiles_x,
                                                                 tiles_y, kzw, st);
    }
    int kz = KZ;
    if (KZ == 0) {
        // sweeps A and B share the register budget, hence the residency, of their form
        const void* k = big ? (wide ? (const void*)fused_kernel<T, TX, TY, false, true, true, false>
                                    : (const void*)fused_kernel<T, TX, TY, false, true, false, false>)
                            : (wide ? (const void*)fused_kernel<T, TX, TY, false, false, true, false>
                                    : (const void*)fused_kernel<T, TX, TY, false, false, false, false>);
        kz = launch_chunk_planes(k, TX * TY, (long long)tiles_x * tiles_y, a.nz, 5);
        if (kz <= 0) return hipErrorInvalidDevice;
    }
    const long long blocks = (long long)tiles_x * tiles_y * ((a.nz + kz - 1) / kz);
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)blocks;
    if (big)
        return wide ? launch_fused_sweep<T, TX, TY, true, true>(a, sweep_b, nb, tiles_x, tiles_y, kz, st)
                    : launch_fused_sweep<T, TX, TY, true, false>(a, sweep_b, nb, tiles_x, tiles_y, kz, st);
    return wide ? launch_fused_sweep<T, TX, TY, false, true>(a, sweep_b, nb, tiles_x, tiles_y, kz, st)
                : launch_fused_sweep<T, TX, TY, false, false>(a, sweep_b, nb, tiles_x, tiles_y, kz, st);
}

}  // namespace pf

#define PF_FUSED_INST(T, TX, TY, KZ, FB)                                                 \
    template hipError_t pf::launch_fused<T, TX, TY, KZ, FB>(const pf::FusedArgs<T>&, bool, \
                                                            hipStream_t);
