// Fused two-stage sweeps (see pf_fused_body.h): launchers for the tile shapes in the variant
// table. Tile order is XCD-aware as in the per-stage kernels.
#include "pf_fused_body.h"

namespace pf {

template <typename T, int TX, int TY, int KZ, bool SWEEP_B>
__global__ void __launch_bounds__(TX* TY) fused_kernel(FusedArgs<T> a, int tiles_x, int tiles_y)
{
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int ti = b % tiles_x;
    b /= tiles_x;
    const int tj = b % tiles_y;
    const int tk = b / tiles_y;
    fused_body<T, TX, TY, KZ, SWEEP_B>(a, ti, tj, tk);
}

template <typename T, int TX, int TY, int KZ>
hipError_t launch_fused(const FusedArgs<T>& a, bool sweep_b, hipStream_t st)
{
    const int tiles_x = (a.nx + TX - 1) / TX;
    const int tiles_y = (a.ny + TY - 1) / TY;
    const int chunks = (a.nz + KZ - 1) / KZ;
    const long long blocks = (long long)tiles_x * tiles_y * chunks;
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (sweep_b)
        hipLaunchKernelGGL((fused_kernel<T, TX, TY, KZ, true>), dim3((unsigned)blocks),
                           dim3(TX * TY), 0, st, a, tiles_x, tiles_y);
    else
        hipLaunchKernelGGL((fused_kernel<T, TX, TY, KZ, false>), dim3((unsigned)blocks),
                           dim3(TX * TY), 0, st, a, tiles_x, tiles_y);
    return hipGetLastError();
}

#define PF_INST(T, TX, TY, KZ) \
    template hipError_t launch_fused<T, TX, TY, KZ>(const FusedArgs<T>&, bool, hipStream_t);
PF_INST(float, 64, 8, 32)
PF_INST(float, 64, 8, 64)
PF_INST(float, 64, 16, 32)
PF_INST(float, 64, 16, 64)
PF_INST(float, 128, 8, 32)
PF_INST(double, 64, 8, 32)
PF_INST(double, 64, 8, 64)

}  // namespace pf
