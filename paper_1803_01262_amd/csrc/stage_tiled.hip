// Stage kernel, tiled variants: each workgroup owns a TX x TY column tile and marches a chunk of
// KZ planes along z.
//
// Per plane it keeps, in LDS, a three-plane ring of the stage input with a two-cell halo (the
// reach of the sharpening term: the normal at a face neighbour needs its own neighbours), the
// x- and y-components of the sharpening product q = phi(1-phi)n of the current and next plane
// (with a one-cell halo in their own direction only), and in registers the z-component of q and
// the z-face flux, which each thread hands from one plane to the next. Every q is computed once
// per cell (plus the halo ring), every face flux once per face except the x/y faces on the
// tile edge. The next plane is prefetched into registers while the current one is computed.
// Workgroups are ordered so that each of the 8 XCDs sweeps a contiguous block of tiles, which
// keeps the halo rows of neighbouring tiles in that XCD's L2.
#include "pf_tiled_body.h"

namespace pf {

template <typename T, int TX, int TY, int KZ>
__global__ void __launch_bounds__(TX* TY) stage_tiled_kernel(StageArgs<T> a, int tiles_x,
                                                             int tiles_y)
{
    // XCD-aware tile order: consecutive workgroup ids go round-robin over the 8 XCDs; give each
    // XCD a contiguous range of tiles (x fastest, then y, then z-chunk).
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int ti = b % tiles_x;
    b /= tiles_x;
    const int tj = b % tiles_y;
    const int tk = b / tiles_y;
    tiled_stage_body<T, TX, TY, KZ>(a, ti, tj, tk);
}

template <typename T, int TX, int TY, int KZ>
hipError_t launch_stage_tiled(const StageArgs<T>& a, hipStream_t st)
{
    const int tiles_x = (a.nx + TX - 1) / TX;
    const int tiles_y = (a.ny + TY - 1) / TY;
    const int chunks = (a.nz + KZ - 1) / KZ;
    const long long blocks = (long long)tiles_x * tiles_y * chunks;
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage_tiled_kernel<T, TX, TY, KZ>), dim3((unsigned)blocks), dim3(TX * TY),
                       0, st, a, tiles_x, tiles_y);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stage_global(const StageArgs<T>& a, hipStream_t st);

static bool fits_any(int, int, int, int) { return true; }

#define PF_TILED(TX, TY, KZ)                                                            \
    {"tiled_" #TX "x" #TY "x" #KZ, launch_stage_tiled<float, TX, TY, KZ>,               \
     launch_stage_tiled<double, TX, TY, KZ>, fits_any}

static const StageVariant kVariants[] = {
    PF_TILED(64, 8, 32),
    PF_TILED(64, 4, 32),
    PF_TILED(64, 8, 64),
    PF_TILED(64, 4, 64),
    PF_TILED(32, 8, 32),
    PF_TILED(128, 4, 32),
    PF_TILED(64, 8, 16),
    {"global", launch_stage_global<float>, launch_stage_global<double>, fits_any},
};

int stage_variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
const StageVariant& stage_variant(int v) { return kVariants[v]; }

int default_stage_variant(int nx, int ny, int nz, int dtype)
{
    (void)nx;
    (void)ny;
    (void)nz;
    (void)dtype;
    return 0;
}

}  // namespace pf
