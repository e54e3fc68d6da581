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
#include <cstring>

#include "pf_tiled_body.h"

namespace pf {

template <typename T, int TX, int TY, int KZ, bool BIG>
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
    tiled_stage_body<T, TX, TY, KZ, BIG>(a, ti, tj, tk);
}

// FORCE_BIG selects the per-plane descriptor form even for small arrays (it is what arrays of
// 4 GiB or more take), so that form can be checked against the default one at any size.
template <typename T, int TX, int TY, int KZ, bool FORCE_BIG>
hipError_t launch_stage_tiled(const StageArgs<T>& a, hipStream_t st)
{
    const int tiles_x = (a.nx + TX - 1) / TX;
    const int tiles_y = (a.ny + TY - 1) / TY;
    const int chunks = (a.nz + KZ - 1) / KZ;
    const long long blocks = (long long)tiles_x * tiles_y * chunks;
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (FORCE_BIG || field_needs_big(a.nx, a.ny, a.nz, sizeof(T)))
        hipLaunchKernelGGL((stage_tiled_kernel<T, TX, TY, KZ, true>), dim3((unsigned)blocks),
                           dim3(TX * TY), 0, st, a, tiles_x, tiles_y);
    else
        hipLaunchKernelGGL((stage_tiled_kernel<T, TX, TY, KZ, false>), dim3((unsigned)blocks),
                           dim3(TX * TY), 0, st, a, tiles_x, tiles_y);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stage_global(const StageArgs<T>& a, hipStream_t st);
template <typename T, int TX, int TY, int KZ, bool FORCE_BIG>
hipError_t launch_fused(const FusedArgs<T>& a, bool sweep_b, hipStream_t st);

#define PF_TILED(TX, TY, KZ)                                                            \
    {"tiled_" #TX "x" #TY "x" #KZ, launch_stage_tiled<float, TX, TY, KZ, false>,        \
     launch_stage_tiled<double, TX, TY, KZ, false>, nullptr, nullptr}
#define PF_FUSED(TX, TY, KZ)                                                            \
    {"fused_" #TX "x" #TY "x" #KZ, nullptr, nullptr,                                    \
     launch_fused<float, TX, TY, KZ, false>, launch_fused<double, TX, TY, KZ, false>}
#define PF_FUSED32(TX, TY, KZ)                                                          \
    {"fused_" #TX "x" #TY "x" #KZ, nullptr, nullptr,                                    \
     launch_fused<float, TX, TY, KZ, false>, nullptr}

static const StageVariant kVariants[] = {
    PF_TILED(64, 8, 16),
    PF_TILED(64, 4, 16),
    PF_TILED(32, 4, 16),
    PF_TILED(64, 8, 32),
    PF_TILED(64, 8, 64),
    PF_TILED(64, 4, 32),
    PF_TILED(64, 4, 64),
    PF_TILED(32, 8, 32),
    PF_TILED(128, 4, 32),
    {"global", launch_stage_global<float>, launch_stage_global<double>, nullptr, nullptr},
    PF_FUSED(64, 8, 32),
    PF_FUSED(64, 8, 64),
    PF_FUSED(32, 16, 32),
    PF_FUSED(32, 16, 64),
    PF_FUSED32(64, 16, 32),
    PF_FUSED32(64, 16, 64),
    PF_FUSED32(128, 8, 32),
    // the large-array addressing form, forced (selected automatically at 4 GiB per array)
    {"tiled_64x8x16_big", launch_stage_tiled<float, 64, 8, 16, true>,
     launch_stage_tiled<double, 64, 8, 16, true>, nullptr, nullptr},
    {"fused_64x8x32_big", nullptr, nullptr, launch_fused<float, 64, 8, 32, true>,
     launch_fused<double, 64, 8, 32, true>},
};
constexpr int kNumVariants = (int)(sizeof(kVariants) / sizeof(kVariants[0]));

static bool supports(const StageVariant& v, int dtype)
{
    return dtype == PF_F32 ? (v.launch_f32 || v.fused_f32) : (v.launch_f64 || v.fused_f64);
}

// per-dtype index lists into kVariants
static const int* variant_list(int dtype, int* count)
{
    static int lists[2][kNumVariants];
    static int counts[2] = {-1, -1};
    const int d = dtype == PF_F32 ? 0 : 1;
    if (counts[d] < 0) {
        int c = 0;
        for (int v = 0; v < kNumVariants; ++v)
            if (supports(kVariants[v], dtype)) lists[d][c++] = v;
        counts[d] = c;
    }
    *count = counts[d];
    return lists[d];
}

int stage_variant_count(int dtype)
{
    int c;
    variant_list(dtype, &c);
    return c;
}

const StageVariant& stage_variant(int dtype, int v)
{
    int c;
    const int* l = variant_list(dtype, &c);
    return kVariants[l[v]];
}

bool variant_is_fused(int dtype, int v)
{
    const StageVariant& s = stage_variant(dtype, v);
    return dtype == PF_F32 ? s.fused_f32 != nullptr : s.fused_f64 != nullptr;
}

// Default tile choice before (or without) autotuning: the first variant of a per-dtype
// preference list (fastest first, as measured on MI355X at 256^3-512^3) whose launch has at
// least 512 workgroups, i.e. two per compute unit; small grids fall through to small tiles.
int default_stage_variant(int nx, int ny, int nz, int dtype)
{
    struct Cand {
        const char* name;
        int tx, ty, kz;
    };
    static const Cand f32[] = {{"fused_64x8x64", 64, 8, 64},  {"fused_32x16x64", 32, 16, 64},
                               {"fused_64x8x32", 64, 8, 32},  {"fused_32x16x32", 32, 16, 32},
                               {"tiled_64x4x16", 64, 4, 16},  {"tiled_32x4x16", 32, 4, 16}};
    static const Cand f64[] = {{"fused_32x16x64", 32, 16, 64}, {"fused_64x8x64", 64, 8, 64},
                               {"fused_32x16x32", 32, 16, 32}, {"fused_64x8x32", 64, 8, 32},
                               {"tiled_64x4x16", 64, 4, 16},   {"tiled_32x4x16", 32, 4, 16}};
    const Cand* list = dtype == PF_F32 ? f32 : f64;
    const int n = 6;
    int pick = n - 1;
    for (int c = 0; c < n; ++c) {
        const long long blocks = (long long)((nx + list[c].tx - 1) / list[c].tx) *
                                 ((ny + list[c].ty - 1) / list[c].ty) *
                                 ((nz + list[c].kz - 1) / list[c].kz);
        if (blocks >= 512) {
            pick = c;
            break;
        }
    }
    for (int v = 0; v < stage_variant_count(dtype); ++v)
        if (std::strcmp(stage_variant(dtype, v).name, list[pick].name) == 0) return v;
    return 0;
}

}  // namespace pf
