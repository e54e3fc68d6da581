// Stage kernel, tiled variants: each workgroup owns a TX x TY column tile and marches a chunk of
// kz planes along z (kz fixed by the variant, or chosen per launch).
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

template <typename T, int TX, int TY, bool BIG, bool WALLS, bool PREFETCH, bool NU = false>
__global__ void __launch_bounds__(TX* TY) stage_tiled_kernel(StageArgs<T> a, int tiles_x,
                                                             int tiles_y, int kz)
{
    // XCD-aware tile order: consecutive workgroup ids go round-robin over the 8 XCDs; give each
    // XCD a contiguous range of tiles (x fastest, then y, then z-chunk).
    int b = xcd_tile_order(blockIdx.x, gridDim.x);
    const int ti = b % tiles_x;
    b /= tiles_x;
    const int tj = b % tiles_y;
    const int k0 = (b / tiles_y) * kz;
    tiled_stage_body<T, TX, TY, BIG, WALLS, PREFETCH, NU>(a, ti, tj, k0, min(k0 + kz, a.nz));
}

// The same stage on a grid of one plane (nz = 1): the z-neighbours of every cell are the cell
// itself (periodic wrap, or the mirror of a z-wall), so the march's warm-up planes and its
// plane-to-plane hand-over carry copies of the one plane. This kernel loads the tile with its
// two-cell halo once and feeds the cell function exactly the values the march would (z-face sum
// 2 phi, z-face difference and z-gradient zero, both z-faces of q and of W the cell's own), so
// the two agree bitwise, with one load round and two barriers instead of six march iterations.
template <typename T, int TX, int TY, bool WALLS>
__global__ void __launch_bounds__(TX* TY) stage_plane_kernel(StageArgs<T> a, int tiles_x)
{
    constexpr int NT = TX * TY;
    constexpr int PW = TX + 4, PH = TY + 4, PS = PW * PH;
    constexpr int QXW = TX + 2, QXS = QXW * TY;
    constexpr int QYS = TX * (TY + 2);
    constexpr int NL = (PS + NT - 1) / NT;
    static_assert(NT >= 2 * TX + 2 * TY, "halo ring needs one thread per halo cell");
    __shared__ T sp[PS];
    __shared__ T sqx[QXS];
    __shared__ T sqy[QYS];

    const int b = xcd_tile_order(blockIdx.x, gridDim.x);
    const int i0 = (b % tiles_x) * TX, j0 = (b / tiles_x) * TY;
    const int nx = a.nx, ny = a.ny;
    const bool wx = WALLS && (a.walls & 1), wy = WALLS && (a.walls & 2), wz = WALLS && (a.walls & 4);
    auto mapx = [&](int v) { return WALLS && wx ? reflectn(v, nx) : wrapn(v, nx); };
    auto mapy = [&](int v) { return WALLS && wy ? reflectn(v, ny) : wrapn(v, ny); };
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool active = (i < nx) && (j < ny);
    const int iw = wrapn(i, nx), jw = wrapn(j, ny);
    const size_t col = (size_t)jw * nx + iw;
    const size_t col_xp = (size_t)jw * nx + wrapn(i + 1, nx);
    const size_t col_yp = (size_t)wrapn(j + 1, ny) * nx + iw;

#pragma unroll
    for (int s = 0; s < NL; ++s) {
        const int e = tid + s * NT;
        if (e < PS) {
            const int r = e / PW, c = e - r * PW;
            sp[e] = a.y[(size_t)mapy(j0 - 2 + r) * nx + mapx(i0 - 2 + c)];
        }
    }
    T u0 = a.U[col], u1 = a.U[col_xp], v0 = a.V[col], v1 = a.V[col_yp], w = a.W[col];
    if constexpr (WALLS) {  // velocities on wall faces (index 0 of a walled axis)
        if (wx && iw == 0) u0 = T(0);
        if (wx && iw == nx - 1) u1 = T(0);
        if (wy && jw == 0) v0 = T(0);
        if (wy && jw == ny - 1) v1 = T(0);
        if (wz) w = T(0);
    }
    T b1 = T(0), b2 = T(0);
    if (a.out1) b1 = a.base1[col];
    if (a.out2) b2 = a.base2[col];
    __syncthreads();

    const T inv_2dx = a.inv_2dx, d2 = a.delta2, hg = a.hg;
    const int o = (ty + 2) * PW + (tx + 2);
    const T pc = sp[o];
    const T gx = grad1(sp[o + 1], sp[o - 1], inv_2dx);
    const T gy = grad1(sp[o + PW], sp[o - PW], inv_2dx);
    const T gz = grad1(pc, pc, inv_2dx);
    const T fac = sharpen_factor(pc, gx, gy, gz, d2, hg);
    sqx[ty * QXW + tx + 1] = fac * gx;
    sqy[(ty + 1) * TX + tx] = fac * gy;
    const T qz = fac * gz;
    // halo ring, assigned as in the march
    if (tid < 2 * TY) {
        const int side = tid / TY, r = tid - side * TY;
        const int h = (r + 2) * PW + (side ? TX + 2 : 1);
        const T hgx = grad1(sp[h + 1], sp[h - 1], inv_2dx);
        const T hgy = grad1(sp[h + PW], sp[h - PW], inv_2dx);
        const T hgz = grad1(sp[h], sp[h], inv_2dx);
        sqx[r * QXW + (side ? TX + 1 : 0)] = sharpen_factor(sp[h], hgx, hgy, hgz, d2, hg) * hgx;
    } else if (tid < 2 * TY + 2 * TX) {
        const int t2 = tid - 2 * TY;
        const int side = t2 / TX, c = t2 - side * TX;
        const int h = (side ? TY + 2 : 1) * PW + c + 2;
        const T hgx = grad1(sp[h + 1], sp[h - 1], inv_2dx);
        const T hgy = grad1(sp[h + PW], sp[h - PW], inv_2dx);
        const T hgz = grad1(sp[h], sp[h], inv_2dx);
        sqy[(side ? TY + 1 : 0) * TX + c] = sharpen_factor(sp[h], hgx, hgy, hgz, d2, hg) * hgy;
    }
    __syncthreads();
    if (!active) return;
    const T sz = face_sum(pc, pc), dz = face_diff(pc, pc);
    const T* QX = sqx + ty * QXW + tx;
    const T* QY = sqy + ty * TX + tx;
    const T pxm = sp[o - 1], pxp = sp[o + 1], pym = sp[o - PW], pyp = sp[o + PW];
    const T f = cell_rhs(face_sum(pxm, pc), face_sum(pc, pxp), face_sum(pym, pc), face_sum(pc, pyp),
                         sz, sz, face_diff(pxm, pc), face_diff(pc, pxp), face_diff(pym, pc),
                         face_diff(pc, pyp), dz, dz, QX[0], QX[2], QY[0], QY[2 * TX], qz, qz, u0,
                         u1, v0, v1, w, w, a.nhs, a.ge);
    if (a.out1) a.out1[col] = fma(a.c1, f, b1);
    if (a.out2) a.out2[col] = fma(a.c2, f, b2);
}

// KZ: planes per z-chunk; KZ = 0 chooses it per launch (launch_chunk_planes).
// FORCE_BIG selects the per-plane descriptor form even for small arrays (it is what arrays of
// 4 GiB or more take), so that form can be checked against the default one at any size.
// NU: the non-uniform mesh form (a.nu set), which marches one-plane grids too.
template <typename T, int TX, int TY, int KZ, bool FORCE_BIG, bool NU = false>
hipError_t launch_stage_tiled(const StageArgs<T>& a, hipStream_t st)
{
    const int tiles_x = (a.nx + TX - 1) / TX;
    const int tiles_y = (a.ny + TY - 1) / TY;
    if (a.nz <= 0 || tiles_x <= 0 || tiles_y <= 0) return hipErrorInvalidValue;
    const bool walls = a.walls != 0;
    if (a.nz == 1 && !NU) {  // one plane: no march (a plane is below 2^28 cells, plain addressing)
        const long long blocks = (long long)tiles_x * tiles_y;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
        hipLaunchKernelGGL((walls ? stage_plane_kernel<T, TX, TY, true> : stage_plane_kernel<T, TX, TY, false>),
                           dim3((unsigned)blocks), dim3(TX * TY), 0, st, a, tiles_x);
        return hipGetLastError();
    }
    const bool big = FORCE_BIG || field_needs_big(a.nx, a.ny, a.nz, sizeof(T));
    using Kernel = void (*)(StageArgs<T>, int, int, int);
    // chunks of kPrefetchPlanes planes or more take the form that loads the per-cell operands one
    // iteration ahead
    constexpr int kPrefetchPlanes = 48;
    auto pick = [&](bool prefetch) -> Kernel {
        if (prefetch)
            return big ? (walls ? stage_tiled_kernel<T, TX, TY, true, true, true, NU>
                                : stage_tiled_kernel<T, TX, TY, true, false, true, NU>)
                       : (walls ? stage_tiled_kernel<T, TX, TY, false, true, true, NU>
                                : stage_tiled_kernel<T, TX, TY, false, false, true, NU>);
        return big ? (walls ? stage_tiled_kernel<T, TX, TY, true, true, false, NU>
                            : stage_tiled_kernel<T, TX, TY, true, false, false, NU>)
                   : (walls ? stage_tiled_kernel<T, TX, TY, false, true, false, NU>
                            : stage_tiled_kernel<T, TX, TY, false, false, false, NU>);
    };
    int kz = KZ;
    bool prefetch = KZ >= kPrefetchPlanes;
    if (KZ == 0) {  // the chunk the prefetching form would take (its own occupancy), if long
        kz = launch_chunk_planes((const void*)pick(true), TX * TY, (long long)tiles_x * tiles_y,
                                 a.nz, 1);
        prefetch = kz >= kPrefetchPlanes;
        if (!prefetch)
            kz = launch_chunk_planes((const void*)pick(false), TX * TY,
                                     (long long)tiles_x * tiles_y, a.nz, 1);
        if (kz <= 0) return hipErrorInvalidDevice;
    }
    const Kernel kern = pick(prefetch);
    const long long blocks = (long long)tiles_x * tiles_y * ((a.nz + kz - 1) / kz);
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(TX * TY), 0, st, a, tiles_x, tiles_y, kz);
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
// chunk length chosen per launch (launch_chunk_planes)
#define PF_TILED_AUTO(TX, TY)                                                           \
    {"tiled_" #TX "x" #TY, launch_stage_tiled<float, TX, TY, 0, false>,                  \
     launch_stage_tiled<double, TX, TY, 0, false>, nullptr, nullptr}
#define PF_FUSED_AUTO(TX, TY)                                                           \
    {"fused_" #TX "x" #TY, nullptr, nullptr, launch_fused<float, TX, TY, 0, false>,     \
     launch_fused<double, TX, TY, 0, false>}
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
    PF_TILED_AUTO(64, 8),
    PF_TILED_AUTO(64, 4),
    PF_TILED_AUTO(32, 4),
    {"global", launch_stage_global<float>, launch_stage_global<double>, nullptr, nullptr},
    PF_FUSED(64, 8, 32),
    PF_FUSED(64, 8, 64),
    PF_FUSED(32, 16, 32),
    PF_FUSED(32, 16, 64),
    PF_FUSED_AUTO(64, 8),
    PF_FUSED_AUTO(32, 16),
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

static int variant_by_name(int dtype, const char* name)
{
    for (int v = 0; v < stage_variant_count(dtype); ++v)
        if (std::strcmp(stage_variant(dtype, v).name, name) == 0) return v;
    return 0;
}

int stage_variant_index(int dtype, const char* name) { return variant_by_name(dtype, name); }

// 64-wide tiles unless they pad more columns than 32-wide ones.
static bool prefer_x64(int nx)
{
    return (nx + 63) / 64 * 64 <= (nx + 31) / 32 * 32;
}

// A stage on a non-uniform mesh: the tiled per-stage kernel in its NU form on 64x4 tiles (32x4
// where 64-wide tiles pad more columns), chunk length chosen per launch.
template <typename T>
hipError_t launch_stage_nu(const StageArgs<T>& a, hipStream_t st)
{
    return prefer_x64(a.nx) ? launch_stage_tiled<T, 64, 4, 0, false, true>(a, st)
                            : launch_stage_tiled<T, 32, 4, 0, false, true>(a, st);
}
template hipError_t launch_stage_nu<float>(const StageArgs<float>&, hipStream_t);
template hipError_t launch_stage_nu<double>(const StageArgs<double>&, hipStream_t);

// Grids from this many cells up take the fused sweeps by default, smaller ones the per-stage
// kernels (MI355X, ms per step, best per-stage / best fused: FP32 80^3 0.036 / 0.044, 96^3
// 0.041 / 0.045, 112^3 0.058 / 0.057, 128^3 0.066 / 0.058; FP64 128^3 0.094 / 0.099, 160^3
// 0.152 / 0.155, 192^3 0.325 / 0.272). FP64 takes the fused sweeps from 128^3 all the same: a
// per-stage forward variant lends its tile to the adjoint, and at 128^3 the adjoint step on 32x4
// tiles took 0.284 ms against 0.259 after a fused forward variant (64x8 tiles).
constexpr long long kFusedMinCellsF32 = 104LL * 104 * 104;
constexpr long long kFusedMinCellsF64 = 128LL * 128 * 128;
constexpr long long kX64MinCellsF32 = 256LL * 256 * 256;

// Default variant before (or without) autotuning, from MI355X measurements at 32^3-640^3, all with
// the chunk length chosen per launch: the fused sweeps (FP32 on 64x8 tiles unless those pad more
// columns than 32x16, FP64 on 32x16) and, below the size thresholds or on one-plane grids, the
// per-stage kernel.
int default_stage_variant(int nx, int ny, int nz, int dtype)
{
    // one plane: the per-stage launch takes the march-free plane kernel (a fused sweep would march
    // its warm-up over copies of the same plane: 3-8 x slower at 512^2-4096^2); from 256^2 cells
    // on 64x8 tiles (fastest at 512^2-4096^2 in both precisions) unless those pad more columns
    // than 32x4, below that on the per-stage rule's smaller tiles (more workgroups: 64^2 FP64
    // 14.2 against 15.8 us per step)
    if (nz == 1)
        return (long long)nx * ny >= 256LL * 256 && prefer_x64(nx) ? variant_by_name(dtype, "tiled_64x8")
                                                                   : per_stage_variant(nx, ny, nz, dtype);
    const long long cells = (long long)nx * ny * nz;
    // FP32 fused tiles: 64x8 from 256^3 cells (512^3: 1.87 against 2.09 ms) unless they pad more
    // columns than 32x16; 32x16 below (128^3 and 192^3: 2-3 % faster, medians of four runs)
    if (dtype == PF_F32)
        return cells >= kFusedMinCellsF32
                   ? variant_by_name(dtype, cells >= kX64MinCellsF32 && prefer_x64(nx) ? "fused_64x8"
                                                                                     : "fused_32x16")
                   : per_stage_variant(nx, ny, nz, dtype);
    return cells >= kFusedMinCellsF64 ? variant_by_name(dtype, "fused_32x16")
                                      : per_stage_variant(nx, ny, nz, dtype);
}

// FP32 on 64x4 tiles unless those pad more columns than 32x4 (512^3: 3.36 ms per RK4 step against
// 3.49 on 64x8); FP64 on 32x4 below 176^3 cells (128^3: 0.094 ms, 160^3: 0.152 against 0.162 on
// 64x8) and on 64x8 from there unless those pad more columns (192^3: 64x8 0.325, 32x4 slower;
// 512^3: 6.16 against 7.12 ms).
int per_stage_variant(int nx, int ny, int nz, int dtype)
{
    if (dtype == PF_F32) return variant_by_name(dtype, prefer_x64(nx) ? "tiled_64x4" : "tiled_32x4");
    const long long cells = (long long)nx * ny * nz;
    return variant_by_name(dtype, cells >= 176LL * 176 * 176 && prefer_x64(nx) ? "tiled_64x8" : "tiled_32x4");
}

}  // namespace pf
