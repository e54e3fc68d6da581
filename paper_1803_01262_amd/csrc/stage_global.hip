// Stage kernel, plain variant: one thread per cell, every operand read from global memory
// (L1/L2 supply the reuse). It is the reference shape for the tiled variants and the fallback
// for grids the tiled variants do not cover; all variants share pf_cell.h and agree bitwise.
#include "pf_cell.h"
#include "pf_internal.h"

namespace pf {

template <typename T>
__global__ void __launch_bounds__(256) stage_global_kernel(StageArgs<T> a)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= a.nx || j >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const T* __restrict__ y = a.y;
    const bool wx = a.walls & 1, wy = a.walls & 2, wz = a.walls & 4;
    // velocity faces: periodic storage (the high wall face of a walled axis is index 0)
    auto idx = [&](int di, int dj, int dk) -> size_t {
        return ((size_t)wrapn(k + dk, nz) * ny + wrapn(j + dj, ny)) * nx + wrapn(i + di, nx);
    };
    // stage input: periodic, or mirrored across walls
    auto at = [&](int di, int dj, int dk) -> T {
        const int ii = wx ? reflectn(i + di, nx) : wrapn(i + di, nx);
        const int jj = wy ? reflectn(j + dj, ny) : wrapn(j + dj, ny);
        const int kk = wz ? reflectn(k + dk, nz) : wrapn(k + dk, nz);
        return y[((size_t)kk * ny + jj) * nx + ii];
    };
    // a face velocity, zero on the wall faces (index 0 of a walled axis)
    auto vel = [&](const T* f, int di, int dj, int dk, bool wall, int ax) -> T {
        const int w = ax == 0 ? wrapn(i + di, nx) : (ax == 1 ? wrapn(j + dj, ny) : wrapn(k + dk, nz));
        return wall && w == 0 ? T(0) : f[idx(di, dj, dk)];
    };
    // one component of the sharpening product at a neighbouring centre
    auto qcomp = [&](int di, int dj, int dk, int ax) -> T {
        const T gx = grad1(at(di + 1, dj, dk), at(di - 1, dj, dk), a.inv_2dx);
        const T gy = grad1(at(di, dj + 1, dk), at(di, dj - 1, dk), a.inv_2dx);
        const T gz = grad1(at(di, dj, dk + 1), at(di, dj, dk - 1), a.inv_2dx);
        const T fac = sharpen_factor(at(di, dj, dk), gx, gy, gz, a.delta2, a.hg);
        return fac * (ax == 0 ? gx : (ax == 1 ? gy : gz));
    };
    const size_t c = idx(0, 0, 0);
    const T pc = at(0, 0, 0);
    const T pxm = at(-1, 0, 0), pxp = at(1, 0, 0), pym = at(0, -1, 0), pyp = at(0, 1, 0);
    const T pzm = at(0, 0, -1), pzp = at(0, 0, 1);
    const T f = cell_rhs(face_sum(pxm, pc), face_sum(pc, pxp), face_sum(pym, pc), face_sum(pc, pyp),
                         face_sum(pzm, pc), face_sum(pc, pzp), face_diff(pxm, pc), face_diff(pc, pxp),
                         face_diff(pym, pc), face_diff(pc, pyp), face_diff(pzm, pc), face_diff(pc, pzp),
                         qcomp(-1, 0, 0, 0), qcomp(1, 0, 0, 0), qcomp(0, -1, 0, 1), qcomp(0, 1, 0, 1),
                         qcomp(0, 0, -1, 2), qcomp(0, 0, 1, 2), vel(a.U, 0, 0, 0, wx, 0),
                         vel(a.U, 1, 0, 0, wx, 0), vel(a.V, 0, 0, 0, wy, 1), vel(a.V, 0, 1, 0, wy, 1),
                         vel(a.W, 0, 0, 0, wz, 2), vel(a.W, 0, 0, 1, wz, 2), a.nhs, a.ge);
    if (a.out1) a.out1[c] = fma(a.c1, f, a.base1[c]);
    if (a.out2) a.out2[c] = fma(a.c2, f, a.base2[c]);
}

template <typename T>
hipError_t launch_stage_global(const StageArgs<T>& a, hipStream_t st)
{
    dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4, a.nz);
    hipLaunchKernelGGL(stage_global_kernel<T>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

template hipError_t launch_stage_global<float>(const StageArgs<float>&, hipStream_t);
template hipError_t launch_stage_global<double>(const StageArgs<double>&, hipStream_t);

}  // namespace pf
