// Mass / bounds reduction: sum(phi) in double, min, max and a count of non-finite cells.
// Two passes with a fixed grid and a fixed tree, so the result does not depend on timing.
#include <cmath>
#include <type_traits>

#include "pf_internal.h"

namespace pf {

constexpr int kReduceThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kReduceThreads) reduce_partial_kernel(const T* __restrict__ phi,
                                                                        size_t n,
                                                                        double* __restrict__ part)
{
    __shared__ double s_sum[kReduceThreads], s_min[kReduceThreads], s_max[kReduceThreads],
        s_bad[kReduceThreads];
    double sum = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
    auto take = [&](T x) {
        const double v = (double)x;
        if (!isfinite(v)) {
            bad += 1.0;
            return;
        }
        sum += v;
        mn = fmin(mn, v);
        mx = fmax(mx, v);
    };
    // 16-byte pieces (phi is 16-byte aligned), four in flight per thread, in a fixed order; the
    // elements past the last whole piece go to the first threads of block 0
    using Piece = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    constexpr int PE = 16 / (int)sizeof(T);
    const Piece* __restrict__ pp = reinterpret_cast<const Piece*>(phi);
    const size_t np = n / PE;
    const size_t stride = (size_t)gridDim.x * kReduceThreads;
    size_t i = (size_t)blockIdx.x * kReduceThreads + threadIdx.x;
    auto take_piece = [&](const Piece& q) {
        if constexpr (PE == 4) {
            take(q.x);
            take(q.y);
            take(q.z);
            take(q.w);
        } else {
            take(q.x);
            take(q.y);
        }
    };
    for (; i + 3 * stride < np; i += 4 * stride) {
        const Piece a = pp[i], b = pp[i + stride], c = pp[i + 2 * stride], d = pp[i + 3 * stride];
        take_piece(a);
        take_piece(b);
        take_piece(c);
        take_piece(d);
    }
    for (; i < np; i += stride) take_piece(pp[i]);
    if (blockIdx.x == 0 && threadIdx.x < n - np * PE) take(phi[np * PE + threadIdx.x]);
    const int t = threadIdx.x;
    s_sum[t] = sum;
    s_min[t] = mn;
    s_max[t] = mx;
    s_bad[t] = bad;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            s_sum[t] += s_sum[t + w];
            s_min[t] = fmin(s_min[t], s_min[t + w]);
            s_max[t] = fmax(s_max[t], s_max[t + w]);
            s_bad[t] += s_bad[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        part[4 * blockIdx.x + 0] = s_sum[0];
        part[4 * blockIdx.x + 1] = s_min[0];
        part[4 * blockIdx.x + 2] = s_max[0];
        part[4 * blockIdx.x + 3] = s_bad[0];
    }
}

// The partial pass on a non-uniform mesh: each cell (i, j, k) enters the sum with the weight
// wx[i] wy[j] wz[k] (its volume), one element at a time in a fixed order; the tree is the one
// above.
template <typename T>
__global__ void __launch_bounds__(kReduceThreads)
reduce_partial_weighted_kernel(const T* __restrict__ phi, int nx, int ny, int nz,
                               const double* __restrict__ wx, const double* __restrict__ wy,
                               const double* __restrict__ wz, double* __restrict__ part)
{
    __shared__ double s_sum[kReduceThreads], s_min[kReduceThreads], s_max[kReduceThreads],
        s_bad[kReduceThreads];
    double sum = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
    const size_t n = (size_t)nx * ny * nz;
    const size_t stride = (size_t)gridDim.x * kReduceThreads;
    for (size_t c = (size_t)blockIdx.x * kReduceThreads + threadIdx.x; c < n; c += stride) {
        const double v = (double)phi[c];
        if (!isfinite(v)) {
            bad += 1.0;
            continue;
        }
        const size_t r = c / nx;
        const int i = (int)(c - r * nx), j = (int)(r % ny), k = (int)(r / ny);
        sum += v * (wx[i] * wy[j] * wz[k]);
        mn = fmin(mn, v);
        mx = fmax(mx, v);
    }
    const int t = threadIdx.x;
    s_sum[t] = sum;
    s_min[t] = mn;
    s_max[t] = mx;
    s_bad[t] = bad;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            s_sum[t] += s_sum[t + w];
            s_min[t] = fmin(s_min[t], s_min[t + w]);
            s_max[t] = fmax(s_max[t], s_max[t + w]);
            s_bad[t] += s_bad[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        part[4 * blockIdx.x + 0] = s_sum[0];
        part[4 * blockIdx.x + 1] = s_min[0];
        part[4 * blockIdx.x + 2] = s_max[0];
        part[4 * blockIdx.x + 3] = s_bad[0];
    }
}

__global__ void __launch_bounds__(kReduceThreads) reduce_final_kernel(const double* __restrict__ part,
                                                                      int nblocks,
                                                                      double* __restrict__ out4)
{
    __shared__ double s_sum[kReduceThreads], s_min[kReduceThreads], s_max[kReduceThreads],
        s_bad[kReduceThreads];
    const int t = threadIdx.x;
    double sum = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
    for (int b = t; b < nblocks; b += kReduceThreads) {
        sum += part[4 * b + 0];
        mn = fmin(mn, part[4 * b + 1]);
        mx = fmax(mx, part[4 * b + 2]);
        bad += part[4 * b + 3];
    }
    s_sum[t] = sum;
    s_min[t] = mn;
    s_max[t] = mx;
    s_bad[t] = bad;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            s_sum[t] += s_sum[t + w];
            s_min[t] = fmin(s_min[t], s_min[t + w]);
            s_max[t] = fmax(s_max[t], s_max[t + w]);
            s_bad[t] += s_bad[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        out4[0] = s_sum[0];
        out4[1] = s_min[0];
        out4[2] = s_max[0];
        out4[3] = s_bad[0];
    }
}

template <typename T>
hipError_t launch_reduce(const T* phi, size_t n, double* partial, double* out4, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_partial_kernel<T>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
                       phi, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kReduceThreads), 0, st, partial,
                       kReduceBlocks, out4);
    return hipGetLastError();
}

template hipError_t launch_reduce<float>(const float*, size_t, double*, double*, hipStream_t);
template hipError_t launch_reduce<double>(const double*, size_t, double*, double*, hipStream_t);

template <typename T>
hipError_t launch_reduce_weighted(const T* phi, int nx, int ny, int nz, const double* wx,
                                  const double* wy, const double* wz, double* partial,
                                  double* out4, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_partial_weighted_kernel<T>, dim3(kReduceBlocks), dim3(kReduceThreads),
                       0, st, phi, nx, ny, nz, wx, wy, wz, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kReduceThreads), 0, st, partial,
                       kReduceBlocks, out4);
    return hipGetLastError();
}

template hipError_t launch_reduce_weighted<float>(const float*, int, int, int, const double*,
                                                  const double*, const double*, double*, double*,
                                                  hipStream_t);
template hipError_t launch_reduce_weighted<double>(const double*, int, int, int, const double*,
                                                   const double*, const double*, double*, double*,
                                                   hipStream_t);

}  // namespace pf
