// Small element-wise kernels (copy, fill) used by the step schedules. They are plain kernels
// rather than hipMemcpyAsync / hipMemsetAsync so that captured graphs hold kernel nodes only.
#include "pf_internal.h"

namespace pf {

template <typename T>
__global__ void copy_kernel(T* __restrict__ dst, const T* __restrict__ src, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) dst[c] = src[c];
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ dst, T value, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) dst[c] = value;
}

static unsigned grid_for(size_t n)
{
    size_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <typename T>
hipError_t launch_copy(T* dst, const T* src, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(copy_kernel<T>, dim3(grid_for(n)), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* dst, T value, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(n)), dim3(256), 0, st, dst, value, n);
    return hipGetLastError();
}

template hipError_t launch_copy<float>(float*, const float*, size_t, hipStream_t);
template hipError_t launch_copy<double>(double*, const double*, size_t, hipStream_t);
template hipError_t launch_fill<float>(float*, float, size_t, hipStream_t);
template hipError_t launch_fill<double>(double*, double, size_t, hipStream_t);

}  // namespace pf
