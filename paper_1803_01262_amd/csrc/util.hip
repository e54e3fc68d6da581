// Small element-wise kernels (copy, fill) used by the step schedules. They are plain kernels
// rather than hipMemcpyAsync / hipMemsetAsync so that captured graphs hold kernel nodes only.
#include <atomic>
#include <cstdint>
#include <mutex>
#include <utility>
#include <vector>

#include "pf_internal.h"

namespace pf {

template <typename T>
__global__ void copy_kernel(T* __restrict__ dst, const T* __restrict__ src, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) dst[c] = src[c];
}

// The same copy in 16-byte pieces (both pointers 16-byte aligned); the elements past the last
// whole piece go to the first threads of block 0.
template <typename T>
__global__ void copy16_kernel(T* __restrict__ dst, const T* __restrict__ src, size_t n)
{
    constexpr int PE = 16 / (int)sizeof(T);
    const size_t np = n / PE;
    const uint4* __restrict__ s4 = reinterpret_cast<const uint4*>(src);
    uint4* __restrict__ d4 = reinterpret_cast<uint4*>(dst);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; c + 3 * stride < np; c += 4 * stride) {  // four pieces in flight
        const uint4 a = s4[c], b = s4[c + stride], e = s4[c + 2 * stride], f = s4[c + 3 * stride];
        d4[c] = a;
        d4[c + stride] = b;
        d4[c + 2 * stride] = e;
        d4[c + 3 * stride] = f;
    }
    for (; c < np; c += stride) d4[c] = s4[c];
    if (blockIdx.x == 0 && threadIdx.x < n - np * PE) dst[np * PE + threadIdx.x] = src[np * PE + threadIdx.x];
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ dst, T value, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) dst[c] = value;
}

// Compute units of the current device, read once per device.
int device_compute_units()
{
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
    if (dev < 64) {
        const int c = cached[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (dev < 64) cached[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

int resident_groups_per_cu(const void* kernel, int threads)
{
    static std::mutex mu;
    static std::vector<std::pair<const void*, int>> cache;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (const auto& e : cache)
            if (e.first == kernel) return e.second;
    }
    int groups = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&groups, kernel, threads, 0) != hipSuccess ||
        groups <= 0)
        return 0;
    std::lock_guard<std::mutex> lock(mu);
    cache.emplace_back(kernel, groups);
    return groups;
}

int launch_chunk_planes(const void* kernel, int threads, long long tiles, int nz, int extra)
{
    const int cus = device_compute_units();
    const int groups = resident_groups_per_cu(kernel, threads);
    if (cus <= 0 || groups <= 0 || tiles <= 0 || nz <= 0) return 0;
    return march_chunk_planes(tiles, nz, (long long)cus * groups, extra);
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
    if ((((uintptr_t)dst | (uintptr_t)src) & 15) == 0)
        hipLaunchKernelGGL(copy16_kernel<T>, dim3(grid_for(n / (16 / sizeof(T)) + 1)), dim3(256), 0, st,
                           dst, src, n);
    else
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
