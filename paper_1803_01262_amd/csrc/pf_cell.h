// Per-cell arithmetic of the flux-form update (Sec. 2.2, five-step recipe), shared by every
// stage-kernel variant so that all variants produce bit-identical results. The library is
// compiled with floating-point contraction off; every fused multiply-add below is explicit.
#pragma once

#include <hip/hip_runtime.h>

namespace pf {

__device__ __forceinline__ float rsq(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }

// Central gradient component from the two neighbours along one axis (step 1).
template <typename T>
__device__ __forceinline__ T grad1(T p_plus, T p_minus, T inv_2dx)
{
    return (p_plus - p_minus) * inv_2dx;
}

// 1 / sqrt(|g|^2 + delta^2), and 0 where that vanishes: the unit normal is then 0, the
// reading of sgn(0) = 0 for a flat field (steps 1-2).
template <typename T>
__device__ __forceinline__ T inv_mag(T gx, T gy, T gz, T delta2)
{
    const T m2 = fma(gx, gx, fma(gy, gy, fma(gz, gz, delta2)));
    return m2 > T(0) ? rsq(m2) : T(0);
}

// Sharpening product q = phi (1 - phi) n at a cell centre (step 2), returned as the common
// factor phi (1 - phi) / |g|; q_a = factor * g_a.
template <typename T>
__device__ __forceinline__ T sharpen_factor(T p, T gx, T gy, T gz, T delta2)
{
    return (p * (T(1) - p)) * inv_mag(gx, gy, gz, delta2);
}

// Total flux on the face between cells m (low side) and c (high side) (steps 3-4):
//   F = -s u (phi_m + phi_c)/2 + gamma eps (phi_c - phi_m)/dx - gamma (q_m + q_c)/2
// hs = s/2, ge = gamma eps/dx, hg = gamma/2.
template <typename T>
__device__ __forceinline__ T face_flux(T pm, T pc, T qm, T qc, T u, T hs, T ge, T hg)
{
    const T adv = (-hs * u) * (pm + pc);
    return fma(-hg, qm + qc, fma(ge, pc - pm, adv));
}

// Divergence of the six face fluxes of a cell (step 5).
template <typename T>
__device__ __forceinline__ T flux_divergence(T fx0, T fx1, T fy0, T fy1, T fz0, T fz1, T inv_dx)
{
    return (((fx1 - fx0) + (fy1 - fy0)) + (fz1 - fz0)) * inv_dx;
}

// ---------------------------------------------------------------- adjoint (transpose) helpers
// Cotangent of the flux on the face between cells lo and hi: the flux enters f[lo] with +1/dx
// and f[hi] with -1/dx, so Fbar = (kap[lo] - kap[hi]) / dx.
template <typename T>
__device__ __forceinline__ T adj_face(T kap_lo, T kap_hi, T inv_dx)
{
    return (kap_lo - kap_hi) * inv_dx;
}

// Per-cell part of the transpose: given the stage input p and central gradient g at a cell and
// the cotangents qb of its sharpening product (qb_a = -gamma/2 (Fbar_a[low] + Fbar_a[high])),
// return gbar = (dq/dg)^T qb through n = g r, r = (|g|^2 + delta^2)^(-1/2), and the local term
// (1 - 2p)(n . qb) of d(p(1-p))/dp.
template <typename T>
__device__ __forceinline__ T adj_cell(T p, const T g[3], const T qb[3], T delta2, T gb[3])
{
    const T r = inv_mag(g[0], g[1], g[2], delta2);
    const T w = p * (T(1) - p);
    T nq = T(0), gn = T(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        nq = fma(g[b] * r, qb[b], nq);
        gn = fma(g[b], w * qb[b], gn);
    }
    const T r3gn = r * r * r * gn;
#pragma unroll
    for (int b = 0; b < 3; ++b) gb[b] = r * (w * qb[b]) - g[b] * r3gn;
    return (T(1) - T(2) * p) * nq;
}

// Global-memory access through a uniform base pointer plus a 32-bit byte offset, so the load or
// store uses the scalar-base / vector-offset addressing form with no 64-bit address arithmetic
// in vector registers. Offsets stay below 4 GiB (they never cross a plane).
template <typename T>
__device__ __forceinline__ T ldg(const T* base, unsigned byte_off)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void stg(T* base, unsigned byte_off, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// Raw buffer access: a scalar resource descriptor for one plane (base, size in bytes; range
// checked by the hardware) and a 32-bit byte offset in a vector register. No per-access
// address arithmetic in vector registers.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t plane_rsrc(const void* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ __forceinline__ float bload(rsrc_t r, unsigned off, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ double bload(rsrc_t r, unsigned off, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <typename T>
__device__ __forceinline__ T bload(rsrc_t r, unsigned off)
{
    return bload(r, off, T(0));
}
__device__ __forceinline__ void bstore(rsrc_t r, unsigned off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void bstore(rsrc_t r, unsigned off, double v)
{
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(rsrc_t(), 0, 0, 0)) u64v;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u64v, v), r, (int)off, 0, 0);
}

template <int N>
struct IntC {
    static constexpr int value = N;
};

// Periodic wrap of a plane index for the z-march: the marches reach at most 8 planes outside
// [0, n); for n >= 8 two compares suffice, smaller grids take the general modulo.
__device__ __forceinline__ int wrapz(int k, int n)
{
    if (n >= 8) return k < 0 ? k + n : (k >= n ? k - n : k);
    k %= n;
    return k < 0 ? k + n : k;
}

// Periodic wrap of an index that is at most one period out of range.
__device__ __forceinline__ int wrap1(int i, int n)
{
    i = i < 0 ? i + n : i;
    return i >= n ? i - n : i;
}

// Periodic wrap of any index (n >= 1).
__device__ __forceinline__ int wrapn(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

}  // namespace pf
