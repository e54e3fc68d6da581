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
