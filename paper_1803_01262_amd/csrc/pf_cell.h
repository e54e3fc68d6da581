// Per-cell arithmetic of the flux-form update (Sec. 2.2, five-step recipe), shared by every
// stage-kernel variant so that all variants produce bit-identical results. The library is
// compiled with floating-point contraction off; every fused multiply-add below is explicit.
#pragma once

#include <hip/hip_runtime.h>

namespace pf {

__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }

// Central gradient component from the two neighbours along one axis (step 1).
template <typename T>
__device__ __forceinline__ T grad1(T p_plus, T p_minus, T inv_2dx)
{
    return (p_plus - p_minus) * inv_2dx;
}

// 1 / sqrt(|g|^2 + delta^2), and 0 where that vanishes: the unit normal is then 0, the
// reading of sgn(0) = 0 for a flat field (steps 1-2).
// FP32 uses the hardware reciprocal square root (1 ulp) on an argument clamped at the smallest
// normal number. The clamp keeps the result finite, so a flat cell (g = 0) still gets n = g r = 0
// without a compare; |g|^2 + delta^2 is subnormal only where phi itself is below ~1e-19, and
// there the sharpening product phi (1 - phi) n is below ~1e-19 whatever the normal.
__device__ __forceinline__ float inv_mag(float gx, float gy, float gz, float delta2)
{
    const float m2 = fmaf(gx, gx, fmaf(gy, gy, fmaf(gz, gz, delta2)));
    return __builtin_amdgcn_rsqf(fmaxf(m2, 1.17549435e-38f));
}
// FP64 computes the reciprocal square root on every lane and then selects: with a branch around
// it, waves over flat regions (g = 0) skip it, tiles there march ahead of their neighbours, and
// the halo rows the neighbours share are fetched from HBM twice instead of once from L2.
__device__ __forceinline__ double inv_mag(double gx, double gy, double gz, double delta2)
{
    const double m2 = fma(gx, gx, fma(gy, gy, fma(gz, gz, delta2)));
    const double r = rsq(m2);
    return m2 > 0.0 ? r : 0.0;
}

// Sharpening product at a cell centre (step 2), pre-scaled for the flux: returns
// hg * phi (1 - phi) / |g| with hg = gamma / (2 dx), so that q'_a = factor * g_a is the cell's
// share gamma q_a / (2 dx) of the face-averaged sharpening flux.
template <typename T>
__device__ __forceinline__ T sharpen_factor(T p, T gx, T gy, T gz, T delta2, T hg)
{
    return ((p * (T(1) - p)) * inv_mag(gx, gy, gz, delta2)) * hg;
}

// Per face, between cells lo and hi: the sum (for the face mean of phi) and the difference (for
// the diffusive flux) of the two stage-input values.
template <typename T>
__device__ __forceinline__ T face_sum(T p_lo, T p_hi) { return p_lo + p_hi; }
template <typename T>
__device__ __forceinline__ T face_diff(T p_lo, T p_hi) { return p_hi - p_lo; }

// f = d(phi)/dt at a cell (steps 3-5): the divergence of its six face fluxes
//   F_a = -s u_a (phi_lo + phi_hi)/2 + gamma eps (phi_hi - phi_lo)/dx - gamma (q_lo + q_hi)/2,
// with the fluxes of each axis' high (+) and low (-) face summed per term:
//   f = nhs * sum_a [u_a+ S_a+ - u_a- S_a-] + ge * sum_a [D_a+ - D_a-] - sum_a [q'_a+ - q'_a-]
// where S, D are the face sums and differences above, nhs = -s/(2 dx), ge = gamma eps / dx^2,
// and q'_a+ / q'_a- the pre-scaled sharpening products of the two neighbours along axis a (the
// cell's own q cancels between its two faces). Exactly the flux difference of the recipe,
// regrouped; every variant evaluates it through this one function, in this order.
template <typename T>
__device__ __forceinline__ T cell_rhs(T sxm, T sxp, T sym, T syp, T szm, T szp,
                                      T dxm, T dxp, T dym, T dyp, T dzm, T dzp,
                                      T qxm, T qxp, T qym, T qyp, T qzm, T qzp,
                                      T u0, T u1, T v0, T v1, T w0, T w1, T nhs, T ge)
{
    T adv = u1 * sxp;
    adv = fma(-u0, sxm, adv);
    adv = fma(v1, syp, adv);
    adv = fma(-v0, sym, adv);
    adv = fma(w1, szp, adv);
    adv = fma(-w0, szm, adv);
    const T dif = ((dxp - dxm) + (dyp - dym)) + (dzp - dzm);
    const T shp = ((qxp - qxm) + (qyp - qym)) + (qzp - qzm);
    return fma(nhs, adv, fma(ge, dif, -shp));
}

// f on a non-uniform rectilinear mesh: per axis the flux difference of the cell's two faces over
// the cell's width,
//   f = sum_a iw_a [ nhs (u_a+ S_a+ - u_a- S_a-) + (g_a+ D_a+ - g_a- D_a-) - (q'_a+ - q'_a-) ]
// with nhs = -s/2, g_a-/+ = gamma eps_face / (centre distance across the low/high face), q' the
// sharpening products pre-scaled by gamma/2 (the face mean stays the arithmetic mean, so the
// cell's own q cancels as on the uniform mesh) and iw_a = 1 / h_a.
template <typename T>
__device__ __forceinline__ T cell_rhs_nu(T sxm, T sxp, T sym, T syp, T szm, T szp,
                                         T dxm, T dxp, T dym, T dyp, T dzm, T dzp,
                                         T qxm, T qxp, T qym, T qyp, T qzm, T qzp,
                                         T u0, T u1, T v0, T v1, T w0, T w1, T nhs,
                                         T gxm, T gxp, T gym, T gyp, T gzm, T gzp,
                                         T iwx, T iwy, T iwz)
{
    const T ax = fma(-u0, sxm, u1 * sxp), ay = fma(-v0, sym, v1 * syp), az = fma(-w0, szm, w1 * szp);
    const T fx = fma(nhs, ax, fma(gxp, dxp, -(gxm * dxm))) - (qxp - qxm);
    const T fy = fma(nhs, ay, fma(gyp, dyp, -(gym * dym))) - (qyp - qym);
    const T fz = fma(nhs, az, fma(gzp, dzp, -(gzm * dzm))) - (qzp - qzm);
    return fma(iwx, fx, fma(iwy, fy, iwz * fz));
}

// ---------------------------------------------------------------- adjoint (transpose) helpers
// Cotangent of the flux on the face between cells lo and hi: the flux enters f[lo] with +1/dx
// and f[hi] with -1/dx, so Fbar = (kap[lo] - kap[hi]) / dx.
template <typename T>
__device__ __forceinline__ T adj_face(T kap_lo, T kap_hi, T inv_dx)
{
    return (kap_lo - kap_hi) * inv_dx;
}

// 1 / sqrt(|g|^2 + delta^2) for the transpose: as inv_mag, but 0 wherever the argument is below
// the smallest normal number. The forward's clamp gives such a cell a finite but huge r (up to
// 2^63), harmless there because the sharpening product multiplies it by phi (1 - phi) ~ |g| dx;
// the transpose would multiply it by the cotangent, so r = 0 instead: the normal and its
// derivative vanish, as for a flat cell (g = 0) in FP64.
__device__ __forceinline__ float inv_mag_adj(float gx, float gy, float gz, float delta2)
{
    const float m2 = fmaf(gx, gx, fmaf(gy, gy, fmaf(gz, gz, delta2)));
    return m2 >= 1.17549435e-38f ? __builtin_amdgcn_rsqf(m2) : 0.0f;
}
__device__ __forceinline__ double inv_mag_adj(double gx, double gy, double gz, double delta2)
{
    return inv_mag(gx, gy, gz, delta2);
}

// Per-cell part of the transpose: given the stage input p and central gradient g at a cell and
// the cotangents qb of its sharpening product (qb_a = -gamma/2 (Fbar_a[low] + Fbar_a[high])),
// return gbar = (dq/dg)^T qb through n = g r, r = (|g|^2 + delta^2)^(-1/2), and the local term
// (1 - 2p)(n . qb) of d(p(1-p))/dp. With nbar = p (1 - p) qb,
//   gbar_b = sum_a (r delta_ab - g_a g_b r^3) nbar_a = r (nbar_b - n_b (n . nbar)),
// written with n = g r so that r^3 is never formed (it overflows FP32 where |g| is tiny).
template <typename T>
__device__ __forceinline__ T adj_cell(T p, const T g[3], const T qb[3], T delta2, T gb[3])
{
    const T r = inv_mag_adj(g[0], g[1], g[2], delta2);
    const T w = p * (T(1) - p);
    T n[3];
    T nq = T(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        n[b] = g[b] * r;
        nq = fma(n[b], qb[b], nq);
    }
    const T wnq = w * nq;
#pragma unroll
    for (int b = 0; b < 3; ++b) gb[b] = r * fma(-n[b], wnq, w * qb[b]);
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

__device__ __forceinline__ float bload_so(rsrc_t r, unsigned off, unsigned soff, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, 0));
}
__device__ __forceinline__ double bload_so(rsrc_t r, unsigned off, unsigned soff, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, 0));
}
__device__ __forceinline__ void bstore_so(rsrc_t r, unsigned off, unsigned soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, (int)soff, 0);
}
__device__ __forceinline__ void bstore_so(rsrc_t r, unsigned off, unsigned soff, double v)
{
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(rsrc_t(), 0, 0, 0)) u64v;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u64v, v), r, (int)off, (int)soff, 0);
}

// 16 bytes of a field (four floats or two doubles), moved as one unit.
typedef int v4i_t __attribute__((ext_vector_type(4)));

// One field (an array of nz planes) for the z-marches. Element (plane kw, byte offset off in
// the plane) is addressed with one descriptor for the whole array, the plane offset kw * pbytes
// in the scalar soffset operand and off in a vector register. Arrays of 4 GiB or more (BIG)
// take a descriptor per plane instead, since buffer offsets are 32-bit.
template <typename T, bool BIG>
struct FieldRef {
    const T* base;
    rsrc_t whole;
    unsigned pbytes;
    size_t pelems;
    __device__ __forceinline__ FieldRef(const T* b, size_t plane_elems, int nplanes)
        : base(b), pbytes((unsigned)(plane_elems * sizeof(T))), pelems(plane_elems)
    {
        whole = plane_rsrc(b, BIG ? 0u : (unsigned)(plane_elems * sizeof(T) * (size_t)nplanes));
    }
    __device__ __forceinline__ T load(int kw, unsigned off) const
    {
        if constexpr (BIG)
            return bload<T>(plane_rsrc(base + (size_t)kw * pelems, pbytes), off);
        else
            return bload_so(whole, off, (unsigned)kw * pbytes, T(0));
    }
    // 16 bytes at (plane kw, byte offset off); off must be a multiple of 16
    __device__ __forceinline__ v4i_t load16(int kw, unsigned off) const
    {
        if constexpr (BIG)
            return __builtin_amdgcn_raw_buffer_load_b128(plane_rsrc(base + (size_t)kw * pelems, pbytes),
                                                         (int)off, 0, 0);
        else
            return __builtin_amdgcn_raw_buffer_load_b128(whole, (int)off, (int)((unsigned)kw * pbytes), 0);
    }
    __device__ __forceinline__ void store(int kw, unsigned off, T v) const
    {
        if constexpr (BIG)
            bstore(plane_rsrc(base + (size_t)kw * pelems, pbytes), off, v);
        else
            bstore_so(whole, off, (unsigned)kw * pbytes, v);
    }
};

// Periodic wrap of a plane index for the z-march: the marches (with the iterations that pad a
// chunk to whole groups of six) reach at most 10 planes outside [0, n); for n >= 16 two compares
// suffice, smaller grids take the general modulo.
__device__ __forceinline__ int wrapz(int k, int n)
{
    if (n >= 16) return k < 0 ? k + n : (k >= n ? k - n : k);
    k %= n;
    return k < 0 ? k + n : k;
}

// XCD-aware tile order. Consecutive workgroup ids are dispatched round-robin over the 8 XCDs, so
// workgroup b runs on XCD b mod 8; this maps the ids onto [0, nb) such that each XCD takes one
// contiguous range of tile indices (nb/8 of them, one more for the first nb mod 8 XCDs), and the
// halo rows that neighbouring tiles share stay in that XCD's L2.
__device__ __forceinline__ int xcd_tile_order(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
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

// Mirror index across walls at 0 and n (any index, n >= 1): the ghost of cell -1 is cell 0, of
// -2 cell 1, of n cell n-1; equivalently, the index on a periodic axis of 2n cells holding the
// data and its mirror image.
__device__ __forceinline__ int reflectn(int i, int n)
{
    const int m2 = 2 * n;
    int m = i % m2;
    m = m < 0 ? m + m2 : m;
    return m < n ? m : m2 - 1 - m;
}

// The same for a z-march plane index, which lies at most 10 planes outside [0, n) (see wrapz):
// for n >= 16 two compares suffice.
__device__ __forceinline__ int reflectz(int k, int n)
{
    if (n >= 16) return k < 0 ? -k - 1 : (k >= n ? 2 * n - 1 - k : k);
    return reflectn(k, n);
}

}  // namespace pf
