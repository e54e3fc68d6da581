// Adjoint of one explicit stage: ybar = (df/dy)^T kap, gathered per cell, plus the face-velocity
// gradient (df/dU)^T kap. f is the flux-form right-hand side of Eq. 1 (Sec. 2.2 recipe); its
// transpose runs the recipe backwards:
//   step 5^T: Fbar_a on the low face of c        = (kap[c - e_a] - kap[c]) / dx
//   step 4^T: phi through the face interpolation and the diffusive difference;
//             qbar_a[c]                          = -gamma/2 (Fbar_a[c] + Fbar_a[c + e_a]);
//             Ubar_a[c]                         += -s/2 (y[c - e_a] + y[c]) Fbar_a[c]
//   step 3^T: q = w n with w = y (1 - y):   ybar += (1 - 2y)(n . qbar);  nbar = w qbar
//   step 2^T: n = g r, r = (|g|^2 + delta^2)^(-1/2):   gbar = r (nbar - r^2 g (g . nbar))
//   step 1^T: g_a = (y[c + e_a] - y[c - e_a]) / (2 dx):  ybar[c] += (gbar_a[c - e_a] - gbar_a[c + e_a]) / (2 dx)
// The cotangent stencil has the same 25-point reach as the forward stencil.
#include "pf_cell.h"
#include "pf_internal.h"

namespace pf {

template <typename T>
__global__ void __launch_bounds__(256) adjoint_stage_kernel(AdjArgs<T> a)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= a.nx || j >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    auto idx = [&](int di, int dj, int dk) -> size_t {
        return ((size_t)wrapn(k + dk, nz) * ny + wrapn(j + dj, ny)) * nx + wrapn(i + di, nx);
    };
    auto Y = [&](int di, int dj, int dk) -> T { return a.y[idx(di, dj, dk)]; };
    auto K = [&](int di, int dj, int dk) -> T { return a.kap_scale * a.kap_in[idx(di, dj, dk)]; };
    // cotangent of the flux on the low ax-face of cell (di, dj, dk)
    auto Fb = [&](int di, int dj, int dk, int ax) -> T {
        return (K(di - (ax == 0), dj - (ax == 1), dk - (ax == 2)) - K(di, dj, dk)) * a.inv_dx;
    };
    // gbar (all three components) and the local (1-2y)(n.qbar) term of cell (di, dj, dk)
    auto cell = [&](int di, int dj, int dk, T gb[3], T& local) {
        const T p = Y(di, dj, dk);
        T g[3];
        g[0] = grad1(Y(di + 1, dj, dk), Y(di - 1, dj, dk), a.inv_2dx);
        g[1] = grad1(Y(di, dj + 1, dk), Y(di, dj - 1, dk), a.inv_2dx);
        g[2] = grad1(Y(di, dj, dk + 1), Y(di, dj, dk - 1), a.inv_2dx);
        const T r = inv_mag(g[0], g[1], g[2], a.delta2);
        const T w = p * (T(1) - p);
        T qb[3];
        qb[0] = -a.hg * (Fb(di, dj, dk, 0) + Fb(di + 1, dj, dk, 0));
        qb[1] = -a.hg * (Fb(di, dj, dk, 1) + Fb(di, dj + 1, dk, 1));
        qb[2] = -a.hg * (Fb(di, dj, dk, 2) + Fb(di, dj, dk + 1, 2));
        T nq = T(0), gn = T(0);
        for (int b = 0; b < 3; ++b) {
            nq = fma(g[b] * r, qb[b], nq);
            gn = fma(g[b], w * qb[b], gn);
        }
        local = (T(1) - T(2) * p) * nq;
        const T r3gn = r * r * r * gn;
        for (int b = 0; b < 3; ++b) gb[b] = r * (w * qb[b]) - g[b] * r3gn;
    };

    const size_t c = idx(0, 0, 0);
    const T yc = a.y[c];
    T gbc[3], local;
    cell(0, 0, 0, gbc, local);
    T ybar = local;
    const T* vel[3] = {a.U, a.V, a.W};
    T* velbar[3] = {a.gU, a.gV, a.gW};
    for (int ax = 0; ax < 3; ++ax) {
        const int ex = ax == 0, ey = ax == 1, ez = ax == 2;
        // the two faces of this cell along ax
        const T fb_lo = Fb(0, 0, 0, ax);
        const T fb_hi = Fb(ex, ey, ez, ax);
        const T u_lo = vel[ax][c];
        const T u_hi = vel[ax][idx(ex, ey, ez)];
        ybar = fma(fb_lo, fma(-a.hs, u_lo, a.ge), ybar);
        ybar = fma(fb_hi, fma(-a.hs, u_hi, -a.ge), ybar);
        if (velbar[ax]) velbar[ax][c] = fma(-a.hs * (Y(-ex, -ey, -ez) + yc), fb_lo, velbar[ax][c]);
        // gradient transpose from the two neighbours along ax
        T gbm[3], gbp[3], dummy;
        cell(-ex, -ey, -ez, gbm, dummy);
        cell(ex, ey, ez, gbp, dummy);
        ybar = fma(gbm[ax] - gbp[ax], a.inv_2dx, ybar);
    }
    if (a.lam_out) a.lam_out[c] = a.lam_base[c] + ybar;
    if (a.kap_out) a.kap_out[c] = fma(a.ka, ybar, a.kb * a.lamp[c]);
}

template <typename T>
hipError_t launch_adjoint_stage(const AdjArgs<T>& a, hipStream_t st)
{
    dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4, a.nz);
    hipLaunchKernelGGL(adjoint_stage_kernel<T>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

template hipError_t launch_adjoint_stage<float>(const AdjArgs<float>&, hipStream_t);
template hipError_t launch_adjoint_stage<double>(const AdjArgs<double>&, hipStream_t);

}  // namespace pf
