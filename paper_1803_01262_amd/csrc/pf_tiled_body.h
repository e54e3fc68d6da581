// Per-tile body of the tiled stage kernel, shared by the single-grid launch (stage_tiled.hip)
// and the batched persistent launch (batch.hip) so that both give bit-identical results.
//
// A workgroup of TX x TY threads owns the column tile [i0, i0+TX) x [j0, j0+TY) and marches the
// planes [k0, k0+KZ) along z. Per plane it keeps, in LDS, a three-plane ring of the stage input
// with a two-cell halo (the reach of the sharpening term: the normal at a face neighbour needs
// its own neighbours), and the x- and y-components of the sharpening product q = phi(1-phi)n of
// the current and next plane (with a one-cell halo in their own direction only); the
// z-component of q and the z-face flux stay in registers and are handed from one plane to the
// next. Every q is computed once per cell plus the halo ring, every face flux once per face
// except the x/y faces on the tile edge. The next plane is prefetched into registers while the
// current one is computed. Grids smaller than a tile, and ragged tiles, work through periodic
// wrapping of every load; only the writes are masked.
#pragma once

#include "pf_cell.h"
#include "pf_internal.h"

namespace pf {

template <typename T, int TX, int TY, int KZ>
__device__ __forceinline__ void tiled_stage_body(const StageArgs<T>& a, int ti, int tj, int tk)
{
    constexpr int NT = TX * TY;
    constexpr int PW = TX + 4, PH = TY + 4, PS = PW * PH;  // stage-input plane with halo 2
    constexpr int QXW = TX + 2, QXS = QXW * TY;             // q_x plane, x-halo 1
    constexpr int QYS = TX * (TY + 2);                      // q_y plane, y-halo 1
    constexpr int NL = (PS + NT - 1) / NT;                  // plane elements loaded per thread
    static_assert(NT >= 2 * TX + 2 * TY, "halo ring needs one thread per halo cell");
    __shared__ T sp[3 * PS];
    __shared__ T sqx[2 * QXS];
    __shared__ T sqy[2 * QYS];

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t plane = (size_t)nx * ny;

    const int i0 = ti * TX, j0 = tj * TY, k0 = tk * KZ;
    const int k1 = min(k0 + KZ, nz);

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool active = (i < nx) && (j < ny);
    // wrapped coordinates of this thread's column and of its +1 neighbours (face velocities)
    const int iw = wrapn(i, nx), jw = wrapn(j, ny);
    constexpr unsigned ES = sizeof(T);  // byte offsets within a plane
    const unsigned col = (unsigned)(jw * nx + iw) * ES;
    const unsigned col_xp = (unsigned)(jw * nx + wrapn(i + 1, nx)) * ES;
    const unsigned col_yp = (unsigned)(wrapn(j + 1, ny) * nx + iw) * ES;

    // fixed (x, y) sources of this thread's share of every plane load
    unsigned loff[NL];
    int lpos[NL];
#pragma unroll
    for (int s = 0; s < NL; ++s) {
        const int e = tid + s * NT;
        if (e < PS) {
            const int r = e / PW, c = e - r * PW;
            loff[s] = (unsigned)(wrapn(j0 - 2 + r, ny) * nx + wrapn(i0 - 2 + c, nx)) * ES;
            lpos[s] = e;
        } else {
            loff[s] = 0;
            lpos[s] = -1;
        }
    }
    T pre[NL];
    const unsigned pbytes = (unsigned)(plane * sizeof(T));
    auto prs = [&](const T* base, int kk) { return plane_rsrc(base + (size_t)wrapz(kk, nz) * plane, pbytes); };
    auto fetch = [&](int kk) {
        const rsrc_t r = prs(a.y, kk);
#pragma unroll
        for (int s = 0; s < NL; ++s)
            if (lpos[s] >= 0) pre[s] = bload<T>(r, loff[s]);
    };
    auto commit = [&](int slot) {
#pragma unroll
        for (int s = 0; s < NL; ++s)
            if (lpos[s] >= 0) sp[slot * PS + lpos[s]] = pre[s];
    };

    // halo-ring assignment: threads [0, 2TY) compute q_x at x = i0-1 / i0+TX for one tile row,
    // threads [2TY, 2TY+2TX) compute q_y at y = j0-1 / j0+TY for one tile column
    int h_o = -1, h_dst = 0, h_axis = 0;
    if (tid < 2 * TY) {
        const int side = tid / TY, r = tid - side * TY;
        h_o = (r + 2) * PW + (side ? TX + 2 : 1);
        h_dst = r * QXW + (side ? TX + 1 : 0);
        h_axis = 0;
    } else if (tid < 2 * TY + 2 * TX) {
        const int t2 = tid - 2 * TY;
        const int side = t2 / TX, c = t2 - side * TX;
        h_o = (side ? TY + 2 : 1) * PW + c + 2;
        h_dst = (side ? TY + 1 : 0) * TX + c;
        h_axis = 1;
    }

    const T inv_2dx = a.inv_2dx, d2 = a.delta2;
    const int o = (ty + 2) * PW + (tx + 2);  // this thread's cell in a plane of sp

    fetch(k0 - 2);
    commit(0);
    fetch(k0 - 1);
    commit(1);
    fetch(k0);

    T qz_cur = T(0), fz_prev = T(0);
    // One iteration of the march; R = (k - k0 + 2) mod 6 fixes every ring slot at compile time.
    auto iteration = [&](auto RC, int k) {
        constexpr int R = decltype(RC)::value;
        constexpr int s0 = R % 3, s1 = (R + 1) % 3, s2 = (R + 2) % 3;  // planes k, k+1, k+2
        constexpr int q0 = R & 1, q1 = (R + 1) & 1;
        __syncthreads();  // every read of the slots reused below has completed
        commit(s2);       // plane k+2
        if (k + 1 < k1) fetch(k + 3);

        // operands from global memory for this plane's outputs (issued early)
        T u0 = T(0), u1 = T(0), v0 = T(0), v1 = T(0), w1 = T(0), b1 = T(0), b2 = T(0);
        if (active) {
            w1 = bload<T>(prs(a.W, k + 1), col);
            if (k >= k0) {
                const rsrc_t rU = prs(a.U, k), rV = prs(a.V, k);
                u0 = bload<T>(rU, col);
                u1 = bload<T>(rU, col_xp);
                v0 = bload<T>(rV, col);
                v1 = bload<T>(rV, col_yp);
                if (a.out1) b1 = bload<T>(prs(a.base1, k), col);
                if (a.out2) b2 = bload<T>(prs(a.base2, k), col);
            }
        }
        __syncthreads();

        const T* P0 = sp + s0 * PS;  // plane k
        const T* P1 = sp + s1 * PS;  // plane k+1
        const T* P2 = sp + s2 * PS;  // plane k+2

        // sharpening product at plane k+1 for this thread's cell
        const T pc1 = P1[o];
        const T gx = grad1(P1[o + 1], P1[o - 1], inv_2dx);
        const T gy = grad1(P1[o + PW], P1[o - PW], inv_2dx);
        const T gz = grad1(P2[o], P0[o], inv_2dx);
        const T fac = sharpen_factor(pc1, gx, gy, gz, d2);
        sqx[q1 * QXS + ty * QXW + tx + 1] = fac * gx;
        sqy[q1 * QYS + (ty + 1) * TX + tx] = fac * gy;
        const T qz_next = fac * gz;
        // ... and on the halo ring
        if (h_o >= 0) {
            const T hgx = grad1(P1[h_o + 1], P1[h_o - 1], inv_2dx);
            const T hgy = grad1(P1[h_o + PW], P1[h_o - PW], inv_2dx);
            const T hgz = grad1(P2[h_o], P0[h_o], inv_2dx);
            const T hf = sharpen_factor(P1[h_o], hgx, hgy, hgz, d2);
            if (h_axis == 0)
                sqx[q1 * QXS + h_dst] = hf * hgx;
            else
                sqy[q1 * QYS + h_dst] = hf * hgy;
        }

        const T pc = P0[o];
        // flux through the z-face between planes k and k+1
        const T fz1 = face_flux(pc, pc1, qz_cur, qz_next, w1, a.hs, a.ge, a.hg);
        if (k >= k0 && active) {
            const T* QX = sqx + q0 * QXS + ty * QXW + tx;  // q_x at i-1, i, i+1
            const T* QY = sqy + q0 * QYS + ty * TX + tx;   // q_y at j-1, j, j+1 (stride TX)
            const T fx0 = face_flux(P0[o - 1], pc, QX[0], QX[1], u0, a.hs, a.ge, a.hg);
            const T fx1 = face_flux(pc, P0[o + 1], QX[1], QX[2], u1, a.hs, a.ge, a.hg);
            const T fy0 = face_flux(P0[o - PW], pc, QY[0], QY[TX], v0, a.hs, a.ge, a.hg);
            const T fy1 = face_flux(pc, P0[o + PW], QY[TX], QY[2 * TX], v1, a.hs, a.ge, a.hg);
            const T f = flux_divergence(fx0, fx1, fy0, fy1, fz_prev, fz1, a.inv_dx);
            if (a.out1) bstore(prs(a.out1, k), col, fma(a.c1, f, b1));
            if (a.out2) bstore(prs(a.out2, k), col, fma(a.c2, f, b2));
        }
        fz_prev = fz1;
        qz_cur = qz_next;
    };

    for (int k = k0 - 2; k < k1; k += 6) {
        iteration(IntC<0>(), k);
        if (k + 1 < k1) iteration(IntC<1>(), k + 1);
        if (k + 2 < k1) iteration(IntC<2>(), k + 2);
        if (k + 3 < k1) iteration(IntC<3>(), k + 3);
        if (k + 4 < k1) iteration(IntC<4>(), k + 4);
        if (k + 5 < k1) iteration(IntC<5>(), k + 5);
    }
}

}  // namespace pf
