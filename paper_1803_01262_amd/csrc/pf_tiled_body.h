// Per-tile body of the tiled stage kernel, shared by the single-grid launch (stage_tiled.hip)
// and the batched persistent launch (batch.hip) so that both give bit-identical results.
//
// A workgroup of TX x TY threads owns the column tile [i0, i0+TX) x [j0, j0+TY) and marches the
// planes [k0, k1) along z. Per plane it keeps, in LDS, a three-plane ring of the stage input
// with a two-cell halo (the reach of the sharpening term: the normal at a face neighbour needs
// its own neighbours), and the x- and y-components of the sharpening product q = phi(1-phi)n of
// the current and next plane (with a one-cell halo in their own direction only); the
// z-components of q of the planes below and above, the z-face sum and difference of phi and
// the z-face velocity stay in registers and are handed from one plane to the next. Every q is
// computed once per cell plus the halo ring. The next plane is prefetched into registers while
// the current one is computed. Grids smaller than a tile, and ragged tiles, work through periodic
// wrapping of every load; only the writes are masked.
//
// Global memory is read and written through buffer descriptors (FieldRef): one per array, the
// plane offset in a scalar register, so no address arithmetic runs in vector registers. BIG
// selects the per-plane descriptor form needed for arrays of 4 GiB or more. WALLS selects the
// form with solid walls on the axes flagged in a.walls: the stage input is read through mirror
// indices there (so the diffusive and sharpening fluxes through a wall face vanish) and the face
// velocity at index 0 of a walled axis counts as zero. NU selects the non-uniform rectilinear
// mesh (a.nu): the gradient, the diffusive fluxes and the divergence take their coefficients from
// the per-axis tables (this thread's column and row once, the planes' per iteration), and eps
// mode 1 scales the diffusive flux of each face by the mean of its two cells' largest widths.
#pragma once

#include "pf_cell.h"
#include "pf_internal.h"

namespace pf {

template <typename T, int TX, int TY, bool BIG, bool WALLS = false, bool PREFETCH = false,
          bool NU = false>
__device__ __forceinline__ void tiled_stage_body(const StageArgs<T>& a, int ti, int tj, int k0, int k1)
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

    const int i0 = ti * TX, j0 = tj * TY;
    const bool wx = WALLS && (a.walls & 1), wy = WALLS && (a.walls & 2), wz = WALLS && (a.walls & 4);
    // stage-input index maps: periodic wrap, or the mirror across walls
    auto mapx = [&](int v) { return WALLS && wx ? reflectn(v, nx) : wrapn(v, nx); };
    auto mapy = [&](int v) { return WALLS && wy ? reflectn(v, ny) : wrapn(v, ny); };
    auto mapz = [&](int v) { return WALLS && wz ? reflectz(v, nz) : wrapz(v, nz); };

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
            loff[s] = (unsigned)(mapy(j0 - 2 + r) * nx + mapx(i0 - 2 + c)) * ES;
            lpos[s] = e;
        } else {
            loff[s] = 0;
            lpos[s] = -1;
        }
    }
    T pre[NL];
    const FieldRef<T, BIG> fy(a.y, plane, nz), fU(a.U, plane, nz), fV(a.V, plane, nz),
        fW(a.W, plane, nz), fb1(a.base1, plane, nz), fb2(a.base2, plane, nz),
        fo1(a.out1, plane, nz), fo2(a.out2, plane, nz);
    auto fetch = [&](int kk) {
        const int kw = mapz(kk);
#pragma unroll
        for (int s = 0; s < NL; ++s)
            if (lpos[s] >= 0) pre[s] = fy.load(kw, loff[s]);
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

    const T inv_2dx = a.inv_2dx, d2 = a.delta2, hg = NU ? a.nu_hg : a.hg, nhs = a.nhs, ge = a.ge;
    const int o = (ty + 2) * PW + (tx + 2);  // this thread's cell in a plane of sp

    // non-uniform mesh: gradient spans of this thread's cell and of its halo cell, the column's
    // and row's divergence and face coefficients, and the widths around the cell (eps mode 1)
    T sgx = inv_2dx, sgy = inv_2dx, hsgx = inv_2dx, hsgy = inv_2dx;
    T iwx = T(0), iwy = T(0), dxl = T(0), dxh = T(0), dyl = T(0), dyh = T(0);
    T hxm = T(0), hxc = T(0), hxp = T(0), hym = T(0), hyc = T(0), hyp = T(0);
    if constexpr (NU) {
        const T* X = a.nu[0];
        const T* Y = a.nu[1];
        const int cx = mapx(i) * kNuCols, cxm = mapx(i - 1) * kNuCols, cxp = mapx(i + 1) * kNuCols;
        const int cy = mapy(j) * kNuCols, cym = mapy(j - 1) * kNuCols, cyp = mapy(j + 1) * kNuCols;
        sgx = X[cx + kNuInvSpan];
        sgy = Y[cy + kNuInvSpan];
        iwx = X[cx + kNuInvW];
        iwy = Y[cy + kNuInvW];
        dxl = X[cx + kNuInvDist];
        dxh = X[cxp + kNuInvDist];  // the high face is the low face of cell i+1
        dyl = Y[cy + kNuInvDist];
        dyh = Y[cyp + kNuInvDist];
        hxm = X[cxm + kNuWidth];
        hxc = X[cx + kNuWidth];
        hxp = X[cxp + kNuWidth];
        hym = Y[cym + kNuWidth];
        hyc = Y[cy + kNuWidth];
        hyp = Y[cyp + kNuWidth];
        if (h_o >= 0) {  // the halo cell: column i0-1 / i0+TX on a tile row, or row j0-1 / j0+TY
            int hi, hj;
            if (h_axis == 0) {
                const int side = tid / TY;
                hi = side ? i0 + TX : i0 - 1;
                hj = j0 + (tid - side * TY);
            } else {
                const int t2 = tid - 2 * TY, side = t2 / TX;
                hi = i0 + (t2 - side * TX);
                hj = side ? j0 + TY : j0 - 1;
            }
            hsgx = X[mapx(hi) * kNuCols + kNuInvSpan];
            hsgy = Y[mapy(hj) * kNuCols + kNuInvSpan];
        }
    }

    fetch(k0 - 2);
    commit(0);
    fetch(k0 - 1);
    commit(1);
    fetch(k0);

    // z state handed from plane to plane: q_z at k-1 and k, the face (k-1, k) and W at k
    T qz_m1 = T(0), qz_cur = T(0), szm = T(0), dzm = T(0), w0 = T(0);
    // the per-cell operands of iteration k (W at plane k+1; U, V and the bases at plane k); lanes
    // outside the grid read their wrapped column, in bounds, and store nothing. PREFETCH loads
    // them one iteration ahead, so that their latency spans a whole iteration (long chunks: at
    // 512^3 FP32 on 64x4 tiles 3.35 against 3.91 ms per step); otherwise each iteration loads its
    // own after its first barrier (short chunks, where the extra load round in front of the
    // march costs more than it hides: 64^3 and 32^3 about 5 % faster this way)
    T nw1, nu0, nu1, nv0, nv1, nb1, nb2;
    auto load_ops = [&](int k) {
        const int kw1 = wrapz(k + 1, nz);
        nw1 = fW.load(kw1, col);
        if (WALLS && wz && kw1 == 0) nw1 = T(0);  // a wall face
        if (k >= k0 && k < k1) {
            nu0 = fU.load(k, col);
            nu1 = fU.load(k, col_xp);
            nv0 = fV.load(k, col);
            nv1 = fV.load(k, col_yp);
            if constexpr (WALLS) {  // velocities on wall faces (index 0 of a walled axis)
                if (wx && iw == 0) nu0 = T(0);
                if (wx && iw == nx - 1) nu1 = T(0);
                if (wy && jw == 0) nv0 = T(0);
                if (wy && jw == ny - 1) nv1 = T(0);
            }
            if (a.out1) nb1 = fb1.load(k, col);
            if (a.out2) nb2 = fb2.load(k, col);
        }
    };
    if constexpr (PREFETCH) load_ops(k0 - 2);
    // One iteration of the march; R = (k - k0 + 2) mod 6 fixes every ring slot at compile time.
    // The march runs in whole groups of six unconditional iterations (so the values handed from
    // plane to plane stay in place); iterations past the chunk end only compute, on wrapped
    // planes, and store nothing.
    auto iteration = [&](auto RC, int k) {
        constexpr int R = decltype(RC)::value;
        constexpr int s0 = R % 3, s1 = (R + 1) % 3, s2 = (R + 2) % 3;  // planes k, k+1, k+2
        constexpr int q0 = R & 1, q1 = (R + 1) & 1;
        __syncthreads();  // every read of the slots reused below has completed
        commit(s2);       // plane k+2
        fetch(k + 3);
        const bool out_plane = k >= k0 && k < k1;
        if constexpr (!PREFETCH) load_ops(k);
        const T w1 = nw1, u0 = nu0, u1 = nu1, v0 = nv0, v1 = nv1, b1 = nb1, b2 = nb2;
        if constexpr (PREFETCH) load_ops(k + 1);
        // non-uniform mesh: the z coefficients of planes k and k+1 (scalar loads)
        T sgz = inv_2dx, iwz = T(0), dzl = T(0), dzh = T(0), hzm = T(0), hzc = T(0), hzp = T(0);
        if constexpr (NU) {
            const T* Z = a.nu[2];
            const int zc = mapz(k) * kNuCols, zp = mapz(k + 1) * kNuCols;
            sgz = Z[zp + kNuInvSpan];  // the gradient of plane k+1
            iwz = Z[zc + kNuInvW];
            dzl = Z[zc + kNuInvDist];
            dzh = Z[zp + kNuInvDist];
            hzm = Z[mapz(k - 1) * kNuCols + kNuWidth];
            hzc = Z[zc + kNuWidth];
            hzp = Z[zp + kNuWidth];
        }
        __syncthreads();

        const T* P0 = sp + s0 * PS;  // plane k
        const T* P1 = sp + s1 * PS;  // plane k+1
        const T* P2 = sp + s2 * PS;  // plane k+2

        // sharpening product at plane k+1 for this thread's cell
        const T pc1 = P1[o];
        const T gx = grad1(P1[o + 1], P1[o - 1], sgx);
        const T gy = grad1(P1[o + PW], P1[o - PW], sgy);
        const T gz = grad1(P2[o], P0[o], sgz);
        const T fac = sharpen_factor(pc1, gx, gy, gz, d2, hg);
        sqx[q1 * QXS + ty * QXW + tx + 1] = fac * gx;
        sqy[q1 * QYS + (ty + 1) * TX + tx] = fac * gy;
        const T qz_next = fac * gz;
        // ... and on the halo ring
        if (h_o >= 0) {
            const T hgx = grad1(P1[h_o + 1], P1[h_o - 1], hsgx);
            const T hgy = grad1(P1[h_o + PW], P1[h_o - PW], hsgy);
            const T hgz = grad1(P2[h_o], P0[h_o], sgz);
            const T hf = sharpen_factor(P1[h_o], hgx, hgy, hgz, d2, hg);
            if (h_axis == 0)
                sqx[q1 * QXS + h_dst] = hf * hgx;
            else
                sqy[q1 * QYS + h_dst] = hf * hgy;
        }

        const T pc = P0[o];
        // z-face between planes k and k+1
        const T szp = face_sum(pc, pc1), dzp = face_diff(pc, pc1);
        if (out_plane && active) {
            const T* QX = sqx + q0 * QXS + ty * QXW + tx;  // q_x at i-1, i, i+1
            const T* QY = sqy + q0 * QYS + ty * TX + tx;   // q_y at j-1, j, j+1 (stride TX)
            const T pxm = P0[o - 1], pxp = P0[o + 1], pym = P0[o - PW], pyp = P0[o + PW];
            T f;
            if constexpr (NU) {
                // diffusive coefficients of the six faces: gamma eps_face / centre distance
                T exl = a.nu_ge, exh = a.nu_ge, eyl = a.nu_ge, eyh = a.nu_ge, ezl = a.nu_ge,
                  ezh = a.nu_ge;
                if (a.nu_eps_mode == 1) {  // eps of a cell ~ its largest width
                    const T mc = fmax(hxc, fmax(hyc, hzc));
                    const T hh = a.nu_ge * T(0.5);
                    exl = hh * (fmax(hxm, fmax(hyc, hzc)) + mc);
                    exh = hh * (fmax(hxp, fmax(hyc, hzc)) + mc);
                    eyl = hh * (fmax(hxc, fmax(hym, hzc)) + mc);
                    eyh = hh * (fmax(hxc, fmax(hyp, hzc)) + mc);
                    ezl = hh * (fmax(hxc, fmax(hyc, hzm)) + mc);
                    ezh = hh * (fmax(hxc, fmax(hyc, hzp)) + mc);
                }
                f = cell_rhs_nu(face_sum(pxm, pc), face_sum(pc, pxp), face_sum(pym, pc),
                                face_sum(pc, pyp), szm, szp, face_diff(pxm, pc), face_diff(pc, pxp),
                                face_diff(pym, pc), face_diff(pc, pyp), dzm, dzp, QX[0], QX[2],
                                QY[0], QY[2 * TX], qz_m1, qz_next, u0, u1, v0, v1, w0, w1,
                                a.nu_nhs, exl * dxl, exh * dxh, eyl * dyl, eyh * dyh, ezl * dzl,
                                ezh * dzh, iwx, iwy, iwz);
            } else {
                f = cell_rhs(face_sum(pxm, pc), face_sum(pc, pxp), face_sum(pym, pc),
                             face_sum(pc, pyp), szm, szp, face_diff(pxm, pc), face_diff(pc, pxp),
                             face_diff(pym, pc), face_diff(pc, pyp), dzm, dzp, QX[0], QX[2],
                             QY[0], QY[2 * TX], qz_m1, qz_next, u0, u1, v0, v1, w0, w1, nhs, ge);
            }
            if (a.out1) fo1.store(k, col, fma(a.c1, f, b1));
            if (a.out2) fo2.store(k, col, fma(a.c2, f, b2));
        }
        szm = szp;
        dzm = dzp;
        qz_m1 = qz_cur;
        qz_cur = qz_next;
        w0 = w1;
    };

    const int kend = k0 - 2 + 6 * ((k1 - k0 + 7) / 6);  // k0-2 .. k1-1, in groups of six
    for (int k = k0 - 2; k < kend; k += 6) {
        iteration(IntC<0>(), k);
        iteration(IntC<1>(), k + 1);
        iteration(IntC<2>(), k + 2);
        iteration(IntC<3>(), k + 3);
        iteration(IntC<4>(), k + 4);
        iteration(IntC<5>(), k + 5);
    }
}

}  // namespace pf
