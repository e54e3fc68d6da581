// Two reverse RK4 stages in one z-march (the adjoint's counterpart of the fused forward sweeps).
//
// The reverse sweep of a classic RK4 step (api_adjoint.cpp) runs stage 4, 3, 2, 1 in turn; each
// reverse stage s gathers ybar_s = (df/dy at y_s)^T kap_s, adds it to the step's cotangent
// accumulator L, forms the next stage's cotangent kap = kb lam' + ka ybar_s and adds the stage's
// face-velocity gradient. Run as four launches it moves about 15 words per cell and stage. Here
// two consecutive stages H (4, then 2) and L (3, then 1) share one sweep:
//   E1: ybar_H on the tile plus a two-cell halo (the reach of the transposed stencil), from y_H
//       and kap_H = kscale * src_H (both read with a four-cell halo), plane by plane; it forms
//       kap_L = kb_L lam' + ka_L ybar_H into an LDS ring, and for the tile's own cells the
//       partial sums (base + ybar_H, and the gradients plus stage H's contribution).
//   E2: ybar_L at the tile, from y_L (two-cell halo) and kap_L, two planes behind E1; it
//       finishes the partial sums and writes them once: L_out = (base + ybar_H) + ybar_L,
//       optionally kout = ka_o ybar_L + kb_o lam' (the next pair's source), and the gradients.
// Every operation has the order and precision of the single-stage kernel (adjoint.hip), so the
// pair is bit-identical to two single-stage launches. Per RK4 reverse step: pair (4, 3) reads y4,
// lam' (stencil), y3, U, V, W and the gradients, writes L, kap_2, a copy of lam' and the
// gradients (15 words); pair (2, 1) reads y2, kap_2 (stencil), phi, the copy of lam', L, U, V, W
// and the gradients, writes lam and the gradients (15 words): 30 words instead of about 60.
//
// Regions for a TX x TY tile at (i0, j0), as (x range) x (y range):
//   IN   y_H and kap_H, rings of 3 planes     [i0-4, i0+TX+4) x [j0-4, j0+TY+4)
//   MID  E1 cells; y_L and kap_L rings of 3 planes, lam' (1 plane)   [i0-2, i0+TX+2) x [j0-2, j0+TY+2)
//   G1X  gbar_x of E1, 2 planes               [i0-3, i0+TX+3) x [j0-2, j0+TY+2)
//   G1Y  gbar_y of E1, 2 planes               [i0-2, i0+TX+2) x [j0-3, j0+TY+3)
//   G2X  gbar_x of E2, 2 planes               [i0-1, i0+TX+1) x [j0, j0+TY)
//   G2Y  gbar_y of E2, 2 planes               [i0, i0+TX) x [j0-1, j0+TY+1)
// Pipeline: iteration t commits input plane t+4; E1 computes gbar_H at plane t+3 and finishes
// ybar_H at plane t+2; E2 computes gbar_L at plane t+1 and finishes ybar_L at plane t. A z-chunk
// [k0, k1) starts at t = k0-8 (E1 from plane k0-3, E2 from k0-2; the first output plane needs
// both stages' state of the planes below it) and runs in whole groups of six iterations, so the
// ring slots are compile-time constants; iterations past the chunk end store nothing.
#include <type_traits>

#include "pf_cell.h"
#include "pf_internal.h"

namespace pf {

template <typename T, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
adjoint_pair_kernel(AdjPairArgs<T> a, int tiles_x, int tiles_y, int kz)
{
    constexpr int NT = TX * TY;
    constexpr int INW = TX + 8, INH = TY + 8, INS = INW * INH;
    constexpr int MW = TX + 4, MH = TY + 4, MS = MW * MH;
    constexpr int G1XW = TX + 6, G1XS = G1XW * MH;
    constexpr int G1YS = MW * (TY + 6);
    constexpr int G2XW = TX + 2, G2XS = G2XW * TY;
    constexpr int G2YS = TX * (TY + 2);
    constexpr int NRING = 4 * MW + 4 * TY;  // MID cells outside the tile
    constexpr int NOUT = 2 * MH + 2 * MW;   // gbar_H-only cells (x- and y-outer ring)
    constexpr int NH2 = 2 * TX + 2 * TY;    // gbar_L halo cells
    constexpr int OUT0 = (NRING + 63) / 64 * 64;
    constexpr int NLI = (INS + NT - 1) / NT;
    constexpr int NLM = (MS + NT - 1) / NT;
    static_assert(OUT0 + NOUT <= NT, "tile too small for the E1 halo assignment");
    static_assert(NH2 <= NT, "tile too small for the E2 halo assignment");

    __shared__ T s_yh[3 * INS];
    __shared__ T s_kh[3 * INS];
    __shared__ T s_yl[3 * MS];
    __shared__ T s_kl[3 * MS];
    __shared__ T s_lp[MS];
    __shared__ T s_g1x[2 * G1XS];
    __shared__ T s_g1y[2 * G1YS];
    __shared__ T s_g2x[2 * G2XS];
    __shared__ T s_g2y[2 * G2YS];

    int bid = xcd_tile_order(blockIdx.x, gridDim.x);
    const int ti = bid % tiles_x;
    bid /= tiles_x;
    const int tj = bid % tiles_y;
    const int k0 = (bid / tiles_y) * kz;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int k1 = min(k0 + kz, nz);
    const size_t plane = (size_t)nx * ny;
    const int i0 = ti * TX, j0 = tj * TY;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const bool active = (i0 + tx < nx) && (j0 + ty < ny);
    const T inv_dx = a.inv_dx, inv_2dx = a.inv_2dx, d2 = a.delta2, hg = a.hg, ge = a.ge;
    const T hsH = a.hsH, hsL = a.hsL;

    // ---- E1 slots: slot 0 = own cell, slot 1 = a MID ring cell (tid < NRING)
    int e_lx[2], e_ly[2];
    e_lx[0] = tx + 2;
    e_ly[0] = ty + 2;
    const bool has_ring = tid < NRING;
    {
        int r = has_ring ? tid : 0, lx, ly;
        if (r < 2 * MW) {
            ly = r / MW;
            lx = r - ly * MW;
        } else if (r < 4 * MW) {
            const int r2 = r - 2 * MW;
            ly = TY + 2 + r2 / MW;
            lx = r2 % MW;
        } else {
            const int r3 = r - 4 * MW;
            ly = 2 + r3 / 4;
            const int c = r3 % 4;
            lx = c < 2 ? c : TX + c;
        }
        e_lx[1] = lx;
        e_ly[1] = ly;
    }
    constexpr unsigned ES = sizeof(T);
    unsigned e_col[2], e_colx[2], e_coly[2];
    for (int s = 0; s < 2; ++s) {
        const int gx = wrapn(i0 - 2 + e_lx[s], nx), gy = wrapn(j0 - 2 + e_ly[s], ny);
        e_col[s] = (unsigned)(gy * nx + gx) * ES;
        e_colx[s] = (unsigned)(gy * nx + wrapn(gx + 1, nx)) * ES;
        e_coly[s] = (unsigned)(wrapn(gy + 1, ny) * nx + gx) * ES;
    }
    // ---- gbar_H-only cell (x-outer: G1X columns 0 and TX+5; y-outer: G1Y rows 0 and TY+5)
    const int ro = tid - OUT0;
    const bool has_out = ro >= 0 && ro < NOUT;
    int o_in = 0, o_dst = 0, o_axis = 0;
    if (has_out) {
        if (ro < 2 * MH) {
            const int side = ro / MH, ry = ro - side * MH;
            o_in = (side ? TX + 6 : 1) + (ry + 2) * INW;
            o_dst = (side ? TX + 5 : 0) + ry * G1XW;
            o_axis = 0;
        } else {
            const int r2 = ro - 2 * MH;
            const int side = r2 / MW, cx = r2 - side * MW;
            o_in = (cx + 2) + (side ? TY + 6 : 1) * INW;
            o_dst = cx + (side ? TY + 5 : 0) * MW;
            o_axis = 1;
        }
    }
    // ---- gbar_L halo cell (threads at the top of the block)
    const int rh = tid - (NT - NH2);
    const bool has_h2 = rh >= 0;
    int h_om = 0, h_dst = 0, h_axis = 0;
    if (has_h2) {
        if (rh < 2 * TY) {
            const int side = rh / TY, r = rh - side * TY;
            h_om = (side ? TX + 2 : 1) + (r + 2) * MW;
            h_dst = (side ? TX + 1 : 0) + r * G2XW;
            h_axis = 0;
        } else {
            const int r2 = rh - 2 * TY;
            const int side = r2 / TX, c = r2 - side * TX;
            h_om = (c + 2) + (side ? TY + 2 : 1) * MW;
            h_dst = c + (side ? TY + 1 : 0) * TX;
            h_axis = 1;
        }
    }

    // ---- plane loads: IN (y_H, src_H) and MID (y_L, lam')
    unsigned li_off[NLI];
    int li_pos[NLI];
#pragma unroll
    for (int s = 0; s < NLI; ++s) {
        const int e = tid + s * NT;
        const int r = e / INW, c = e - r * INW;
        li_pos[s] = e < INS ? e : -1;
        li_off[s] = e < INS ? (unsigned)(wrapn(j0 - 4 + r, ny) * nx + wrapn(i0 - 4 + c, nx)) * ES : 0u;
    }
    unsigned lm_off[NLM];
    int lm_pos[NLM];
#pragma unroll
    for (int s = 0; s < NLM; ++s) {
        const int e = tid + s * NT;
        const int r = e / MW, c = e - r * MW;
        lm_pos[s] = e < MS ? e : -1;
        lm_off[s] = e < MS ? (unsigned)(wrapn(j0 - 2 + r, ny) * nx + wrapn(i0 - 2 + c, nx)) * ES : 0u;
    }
    const FieldRef<T, false> fyh(a.yH, plane, nz), fsrc(a.srcH, plane, nz), fyl(a.yL, plane, nz),
        flp(a.lamp, plane, nz), fU(a.U, plane, nz), fV(a.V, plane, nz), fW(a.W, plane, nz);
    T pre_yh[NLI], pre_kh[NLI], pre_yl[NLM], pre_lp[NLM];
    auto fetch_in = [&](int kk) {
        const int kw = wrapz(kk, nz);
#pragma unroll
        for (int s = 0; s < NLI; ++s)
            if (li_pos[s] >= 0) {
                pre_yh[s] = fyh.load(kw, li_off[s]);
                pre_kh[s] = a.kscaleH * fsrc.load(kw, li_off[s]);
            }
    };
    auto commit_in = [&](int slot) {
#pragma unroll
        for (int s = 0; s < NLI; ++s)
            if (li_pos[s] >= 0) {
                s_yh[slot * INS + li_pos[s]] = pre_yh[s];
                s_kh[slot * INS + li_pos[s]] = pre_kh[s];
            }
    };
    auto fetch_mid = [&](int kyl, int klp) {
        const int kwy = wrapz(kyl, nz), kwl = wrapz(klp, nz);
#pragma unroll
        for (int s = 0; s < NLM; ++s)
            if (lm_pos[s] >= 0) {
                pre_yl[s] = fyl.load(kwy, lm_off[s]);
                pre_lp[s] = flp.load(kwl, lm_off[s]);
            }
    };

    // gbar (all components) and the local term at LDS offset q of a plane ring with pitch PW
    auto cell = [&](const T* Y0, const T* Y1, const T* Y2, const T* K0, const T* K1, const T* K2,
                    int q, int PW, T gb[3]) -> T {
        T g[3], qb[3];
        g[0] = grad1(Y1[q + 1], Y1[q - 1], inv_2dx);
        g[1] = grad1(Y1[q + PW], Y1[q - PW], inv_2dx);
        g[2] = grad1(Y2[q], Y0[q], inv_2dx);
        qb[0] = -hg * (adj_face(K1[q - 1], K1[q], inv_dx) + adj_face(K1[q], K1[q + 1], inv_dx));
        qb[1] = -hg * (adj_face(K1[q - PW], K1[q], inv_dx) + adj_face(K1[q], K1[q + PW], inv_dx));
        qb[2] = -hg * (adj_face(K0[q], K1[q], inv_dx) + adj_face(K1[q], K2[q], inv_dx));
        return adj_cell(Y1[q], g, qb, d2, gb);
    };

    // E1 per-slot z state (finishing plane p): gbar_z at p-1 and p, the local term at p, the
    // z-face cotangent of (p-1, p), W at p
    T e_gzp[2] = {T(0), T(0)}, e_gzc[2] = {T(0), T(0)}, e_loc[2] = {T(0), T(0)};
    T e_fbz[2] = {T(0), T(0)}, e_w0[2] = {T(0), T(0)};
    // E2 z state (finishing plane t)
    T gzp2 = T(0), gzc2 = T(0), loc2 = T(0), fbz2 = T(0), w20 = T(0);
    // own-cell partial sums from E1 (plane p) to E2 (two iterations later): entries 0, 1, 2 hold
    // planes t, t+1, t+2 after E1 of iteration t; gW is that of plane p+1
    T q_l[3] = {T(0), T(0), T(0)}, q_gu[3] = {T(0), T(0), T(0)}, q_gv[3] = {T(0), T(0), T(0)};
    T q_gw[3] = {T(0), T(0), T(0)};

    const int tbeg = k0 - 8;
    fetch_in(tbeg + 2);
    commit_in(0);
    fetch_in(tbeg + 3);
    commit_in(1);
    fetch_in(tbeg + 4);
    fetch_mid(tbeg + 2, tbeg + 2);

    auto iteration = [&](auto RC, int t) {
        constexpr int R = decltype(RC)::value;
        constexpr int sa = R % 3, sb = (R + 1) % 3, sc = (R + 2) % 3;  // planes t+2, t+3, t+4
        constexpr int gnew = (R + 1) & 1, gold = R & 1;
        const bool e1_gbar = t >= k0 - 6, e1_fin = t >= k0 - 5;
        const bool e2_gbar = t >= k0 - 2, e2_fin = t >= k0 - 1;
        // ---- commits and loads of the next iteration's planes; lam' of plane t+2 on MID
        commit_in(sc);
#pragma unroll
        for (int s = 0; s < NLM; ++s)
            if (lm_pos[s] >= 0) s_lp[lm_pos[s]] = pre_lp[s];
        const T* pre_yl_now = pre_yl;  // y_L of plane t+2, committed after the first barrier
        T yl_now[NLM];
#pragma unroll
        for (int s = 0; s < NLM; ++s) yl_now[s] = pre_yl_now[s];
        fetch_in(t + 5);
        fetch_mid(t + 3, t + 3);
        // E1 per-cell operands of plane p = t+2 (velocities; own cell: gradients of p, W of p+1)
        const int p = t + 2;
        const int pw = wrapz(p, nz), pw1 = wrapz(p + 1, nz);
        T eu0[2], eu1[2], ev0[2], ev1[2], ew1[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (s == 1 && !has_ring) continue;
            eu0[s] = fU.load(pw, e_col[s]);
            eu1[s] = fU.load(pw, e_colx[s]);
            ev0[s] = fV.load(pw, e_col[s]);
            ev1[s] = fV.load(pw, e_coly[s]);
            ew1[s] = fW.load(pw1, e_col[s]);
        }
        const bool own_p = p >= k0 && p < k1 && active;           // plane p is output
        const bool own_p1 = p + 1 >= k0 && p + 1 < k1 && active;  // W gradient of p+1 is output
        const size_t op = (size_t)pw * plane, op1 = (size_t)pw1 * plane;
        T g_u = T(0), g_v = T(0), g_w = T(0), base = T(0);
        if (own_p) {
            if (a.gU) g_u = ldg(a.gU + op, e_col[0]);
            if (a.gV) g_v = ldg(a.gV + op, e_col[0]);
            base = ldg(a.base + op, e_col[0]);
        }
        if (own_p1 && a.gW) g_w = ldg(a.gW + op1, e_col[0]);
        __syncthreads();  // IN plane t+4, lam' of plane t+2 visible; E2 of t-1 done with y_L
#pragma unroll
        for (int s = 0; s < NLM; ++s)
            if (lm_pos[s] >= 0) s_yl[sa * MS + lm_pos[s]] = yl_now[s];

        const T* YA = s_yh + sa * INS;  // plane t+2
        const T* YB = s_yh + sb * INS;  // plane t+3
        const T* YC = s_yh + sc * INS;  // plane t+4
        const T* KA = s_kh + sa * INS;
        const T* KB = s_kh + sb * INS;
        const T* KC = s_kh + sc * INS;
        T* G1Xn = s_g1x + gnew * G1XS;
        T* G1Yn = s_g1y + gnew * G1YS;
        const T* G1Xo = s_g1x + gold * G1XS;
        const T* G1Yo = s_g1y + gold * G1YS;
        T* KL = s_kl + sa * MS;  // kap_L of plane t+2

        // ---- E1: gbar_H at plane t+3 on the slots and the outer ring
        T gz_next[2] = {T(0), T(0)}, loc_next[2] = {T(0), T(0)};
        if (e1_gbar) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (s == 1 && !has_ring) continue;
                const int oi = (e_lx[s] + 2) + (e_ly[s] + 2) * INW;
                T gb[3];
                loc_next[s] = cell(YA, YB, YC, KA, KB, KC, oi, INW, gb);
                G1Xn[(e_lx[s] + 1) + e_ly[s] * G1XW] = gb[0];
                G1Yn[e_lx[s] + (e_ly[s] + 1) * MW] = gb[1];
                gz_next[s] = gb[2];
            }
            if (has_out) {
                T gb[3];
                (void)cell(YA, YB, YC, KA, KB, KC, o_in, INW, gb);
                if (o_axis == 0)
                    G1Xn[o_dst] = gb[0];
                else
                    G1Yn[o_dst] = gb[1];
            }
        }
        // ---- E1: finish ybar_H at plane t+2 -> kap_L, own-cell partial sums
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (s == 1 && !has_ring) continue;
            const int lx = e_lx[s], ly = e_ly[s];
            const int o = (lx + 2) + (ly + 2) * INW;
            const T fbz_next = adj_face(KA[o], KB[o], inv_dx);  // z-face (t+2, t+3)
            if (e1_fin) {
                T ybar = e_loc[s];
                T lo = adj_face(KA[o - 1], KA[o], inv_dx), hi = adj_face(KA[o], KA[o + 1], inv_dx);
                ybar = fma(lo, fma(-hsH, eu0[s], ge), ybar);
                ybar = fma(hi, fma(-hsH, eu1[s], -ge), ybar);
                if (s == 0) g_u = fma(-hsH * (YA[o - 1] + YA[o]), lo, g_u);
                const T* GX = G1Xo + lx + ly * G1XW;  // gbar_x at lx-1, lx, lx+1
                ybar = fma(GX[0] - GX[2], inv_2dx, ybar);
                lo = adj_face(KA[o - INW], KA[o], inv_dx);
                hi = adj_face(KA[o], KA[o + INW], inv_dx);
                ybar = fma(lo, fma(-hsH, ev0[s], ge), ybar);
                ybar = fma(hi, fma(-hsH, ev1[s], -ge), ybar);
                if (s == 0) g_v = fma(-hsH * (YA[o - INW] + YA[o]), lo, g_v);
                const T* GY = G1Yo + lx + ly * MW;  // gbar_y at ly-1, ly, ly+1 (stride MW)
                ybar = fma(GY[0] - GY[2 * MW], inv_2dx, ybar);
                ybar = fma(e_fbz[s], fma(-hsH, e_w0[s], ge), ybar);
                ybar = fma(fbz_next, fma(-hsH, ew1[s], -ge), ybar);
                ybar = fma(e_gzp[s] - gz_next[s], inv_2dx, ybar);
                const T lp = s_lp[lx + ly * MW];
                KL[lx + ly * MW] = fma(a.kaL, ybar, a.kbL * lp);
                if (s == 0) {
                    g_w = fma(-hsH * (YA[o] + YB[o]), fbz_next, g_w);
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        q_l[q] = q_l[q + 1];
                        q_gu[q] = q_gu[q + 1];
                        q_gv[q] = q_gv[q + 1];
                        q_gw[q] = q_gw[q + 1];
                    }
                    q_l[2] = base + ybar;
                    q_gu[2] = g_u;
                    q_gv[2] = g_v;
                    q_gw[2] = g_w;
                }
            }
            e_gzp[s] = e_gzc[s];
            e_gzc[s] = gz_next[s];
            e_loc[s] = loc_next[s];
            e_fbz[s] = fbz_next;
            e_w0[s] = ew1[s];
        }
        // E2 per-cell operands of plane t (reloaded; E1 touched them two iterations ago)
        const int tw = wrapz(t, nz), tw1 = wrapz(t + 1, nz);
        const unsigned c0 = e_col[0], cx = e_colx[0], cy = e_coly[0];
        T u0 = T(0), u1 = T(0), v0 = T(0), v1 = T(0), w1 = T(0), lpc = T(0);
        if (e2_fin) {
            u0 = fU.load(tw, c0);
            u1 = fU.load(tw, cx);
            v0 = fV.load(tw, c0);
            v1 = fV.load(tw, cy);
            w1 = fW.load(tw1, c0);
            if (a.kout || a.lam_copy) lpc = ldg(a.lamp + (size_t)tw * plane, c0);
        }
        __syncthreads();  // kap_L of plane t+2 and y_L of plane t+2 visible

        // ---- E2: gbar_L at plane t+1, finish ybar_L at plane t
        constexpr int m0 = (R + 1) % 3, m1 = (R + 2) % 3;  // MID ring slots of planes t, t+1
        const T *Y0 = s_yl + m0 * MS, *Y1 = s_yl + m1 * MS, *Y2 = s_yl + sa * MS;
        const T *K0 = s_kl + m0 * MS, *K1 = s_kl + m1 * MS, *K2 = s_kl + sa * MS;
        const int om = (tx + 2) + (ty + 2) * MW;
        T gz_n2 = T(0), loc_n2 = T(0);
        if (e2_gbar) {
            T gb[3];
            loc_n2 = cell(Y0, Y1, Y2, K0, K1, K2, om, MW, gb);
            s_g2x[gnew * G2XS + (tx + 1) + ty * G2XW] = gb[0];
            s_g2y[gnew * G2YS + tx + (ty + 1) * TX] = gb[1];
            gz_n2 = gb[2];
            if (has_h2) {
                T hb[3];
                (void)cell(Y0, Y1, Y2, K0, K1, K2, h_om, MW, hb);
                if (h_axis == 0)
                    s_g2x[gnew * G2XS + h_dst] = hb[0];
                else
                    s_g2y[gnew * G2YS + h_dst] = hb[1];
            }
        }
        const T fbz_n2 = adj_face(K0[om], K1[om], inv_dx);  // z-face (t, t+1)
        if (e2_fin) {
            const bool out_t = t >= k0 && t < k1 && active;
            const bool out_t1 = t + 1 >= k0 && t + 1 < k1 && active;
            const size_t ot = (size_t)tw * plane, ot1 = (size_t)tw1 * plane;
            if (out_t1 && a.gW) stg<T>(a.gW + ot1, c0, fma(-hsL * (Y0[om] + Y1[om]), fbz_n2, q_gw[0]));
            if (out_t) {
                T ybar = loc2;
                T lo = adj_face(K0[om - 1], K0[om], inv_dx), hi = adj_face(K0[om], K0[om + 1], inv_dx);
                ybar = fma(lo, fma(-hsL, u0, ge), ybar);
                ybar = fma(hi, fma(-hsL, u1, -ge), ybar);
                if (a.gU) stg<T>(a.gU + ot, c0, fma(-hsL * (Y0[om - 1] + Y0[om]), lo, q_gu[0]));
                const T* GX = s_g2x + gold * G2XS + tx + ty * G2XW;
                ybar = fma(GX[0] - GX[2], inv_2dx, ybar);
                lo = adj_face(K0[om - MW], K0[om], inv_dx);
                hi = adj_face(K0[om], K0[om + MW], inv_dx);
                ybar = fma(lo, fma(-hsL, v0, ge), ybar);
                ybar = fma(hi, fma(-hsL, v1, -ge), ybar);
                if (a.gV) stg<T>(a.gV + ot, c0, fma(-hsL * (Y0[om - MW] + Y0[om]), lo, q_gv[0]));
                const T* GY = s_g2y + gold * G2YS + tx + ty * TX;
                ybar = fma(GY[0] - GY[2 * TX], inv_2dx, ybar);
                ybar = fma(fbz2, fma(-hsL, w20, ge), ybar);
                ybar = fma(fbz_n2, fma(-hsL, w1, -ge), ybar);
                ybar = fma(gzp2 - gz_n2, inv_2dx, ybar);
                stg<T>(a.L_out + ot, c0, q_l[0] + ybar);
                if (a.kout) stg<T>(a.kout + ot, c0, fma(a.kaO, ybar, a.kbO * lpc));
                if (a.lam_copy) stg<T>(a.lam_copy + ot, c0, lpc);
            }
        }
        gzp2 = gzc2;
        gzc2 = gz_n2;
        loc2 = loc_n2;
        fbz2 = fbz_n2;
        w20 = w1;
    };

    const int tend = tbeg + 6 * ((k1 - tbeg + 5) / 6);  // tbeg .. k1-1, in groups of six
    for (int t = tbeg; t < tend; t += 6) {
        iteration(IntC<0>(), t);
        iteration(IntC<1>(), t + 1);
        iteration(IntC<2>(), t + 2);
        iteration(IntC<3>(), t + 3);
        iteration(IntC<4>(), t + 4);
        iteration(IntC<5>(), t + 5);
    }
}

template <typename T, int TX, int TY>
static hipError_t launch_pair(const AdjPairArgs<T>& a, int kz, hipStream_t st)
{
    const int tiles_x = (a.nx + TX - 1) / TX;
    const int tiles_y = (a.ny + TY - 1) / TY;
    if (a.nz <= 0 || tiles_x <= 0 || tiles_y <= 0 || kz < 0) return hipErrorInvalidValue;
    if (field_needs_big(a.nx, a.ny, a.nz, sizeof(T))) return hipErrorInvalidValue;
    if (kz == 0) {
        kz = launch_chunk_planes((const void*)adjoint_pair_kernel<T, TX, TY>, TX * TY,
                                 (long long)tiles_x * tiles_y, a.nz, 7);
        if (kz <= 0) return hipErrorInvalidDevice;
    }
    const long long blocks = (long long)tiles_x * tiles_y * ((a.nz + kz - 1) / kz);
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((adjoint_pair_kernel<T, TX, TY>), dim3((unsigned)blocks), dim3(TX * TY), 0,
                       st, a, tiles_x, tiles_y, kz);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_pair(const AdjPairArgs<T>& a, int tile, int kz, hipStream_t st)
{
    switch (tile) {
    case 0: return launch_pair<T, 64, 8>(a, kz, st);
    case 1: return launch_pair<T, 32, 16>(a, kz, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_adjoint_pair<float>(const AdjPairArgs<float>&, int, int, hipStream_t);
template hipError_t launch_adjoint_pair<double>(const AdjPairArgs<double>&, int, int, hipStream_t);

}  // namespace pf
