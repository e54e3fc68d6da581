// Two RK4 stages in one z-march (the fused variants).
//
// A classic RK4 step is run as two sweeps instead of four:
//   sweep A (stages 1+2):  k1 = f(phi);  ya = phi + dt/2 k1;  acc1 = phi + dt/6 k1;
//                          k2 = f(ya);   writes yb = phi + dt/2 k2,  acc = acc1 + dt/3 k2
//   sweep B (stages 3+4):  k3 = f(yb);   ya = phi + dt k3;   acc3 = acc + dt/3 k3;
//                          k4 = f(ya);   writes phi' = acc3 + dt/6 k4
// with every operation in the same order and precision as the four separate stage launches, so
// the result is bit-identical to them. The intermediate stage value ya never leaves LDS: the
// first evaluation (E1) produces it on the tile plus a two-cell halo (the reach of the second
// evaluation E2), plane by plane, two planes ahead of E2. HBM traffic per cell-update drops from
// 28 to 13 words (A: phi, u, v, w in, yb, acc out; B: yb, phi, acc, u, v, w in, phi' out).
//
// Sweep B cannot write phi in place (other tiles still read phi on their halo), so it writes
// phi' over acc (read only at the cell itself) and the host alternates the roles of the two
// buffers from step to step.
//
// The explicit midpoint rule (RK2) is sweep A alone: with c_mid = dt/2 and c_y2 = dt its out_y
// is the new phi (into the other buffer of the pair), and a null out_acc skips the accumulator.
// Optional outputs (XOUT, a separate instantiation so that the descriptors cost the plain sweeps
// no registers): out_mid receives y_mid on the tile (sweep A: the RK4 stage value y2, so that the
// adjoint can recompute two stage inputs in one sweep; sweep B: y4, so that a step can keep all
// its stage values in two sweeps), and, in sweep A only, out_phi a copy of phi (then sweep B may
// read that copy and write the new phi into phi's own buffer, which ends an odd step count in
// place).
//
// Regions, for a TX x TY tile at (i0, j0), as (x range) x (y range):
//   IN   stage input, ring of 3 planes       [i0-4, i0+TX+4) x [j0-4, j0+TY+4)
//   MID  E1 cells / ya ring of 3 planes      [i0-2, i0+TX+2) x [j0-2, j0+TY+2)
//   Q1X  x-sharpening of E1, 2 planes        [i0-3, i0+TX+3) x [j0-2, j0+TY+2)
//   Q1Y  y-sharpening of E1, 2 planes        [i0-2, i0+TX+2) x [j0-3, j0+TY+3)
//   Q2X  x-sharpening of E2, 2 planes        [i0-1, i0+TX+1) x [j0, j0+TY)
//   Q2Y  y-sharpening of E2, 2 planes        [i0, i0+TX) x [j0-1, j0+TY+1)
//   PB   phi on MID (sweep B only), 1 plane
//   VEL  FP64 only: U, V of plane t+2 and W of plane t+3 on the MID rows (V with one more
//        row), loaded one plane ahead in 16-byte pieces where rows allow. FP32 reads the
//        velocities at the E1 cells directly: within its 128-register budget the staging
//        registers spill, and staging ran slower (also with U and V alone).
// Pipeline: iteration t loads input plane t+4, E1 computes q1 at plane t+3 and ya at plane
// t+2, E2 computes q2 at plane t+1 and the outputs of plane t. Six warm-up iterations precede
// the first output plane of a z-chunk: four with E1 alone (a straight-line prologue), then the
// main loop, which runs E1 and E2 in whole groups of six unconditional iterations so that the
// values handed from plane to plane stay in place; iterations past the chunk end compute on
// wrapped planes and store nothing. Two barriers per iteration.
// LAG (the one-barrier march): E2 trails E1 by one more plane (q2 at plane t, outputs of plane
// t-1) and each iteration commits the planes of the next one, so that within an iteration every
// LDS read is of data written in earlier iterations and every write goes to a slot nobody reads
// in it; one barrier ends the iteration. The cost is deeper rings (four stage-input and four
// middle-stage planes, two of each staged plane, a fourth own-cell queue entry), five warm-up
// iterations and groups of four. Same arithmetic in the same order: bit-identical results.
// Global memory goes through FieldRef buffer descriptors (BIG: arrays of 4 GiB or more). With
// WIDE (nx a multiple of 16 bytes' worth of elements), the planes of the stage input and of phi
// are read in 16-byte pieces: groups of consecutive x-columns that start at a multiple of the
// group size never straddle the periodic wrap, so each group is one aligned load.
// WALLS (walls on any axes, a.walls bits 0-2): the stage input and phi are read through mirror
// indices, so the sharpening products of the ghost cells are the exact mirror images of their
// partners' (the normal component flips sign) and the diffusive and sharpening fluxes through a
// wall face vanish; the face velocity on a wall face counts as zero. In x and y, E1 evaluates
// only cells inside the domain; after it, each ghost cell of the middle-stage ring takes the
// value of its mirror partner (one more barrier), which is exactly what the per-stage kernel
// reads there. In z, E1 also evaluates the ghost planes, with U and V mirrored and W on a face
// beyond the wall the partner face's with its sign flipped: the plane next to a wall then comes
// out as its partner bit for bit (the two z-advection terms swap places with one of them zero),
// and the sharpening product of E2 on that ghost plane is set to the negated partner's (the
// plane two beyond, whose terms do not swap exactly, feeds nothing else that is stored). So the
// walled sweeps stay bit-identical to the per-stage launches.
#pragma once

#include <type_traits>

#include "pf_cell.h"
#include "pf_internal.h"

namespace pf {

// The one-barrier march on 32-wide FP64 tiles (32 x 16: 136-148 KB of LDS, one workgroup per
// compute unit, whose barriers left the compute unit idle: 512^3 step 4.55 -> 3.97 ms). FP64
// 64 x 8 tiles would need 166 KB. FP32 (two workgroups per compute unit) ran the same 512^3
// step in the same time in either form, with 10 % more sweep-B fetch in the one-barrier form,
// and keeps the two-barrier march.
template <typename T, int TX, int TY>
constexpr bool fused_lag()
{
    return sizeof(T) == 8 && TX == 32;
}

// The workgroup owns the TX x TY column tile (ti, tj) and the output planes [k0, k1).
template <typename T, int TX, int TY, bool SWEEP_B, bool BIG, bool WIDE, bool XOUT = false,
          bool WALLS = false, bool LAG = false>
__device__ __forceinline__ void fused_body(const FusedArgs<T>& a, int ti, int tj, int k0, int k1)
{
    static_assert(!(WALLS && WIDE), "mirror reads are element-wise");
    constexpr int NT = TX * TY;
    constexpr int VEC = 16 / (int)sizeof(T);  // elements per 16-byte piece
    static_assert(TX % VEC == 0, "the tile width must be a whole number of 16-byte pieces");
    constexpr int INW = TX + 8, INH = TY + 8, INS = INW * INH;
    constexpr int MW = TX + 4, MH = TY + 4, MS = MW * MH;
    constexpr int Q1XW = TX + 6, Q1XS = Q1XW * MH;
    constexpr int Q1YS = MW * (TY + 6);
    constexpr int Q2XW = TX + 2, Q2XS = Q2XW * TY;
    constexpr int Q2YS = TX * (TY + 2);
    constexpr int NRING = 4 * MW + 4 * TY;  // MID cells outside the tile
    constexpr int NOUT = 2 * MH + 2 * MW;   // q1-only cells (x- and y-outer ring)
    constexpr int NH2 = 2 * TX + 2 * TY;    // q2 halo cells
    // the q1-only cells start at the first whole wave after the ring cells, so no wave carries
    // both kinds of E1 halo work (the waves meet at a barrier after E1)
    constexpr int OUT0 = (NRING + 63) / 64 * 64;
    // plane loads: WIDE moves pieces of VEC elements (IN: whole rows; PB: the MID rows at the IN
    // width, so that pieces stay aligned), else single elements
    constexpr int INGW = INW / VEC;                 // pieces per IN row
    constexpr int PBW = WIDE ? INW : MW, PBS = PBW * MH;  // PB row width and plane size
    constexpr int NLI = WIDE ? (INGW * INH + NT - 1) / NT : (INS + NT - 1) / NT;
    constexpr int NLB = SWEEP_B ? (WIDE ? (INGW * MH + NT - 1) / NT : (MS + NT - 1) / NT) : 0;
    static_assert(OUT0 + NOUT <= NT, "tile too small for the E1 halo assignment");
    static_assert(NH2 <= NT, "tile too small for the E2 halo assignment");
    // ring depths: stage input and middle-stage planes, staged planes (velocities, phi on MID),
    // own-cell queue from E1 to E2
    constexpr int NIN = LAG ? 4 : 3, NMID = LAG ? 4 : 3, NSTG = LAG ? 2 : 1, NQ = LAG ? 4 : 3;

    // separate arrays, so that the compiler knows the regions do not overlap
    __shared__ __align__(16) T s_in[NIN * INS];
    __shared__ T s_mid[NMID * MS];
    __shared__ T s_q1x[2 * Q1XS];
    __shared__ T s_q1y[2 * Q1YS];
    __shared__ T s_q2x[2 * Q2XS];
    __shared__ T s_q2y[2 * Q2YS];
    __shared__ __align__(16) T s_pb[SWEEP_B ? NSTG * PBS : 1];
    // velocity staging (x from i0-4 at the IN width, rows from j0-2): U on MH rows, V on MH+1
    // rows (its +y neighbour), W on MH rows
    constexpr bool STAGE = sizeof(T) == 8;  // velocity staging (FP64)
    constexpr int VSU = 0, VSV = MH * INW, VSW = (2 * MH + 1) * INW, VSS = (3 * MH + 1) * INW;
    __shared__ __align__(16) T s_vel[STAGE ? NSTG * VSS : 1];

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t plane = (size_t)nx * ny;
    const int i0 = ti * TX, j0 = tj * TY;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const bool active = (i0 + tx < nx) && (j0 + ty < ny);
    const T inv_2dx = a.inv_2dx, d2 = a.delta2, hg = a.hg, ge = a.ge;
    // index maps of the stage input and phi: periodic wrap, or the mirror across walls
    const bool wx = WALLS && (a.walls & 1), wy = WALLS && (a.walls & 2), wz = WALLS && (a.walls & 4);
    auto mapx = [&](int v) { return WALLS && wx ? reflectn(v, nx) : wrapn(v, nx); };
    auto mapy = [&](int v) { return WALLS && wy ? reflectn(v, ny) : wrapn(v, ny); };
    auto mapz = [&](int v) { return WALLS && wz ? reflectz(v, nz) : wrapz(v, nz); };
    // W on face p (between planes p-1 and p): the plane to read and the sign. Along a walled z
    // axis (seen as a periodic one of 2 nz planes) the wall faces 0 and nz carry no velocity
    // (sign 0) and a face beyond a wall is its mirror partner with the normal component flipped.
    auto wface = [&](int p, int& kw) -> int {
        if (!(WALLS && wz)) {
            kw = wrapz(p, nz);
            return 1;
        }
        if (p > 0 && p < nz) {
            kw = p;
            return 1;
        }
        if (p == 0 || p == nz) {
            kw = 0;
            return 0;
        }
        if (nz >= 16) {  // the march reaches at most 10 planes beyond the domain
            kw = p < 0 ? -p : 2 * nz - p;
            return -1;
        }
        int m = p % (2 * nz);
        if (m < 0) m += 2 * nz;
        kw = m < nz ? m : 2 * nz - m;
        if (m == 0 || m == nz) {
            kw = 0;
            return 0;
        }
        return m < nz ? 1 : -1;
    };
    auto wval = [](int sg, T v) -> T { return sg == 0 ? T(0) : (sg < 0 ? -v : v); };

    // ---- E1 cell slots: slot 0 = own cell, slot 1 = a MID ring cell (tid < NRING)
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
    // byte offsets within a plane of the slots' (wrapped) columns and their +1 neighbours
    constexpr unsigned ES = sizeof(T);
    unsigned e_col[2], e_colx[2], e_coly[2];
    // WALLS: per slot, bit 0/1: its low/high x-face is a wall face, bit 2/3 likewise in y; bit 4:
    // the cell is a ghost (outside the domain along a walled axis)
    int e_wall[2] = {0, 0};
    int e_gsrc[2] = {0, 0};
    for (int s = 0; s < 2; ++s) {
        const int gx = wrapn(i0 - 2 + e_lx[s], nx), gy = wrapn(j0 - 2 + e_ly[s], ny);
        e_col[s] = (unsigned)(gy * nx + gx) * ES;
        e_colx[s] = (unsigned)(gy * nx + wrapn(gx + 1, nx)) * ES;
        e_coly[s] = (unsigned)(wrapn(gy + 1, ny) * nx + gx) * ES;
        if constexpr (WALLS) {
            const int ux = i0 - 2 + e_lx[s], uy = j0 - 2 + e_ly[s];  // unwrapped
            e_wall[s] = (wx && ux == 0 ? 1 : 0) | (wx && ux == nx - 1 ? 2 : 0) |
                        (wy && uy == 0 ? 4 : 0) | (wy && uy == ny - 1 ? 8 : 0) |
                        ((wx && (ux < 0 || ux >= nx)) || (wy && (uy < 0 || uy >= ny)) ? 16 : 0);
            // a ghost slot's mirror partner in the middle-stage ring (fixed along the march)
            const int mx = wx ? reflectn(ux, nx) : ux, my = wy ? reflectn(uy, ny) : uy;
            e_gsrc[s] = (mx - (i0 - 2)) + (my - (j0 - 2)) * MW;
        }
    }
    // ---- q1-only cell (x-outer: Q1X columns 0 and TX+5; y-outer: Q1Y rows 0 and TY+5)
    const int ro = tid - OUT0;
    const bool has_out = ro >= 0 && ro < NOUT;
    int o_in = 0, o_dst = 0, o_axis = 0;
    if (has_out) {
        if (ro < 2 * MH) {
            const int side = ro / MH, ry = ro - side * MH;
            o_in = (side ? TX + 6 : 1) + (ry + 2) * INW;
            o_dst = (side ? TX + 5 : 0) + ry * Q1XW;
            o_axis = 0;
        } else {
            const int r2 = ro - 2 * MH;
            const int side = r2 / MW, cx = r2 - side * MW;
            o_in = (cx + 2) + (side ? TY + 6 : 1) * INW;
            o_dst = cx + (side ? TY + 5 : 0) * MW;
            o_axis = 1;
        }
    }
    // ---- q2 halo cell (threads at the top of the block, which have no ring work)
    const int rh = tid - (NT - NH2);
    const bool has_h2 = rh >= 0;
    int h_om = 0, h_dst = 0, h_axis = 0;
    if (has_h2) {
        if (rh < 2 * TY) {
            const int side = rh / TY, r = rh - side * TY;
            h_om = (side ? TX + 2 : 1) + (r + 2) * MW;
            h_dst = (side ? TX + 1 : 0) + r * Q2XW;
            h_axis = 0;
        } else {
            const int r2 = rh - 2 * TY;
            const int side = r2 / TX, c = r2 - side * TX;
            h_om = (c + 2) + (side ? TY + 2 : 1) * MW;
            h_dst = c + (side ? TY + 1 : 0) * TX;
            h_axis = 1;
        }
    }

    // ---- plane loads: IN (stage input with halo 4) and, for sweep B, phi on MID
    unsigned li_off[NLI];
    int li_pos[NLI];
#pragma unroll
    for (int s = 0; s < NLI; ++s) {
        const int e = tid + s * NT;
        if (WIDE) {
            const int r = e / INGW, g = e - r * INGW;
            li_pos[s] = e < INGW * INH ? r * INW + g * VEC : -1;
            li_off[s] = e < INGW * INH
                            ? (unsigned)(wrapn(j0 - 4 + r, ny) * nx + wrapn(i0 - 4 + g * VEC, nx)) * ES
                            : 0u;
        } else {
            const int r = e / INW, c = e - r * INW;
            li_pos[s] = e < INS ? e : -1;
            li_off[s] = e < INS ? (unsigned)(mapy(j0 - 4 + r) * nx + mapx(i0 - 4 + c)) * ES : 0u;
        }
    }
    unsigned lb_off[NLB > 0 ? NLB : 1];
    int lb_pos[NLB > 0 ? NLB : 1];
#pragma unroll
    for (int s = 0; s < NLB; ++s) {
        const int e = tid + s * NT;
        if (WIDE) {
            const int r = e / INGW, g = e - r * INGW;
            lb_pos[s] = e < INGW * MH ? r * PBW + g * VEC : -1;
            lb_off[s] = e < INGW * MH
                            ? (unsigned)(wrapn(j0 - 2 + r, ny) * nx + wrapn(i0 - 4 + g * VEC, nx)) * ES
                            : 0u;
        } else {
            const int r = e / MW, c = e - r * MW;
            lb_pos[s] = e < MS ? e : -1;
            lb_off[s] = e < MS ? (unsigned)(mapy(j0 - 2 + r) * nx + mapx(i0 - 2 + c)) * ES : 0u;
        }
    }
    // velocity staging loads: a flattened list of the U, V and W pieces, NLV per thread
    constexpr int PPR = WIDE ? INGW : INW, PV = WIDE ? VEC : 1;  // pieces per row, their width
    constexpr int NGU = PPR * MH, NGV = PPR * (MH + 1), NGVEL = 2 * NGU + NGV;
    constexpr int NLV = STAGE ? (NGVEL + NT - 1) / NT : 0;
    // piece e of the list lands at LDS element e * PV (the regions are stacked row by row at
    // the IN width); only its source offset is kept per thread
    unsigned lv_off[NLV > 0 ? NLV : 1];
#pragma unroll
    for (int s = 0; s < NLV; ++s) {
        const int e = tid + s * NT;
        const int q = e < NGU ? e : (e < NGU + NGV ? e - NGU : e - NGU - NGV);
        const int r = q / PPR, g = q - r * PPR;
        lv_off[s] = e < NGVEL ? (unsigned)(wrapn(j0 - 2 + r, ny) * nx + wrapn(i0 - 4 + g * PV, nx)) * ES
                              : 0u;
    }
    static_assert(VSV == NGU * PV && VSW == (NGU + NGV) * PV, "staging regions must be stacked");
    typedef typename std::conditional<WIDE, v4i_t, T>::type piece_t;
    piece_t pre_in[NLI];
    piece_t pre_b[NLB > 0 ? NLB : 1];
    const FieldRef<T, BIG> fy(a.y, plane, nz), fphi(a.phi, plane, nz), facc(a.acc_in, plane, nz),
        foy(a.out_y, plane, nz), foacc(a.out_acc, plane, nz), fomid(a.out_mid, plane, nz),
        fophi(a.out_phi, plane, nz), fU(a.U, plane, nz),
        fV(a.V, plane, nz), fW(a.W, plane, nz);
    auto load_piece = [&](const FieldRef<T, BIG>& f, int kw, unsigned off) -> piece_t {
        if constexpr (WIDE)
            return f.load16(kw, off);
        else
            return f.load(kw, off);
    };
    auto put_piece = [&](T* dst, const piece_t& v) {
        if constexpr (WIDE)
            *reinterpret_cast<v4i_t*>(dst) = v;
        else
            *dst = v;
    };
    auto fetch_in = [&](int kk) {
        const int kw = mapz(kk);
#pragma unroll
        for (int s = 0; s < NLI; ++s)
            if (li_pos[s] >= 0) pre_in[s] = load_piece(fy, kw, li_off[s]);
    };
    auto commit_in = [&](int slot) {
#pragma unroll
        for (int s = 0; s < NLI; ++s)
            if (li_pos[s] >= 0) put_piece(s_in + slot * INS + li_pos[s], pre_in[s]);
    };
    auto fetch_b = [&](int kk) {
        const int kw = mapz(kk);
#pragma unroll
        for (int s = 0; s < NLB; ++s)
            if (lb_pos[s] >= 0) pre_b[s] = load_piece(fphi, kw, lb_off[s]);
    };
    piece_t pre_v[NLV > 0 ? NLV : 1];
    auto fetch_vel = [&](int p) {  // U, V at plane p, W at plane p+1
        const int kw = mapz(p);
        int kw1;
        const int sg1 = wface(p + 1, kw1);
#pragma unroll
        for (int s = 0; s < NLV; ++s) {
            const int e = tid + s * NT;
            if (e < NGU)
                pre_v[s] = load_piece(fU, kw, lv_off[s]);
            else if (e < NGU + NGV)
                pre_v[s] = load_piece(fV, kw, lv_off[s]);
            else if (e < NGVEL) {
                if constexpr (WALLS)
                    pre_v[s] = wval(sg1, load_piece(fW, kw1, lv_off[s]));
                else
                    pre_v[s] = load_piece(fW, kw1, lv_off[s]);
            }
        }
    };
    auto commit_vel = [&](int slot) {
#pragma unroll
        for (int s = 0; s < NLV; ++s) {
            const int e = tid + s * NT;
            if (e < NGVEL) put_piece(s_vel + slot * VSS + e * PV, pre_v[s]);
        }
    };
    auto commit_b = [&](int slot) {
#pragma unroll
        for (int s = 0; s < NLB; ++s)
            if (lb_pos[s] >= 0) put_piece(s_pb + slot * PBS + lb_pos[s], pre_b[s]);
    };

    // per-slot z state of E1 (q1_z and the z-face flux) and of E2
    // per-slot z state of E1 at plane p: q1_z at p-1 and p, sum and difference of phi on the
    // face (p-1, p), W at p; the same for E2 at plane t
    T e_qzm[2] = {T(0), T(0)}, e_qz[2] = {T(0), T(0)}, e_sz[2] = {T(0), T(0)};
    T e_dz[2] = {T(0), T(0)}, e_w0[2] = {T(0), T(0)};
    T q2zm = T(0), q2z = T(0), sz2 = T(0), dz2 = T(0), w2 = T(0);
    // own-cell queues from E1 (plane p) to E2 (plane p, NQ-1 iterations later): after E1 of
    // iteration t they hold planes t+3-NQ .. t+2 in entries 0 .. NQ-1
    T qa_phi[NQ] = {}, qa_acc[NQ] = {}, qa_u0[NQ] = {}, qa_u1[NQ] = {}, qa_v0[NQ] = {};
    T qa_v1[NQ] = {}, qa_w1[NQ] = {};

    const int tbeg = k0 - 6;
    T eacc_pre = T(0);  // LAG, sweep B: acc at the own cell of the next E1 plane
    if constexpr (LAG) {
        // planes p = tbeg+2 .. tbeg+4 committed to slots (p - tbeg) mod 4, plane tbeg+5 in
        // flight; the staged planes of tbeg+2 committed to slot 0, tbeg+3 in flight
        fetch_in(tbeg + 2);
        commit_in(2);
        fetch_in(tbeg + 3);
        commit_in(3);
        fetch_in(tbeg + 4);
        commit_in(0);
        if (STAGE) {
            fetch_vel(tbeg + 2);
            commit_vel(0);
        }
        if (SWEEP_B) {
            fetch_b(tbeg + 2);
            commit_b(0);
            eacc_pre = facc.load(wrapz(tbeg + 2, nz), e_col[0]);
        }
        fetch_in(tbeg + 5);
        if (STAGE) fetch_vel(tbeg + 3);
        if (SWEEP_B) fetch_b(tbeg + 3);
        __syncthreads();
    } else {
        fetch_in(tbeg + 2);
        commit_in(0);
        fetch_in(tbeg + 3);
        commit_in(1);
        fetch_in(tbeg + 4);
        if (STAGE) fetch_vel(tbeg + 2);
        if (SWEEP_B) fetch_b(tbeg + 2);
    }

    // One iteration of the march; R = (t - tbeg) mod 6 (LAG: mod 4) fixes every ring slot at
    // compile time, WITH_E2 whether the second evaluation runs.
    auto iteration = [&](auto RC, auto E2C, int t) {
        constexpr int R = decltype(RC)::value;
        constexpr bool WITH_E2 = decltype(E2C)::value != 0;
        // slots of the stage input planes t+2, t+3, t+4 (and of ya at plane t+2)
        constexpr int sa = LAG ? (R + 2) % 4 : R % 3;
        constexpr int sb = LAG ? (R + 3) % 4 : (R + 1) % 3;
        constexpr int sc = LAG ? R % 4 : (R + 2) % 3;
        constexpr int q1new = (R + 1) & 1, q1old = R & 1;
        constexpr int vs = LAG ? R % 2 : 0;  // slot of the staged planes of t+2
        if constexpr (LAG) {
            // the planes of the next iteration into the slots this one does not read
            commit_in((R + 1) % 4);  // plane t+5
            if (STAGE) commit_vel((R + 1) % 2);  // velocities of plane t+3 (W: t+4)
            if (SWEEP_B) commit_b((R + 1) % 2);
            fetch_in(t + 6);
            if (STAGE) fetch_vel(t + 4);
            if (SWEEP_B) fetch_b(t + 4);
        } else {
            commit_in(sc);
            if (STAGE) commit_vel(0);  // velocities of plane t+2 (W: t+3)
            if (SWEEP_B) commit_b(0);
            fetch_in(t + 5);
            if (STAGE) fetch_vel(t + 3);
            if (SWEEP_B) fetch_b(t + 3);
        }
        // E1 operands from global memory (plane p = t+2), issued before the barrier; the
        // accumulator is read at the wrapped plane (it is used on the domain's planes only)
        const int pw = mapz(t + 2), pa = wrapz(t + 2, nz), pa1 = wrapz(t + 3, nz);
        int pw1;
        const int sgw = wface(t + 3, pw1);
        T eu0[2], eu1[2], ev0[2], ev1[2], ew1[2], eacc = T(0);
        if (!STAGE) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (s == 1 && !has_ring) continue;  // whole waves without ring cells skip these
                eu0[s] = fU.load(pw, e_col[s]);
                eu1[s] = fU.load(pw, e_colx[s]);
                ev0[s] = fV.load(pw, e_col[s]);
                ev1[s] = fV.load(pw, e_coly[s]);
                if constexpr (WALLS)
                    ew1[s] = wval(sgw, fW.load(pw1, e_col[s]));
                else
                    ew1[s] = fW.load(pw1, e_col[s]);
            }
        }
        if (SWEEP_B) {
            if constexpr (LAG) {  // loaded one iteration ahead
                eacc = eacc_pre;
                eacc_pre = facc.load(pa1, e_col[0]);
            } else {
                eacc = facc.load(pa, e_col[0]);
            }
        }
        // input plane t+4, phi (and staged velocities) of plane t+2 visible (LAG: since the
        // barrier that ended the previous iteration)
        if constexpr (!LAG) __syncthreads();
        if (STAGE) {
            const T* SV = s_vel + vs * VSS;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                // the slot's IN offset (e_lx + 2) + (e_ly + 2) INW, two rows up: same pitch
                const int vo = (e_lx[s] + 2) + (e_ly[s] + 2) * INW - 2 * INW;
                eu0[s] = SV[VSU + vo];
                eu1[s] = SV[VSU + vo + 1];
                ev0[s] = SV[VSV + vo];
                ev1[s] = SV[VSV + vo + INW];
                ew1[s] = SV[VSW + vo];
            }
        }

        if constexpr (WALLS) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (s == 1 && !has_ring) continue;
                if (e_wall[s] & 1) eu0[s] = T(0);
                if (e_wall[s] & 2) eu1[s] = T(0);
                if (e_wall[s] & 4) ev0[s] = T(0);
                if (e_wall[s] & 8) ev1[s] = T(0);
            }
        }

        const T* IA = s_in + sa * INS;  // plane t+2
        const T* IB = s_in + sb * INS;  // plane t+3
        const T* IC = s_in + sc * INS;  // plane t+4
        T* Q1Xn = s_q1x + q1new * Q1XS;
        T* Q1Yn = s_q1y + q1new * Q1YS;
        const T* Q1Xo = s_q1x + q1old * Q1XS;
        const T* Q1Yo = s_q1y + q1old * Q1YS;
        T* YM = s_mid + sa * MS;  // ya at plane t+2

        // q1 at plane t+3 on the E1 slots and the outer ring
        T qzn[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (s == 1 && !has_ring) {
                qzn[s] = T(0);
                continue;
            }
            const int oi = (e_lx[s] + 2) + (e_ly[s] + 2) * INW;
            const T gx = grad1(IB[oi + 1], IB[oi - 1], inv_2dx);
            const T gy = grad1(IB[oi + INW], IB[oi - INW], inv_2dx);
            const T gz = grad1(IC[oi], IA[oi], inv_2dx);
            const T fac = sharpen_factor(IB[oi], gx, gy, gz, d2, hg);
            Q1Xn[(e_lx[s] + 1) + e_ly[s] * Q1XW] = fac * gx;
            Q1Yn[e_lx[s] + (e_ly[s] + 1) * MW] = fac * gy;
            qzn[s] = fac * gz;
        }
        if (has_out) {
            const T gx = grad1(IB[o_in + 1], IB[o_in - 1], inv_2dx);
            const T gy = grad1(IB[o_in + INW], IB[o_in - INW], inv_2dx);
            const T gz = grad1(IC[o_in], IA[o_in], inv_2dx);
            const T fac = sharpen_factor(IB[o_in], gx, gy, gz, d2, hg);
            if (o_axis == 0)
                Q1Xn[o_dst] = fac * gx;
            else
                Q1Yn[o_dst] = fac * gy;
        }
        // E1: f1 at plane t+2 on the slots -> ya (and own-cell queues)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (s == 1 && !has_ring) continue;
            const int lx = e_lx[s], ly = e_ly[s];
            const int oi = (lx + 2) + (ly + 2) * INW;
            const T pc = IA[oi];
            const T pz = IB[oi];
            const T szp = face_sum(pc, pz), dzp = face_diff(pc, pz);
            const T* qx = Q1Xo + lx + ly * Q1XW;  // q1_x at lx-1, lx, lx+1
            const T* qy = Q1Yo + lx + ly * MW;     // q1_y at ly-1, ly, ly+1 (stride MW)
            const T pxm = IA[oi - 1], pxp = IA[oi + 1], pym = IA[oi - INW], pyp = IA[oi + INW];
            const T f1 = cell_rhs(face_sum(pxm, pc), face_sum(pc, pxp), face_sum(pym, pc),
                                  face_sum(pc, pyp), e_sz[s], szp, face_diff(pxm, pc),
                                  face_diff(pc, pxp), face_diff(pym, pc), face_diff(pc, pyp), e_dz[s],
                                  dzp, qx[0], qx[2], qy[0], qy[2 * MW], e_qzm[s], qzn[s], eu0[s],
                                  eu1[s], ev0[s], ev1[s], e_w0[s], ew1[s], a.nhs1, ge);
            const T base = SWEEP_B ? s_pb[vs * PBS + (WIDE ? lx + 2 : lx) + ly * PBW] : pc;
            const T ym = fma(a.c_mid, f1, base);
            YM[lx + ly * MW] = ym;
            if (s == 0) {
                if constexpr (XOUT) {
                    const int p = t + 2;
                    if (a.out_mid && p >= k0 && p < k1 && active) fomid.store(p, e_col[0], ym);
                }
                // own cell: hand plane p's values to E2 (used two iterations later)
#pragma unroll
                for (int q = 0; q < NQ - 1; ++q) {
                    qa_phi[q] = qa_phi[q + 1];
                    qa_acc[q] = qa_acc[q + 1];
                    qa_u0[q] = qa_u0[q + 1];
                    qa_u1[q] = qa_u1[q + 1];
                    qa_v0[q] = qa_v0[q + 1];
                    qa_v1[q] = qa_v1[q + 1];
                    qa_w1[q] = qa_w1[q + 1];
                }
                qa_phi[NQ - 1] = pc;
                qa_acc[NQ - 1] = SWEEP_B ? fma(a.c_acc1, f1, eacc) : fma(a.c_acc1, f1, pc);
                qa_u0[NQ - 1] = eu0[0];
                qa_u1[NQ - 1] = eu1[0];
                qa_v0[NQ - 1] = ev0[0];
                qa_v1[NQ - 1] = ev1[0];
                qa_w1[NQ - 1] = ew1[0];
            }
            e_sz[s] = szp;
            e_dz[s] = dzp;
            e_qzm[s] = e_qz[s];
            e_qz[s] = qzn[s];
            e_w0[s] = ew1[s];
        }
        if constexpr (WALLS) if (wx || wy) {
            __syncthreads();  // every E1 value of plane t+2 is in YM
            // ghost cells of the ring take their mirror partner's value
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (s == 1 && !has_ring) continue;
                if (!(e_wall[s] & 16)) continue;
                YM[e_lx[s] + e_ly[s] * MW] = YM[e_gsrc[s]];
            }
        }
        if constexpr (!LAG) __syncthreads();  // ya at plane t+2 visible

        if constexpr (WITH_E2) {
            // E2: q2 at plane to+1, outputs of plane to (to = t; LAG: to = t-1, so that E2 reads
            // only the planes of earlier iterations)
            const int to = LAG ? t - 1 : t;
            constexpr int m0 = LAG ? (R + 3) % 4 : (R + 1) % 3;  // plane to
            constexpr int m1 = LAG ? R % 4 : (R + 2) % 3;        // plane to+1
            constexpr int m2 = LAG ? (R + 1) % 4 : R % 3;        // plane to+2
            const T* M0 = s_mid + m0 * MS;
            const T* M1 = s_mid + m1 * MS;
            const T* M2 = s_mid + m2 * MS;
            constexpr int q2new = LAG ? R & 1 : (R + 1) & 1, q2old = LAG ? (R + 1) & 1 : R & 1;
            const int om = (tx + 2) + (ty + 2) * MW;
            const T pc1 = M1[om];
            const T gx = grad1(M1[om + 1], M1[om - 1], inv_2dx);
            const T gy = grad1(M1[om + MW], M1[om - MW], inv_2dx);
            const T gz = grad1(M2[om], M0[om], inv_2dx);
            const T fac = sharpen_factor(pc1, gx, gy, gz, d2, hg);
            s_q2x[q2new * Q2XS + (tx + 1) + ty * Q2XW] = fac * gx;
            s_q2y[q2new * Q2YS + tx + (ty + 1) * TX] = fac * gy;
            T q2zn = fac * gz;
            if constexpr (WALLS) {  // walled z: the ghost planes next to the walls mirror exactly
                if (wz && to + 1 == 0) q2z = -q2zn;   // plane -1, from plane 0
                if (wz && to + 1 == nz) q2zn = -q2z;  // plane nz, from plane nz-1
            }
            if (has_h2) {
                const T hgx = grad1(M1[h_om + 1], M1[h_om - 1], inv_2dx);
                const T hgy = grad1(M1[h_om + MW], M1[h_om - MW], inv_2dx);
                const T hgz = grad1(M2[h_om], M0[h_om], inv_2dx);
                const T hf = sharpen_factor(M1[h_om], hgx, hgy, hgz, d2, hg);
                if (h_axis == 0)
                    s_q2x[q2new * Q2XS + h_dst] = hf * hgx;
                else
                    s_q2y[q2new * Q2YS + h_dst] = hf * hgy;
            }
            const T pc = M0[om];
            const T szp = face_sum(pc, pc1), dzp = face_diff(pc, pc1);
            if (to >= k0 && to < k1 && active) {
                const T* qx = s_q2x + q2old * Q2XS + tx + ty * Q2XW;
                const T* qy = s_q2y + q2old * Q2YS + tx + ty * TX;
                const T pxm = M0[om - 1], pxp = M0[om + 1], pym = M0[om - MW], pyp = M0[om + MW];
                const T f2 = cell_rhs(face_sum(pxm, pc), face_sum(pc, pxp), face_sum(pym, pc),
                                      face_sum(pc, pyp), sz2, szp, face_diff(pxm, pc),
                                      face_diff(pc, pxp), face_diff(pym, pc), face_diff(pc, pyp),
                                      dz2, dzp, qx[0], qx[2], qy[0], qy[2 * TX], q2zm, q2zn,
                                      qa_u0[0], qa_u1[0], qa_v0[0], qa_v1[0], w2, qa_w1[0], a.nhs2,
                                      ge);
                const unsigned c = e_col[0];  // own cell (i0+tx, j0+ty): no wrap when active
                if (!SWEEP_B) foy.store(to, c, fma(a.c_y2, f2, qa_phi[0]));
                if constexpr (XOUT && !SWEEP_B)
                    if (a.out_phi) fophi.store(to, c, qa_phi[0]);
                if (SWEEP_B || a.out_acc) foacc.store(to, c, fma(a.c_acc2, f2, qa_acc[0]));
            }
            sz2 = szp;
            dz2 = dzp;
            q2zm = q2z;
            q2z = q2zn;
            w2 = qa_w1[0];
        }
        if constexpr (LAG) __syncthreads();  // the iteration's LDS writes visible to the next
    };

    if constexpr (LAG) {
        // five iterations of E1 alone (ya from plane k0-2 on), then E2 from t = k0-1 (q2 at
        // k0-1) to t = k1 (outputs of plane k1-1)
        iteration(IntC<0>(), IntC<0>(), tbeg);
        iteration(IntC<1>(), IntC<0>(), tbeg + 1);
        iteration(IntC<2>(), IntC<0>(), tbeg + 2);
        iteration(IntC<3>(), IntC<0>(), tbeg + 3);
        iteration(IntC<0>(), IntC<0>(), tbeg + 4);
        const int tend = k0 - 1 + 4 * ((k1 - k0 + 5) / 4);  // k0-1 .. k1, in groups of four
        for (int t = k0 - 1; t < tend; t += 4) {
            iteration(IntC<1>(), IntC<1>(), t);
            iteration(IntC<2>(), IntC<1>(), t + 1);
            iteration(IntC<3>(), IntC<1>(), t + 2);
            iteration(IntC<0>(), IntC<1>(), t + 3);
        }
    } else {
        iteration(IntC<0>(), IntC<0>(), tbeg);
        iteration(IntC<1>(), IntC<0>(), tbeg + 1);
        iteration(IntC<2>(), IntC<0>(), tbeg + 2);
        iteration(IntC<3>(), IntC<0>(), tbeg + 3);
        const int tend = k0 - 2 + 6 * ((k1 - k0 + 7) / 6);  // k0-2 .. k1-1, in groups of six
        for (int t = k0 - 2; t < tend; t += 6) {
            iteration(IntC<4>(), IntC<1>(), t);
            iteration(IntC<5>(), IntC<1>(), t + 1);
            iteration(IntC<0>(), IntC<1>(), t + 2);
            iteration(IntC<1>(), IntC<1>(), t + 3);
            iteration(IntC<2>(), IntC<1>(), t + 4);
            iteration(IntC<3>(), IntC<1>(), t + 5);
        }
    }
}

}  // namespace pf
