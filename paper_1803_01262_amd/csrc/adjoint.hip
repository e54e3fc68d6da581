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

// Cotangent of a face's flux on a non-uniform mesh: kap of the low cell over its width minus kap
// of the high cell over its width, both products rounded (no contraction in this build), so that
// across a wall, where the mirror makes the two products equal, it is exactly zero.
template <typename T>
__device__ __forceinline__ T nu_face(T k_lo, T iw_lo, T k_hi, T iw_hi)
{
    return k_lo * iw_lo - k_hi * iw_hi;
}

template <typename T>
__global__ void __launch_bounds__(256) adjoint_stage_kernel(AdjArgs<T> a)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= a.nx || j >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    // periodic wrap, or the mirror across the walls of a walled axis
    auto mx = [&](int v) { return (a.walls & 1) ? reflectn(v, nx) : wrapn(v, nx); };
    auto my = [&](int v) { return (a.walls & 2) ? reflectn(v, ny) : wrapn(v, ny); };
    auto mz = [&](int v) { return (a.walls & 4) ? reflectn(v, nz) : wrapn(v, nz); };
    auto idx = [&](int di, int dj, int dk) -> size_t {
        return ((size_t)mz(k + dk) * ny + my(j + dj)) * nx + mx(i + di);
    };
    auto Y = [&](int di, int dj, int dk) -> T { return a.y[idx(di, dj, dk)]; };
    auto K = [&](int di, int dj, int dk) -> T { return a.kap_scale * a.kap_in[idx(di, dj, dk)]; };
    // cotangent of the flux on the low ax-face of cell (di, dj, dk)
    auto Fb = [&](int di, int dj, int dk, int ax) -> T {
        return adj_face(K(di - (ax == 0), dj - (ax == 1), dk - (ax == 2)), K(di, dj, dk), a.inv_dx);
    };
    // gbar (all three components) and the local (1-2y)(n.qbar) term of cell (di, dj, dk)
    auto cell = [&](int di, int dj, int dk, T gb[3], T& local) {
        const T p = Y(di, dj, dk);
        T g[3];
        g[0] = grad1(Y(di + 1, dj, dk), Y(di - 1, dj, dk), a.inv_2dx);
        g[1] = grad1(Y(di, dj + 1, dk), Y(di, dj - 1, dk), a.inv_2dx);
        g[2] = grad1(Y(di, dj, dk + 1), Y(di, dj, dk - 1), a.inv_2dx);
        T qb[3];
        qb[0] = -a.hg * (Fb(di, dj, dk, 0) + Fb(di + 1, dj, dk, 0));
        qb[1] = -a.hg * (Fb(di, dj, dk, 1) + Fb(di, dj + 1, dk, 1));
        qb[2] = -a.hg * (Fb(di, dj, dk, 2) + Fb(di, dj, dk + 1, 2));
        local = adj_cell(p, g, qb, a.delta2, gb);
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
    // both per-cell operands are read before either store: lam_out may alias lamp
    const T lb = a.lam_out ? a.lam_base[c] : T(0), lp = a.kap_out ? a.lamp[c] : T(0);
    if (a.lam_out) a.lam_out[c] = lb + ybar;
    if (a.kap_out) a.kap_out[c] = fma(a.ka, ybar, a.kb * lp);
}

// Tiled form of the same stage adjoint: a TX x TY workgroup marches kz planes along z, with
// three-plane LDS rings (two-cell halo) of the stage input and of the cotangent, the x- and
// y-components of gbar of the current and next plane in LDS (one-cell halo in their own
// direction), and the z-component of gbar, the local term, the z-face cotangent and W carried in
// registers. Iteration k computes gbar at plane k+1 and finishes plane k. Same per-cell
// arithmetic, in the same order, as the plain kernel above, so the two agree bitwise. Memory
// access, ring slots and the march in whole groups of six iterations follow the forward tiled
// kernel (buffer descriptors; BIG for arrays of 4 GiB or more).
// WALLS: the form that reads the stage input and the cotangent through mirror indices on the
// walled axes of a.walls.
// NU: the non-uniform mesh form (a.nu set; arrays under 4 GiB), the steps of
// adjoint_stage_nu_kernel in the same order: the coefficients of the tile's columns and rows sit
// in LDS (mapped like the loads), those of the z planes are uniform loads per iteration.
template <typename T, int TX, int TY, bool BIG, bool WALLS = false, bool NU = false>
__global__ void __launch_bounds__(TX* TY) adjoint_tiled_kernel(AdjArgs<T> a, int tiles_x, int tiles_y,
                                                               int kz)
{
    constexpr int NT = TX * TY;
    constexpr int PW = TX + 4, PH = TY + 4, PS = PW * PH;
    constexpr int GXW = TX + 2, GXS = GXW * TY;
    constexpr int GYS = TX * (TY + 2);
    constexpr int NL = (PS + NT - 1) / NT;
    static_assert(NT >= 2 * TX + 2 * TY, "halo ring needs one thread per halo cell");
    static_assert(!NU || NT >= PW + PH, "one thread per coefficient column and row");
    static_assert(!(NU && BIG), "the non-uniform form takes arrays under 4 GiB");
    __shared__ T sy[3 * PS];
    __shared__ T sk[3 * PS];
    __shared__ T sgx[2 * GXS];
    __shared__ T sgy[2 * GYS];
    __shared__ T scx[NU ? kNuCols * PW : 1];  // column-major per coefficient
    __shared__ T scy[NU ? kNuCols * PH : 1];

    int b = xcd_tile_order(blockIdx.x, gridDim.x);
    const int ti = b % tiles_x;
    b /= tiles_x;
    const int tj = b % tiles_y;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t plane = (size_t)nx * ny;
    const int i0 = ti * TX, j0 = tj * TY, k0 = (b / tiles_y) * kz;
    const int k1 = min(k0 + kz, nz);
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool active = (i < nx) && (j < ny);
    const int iw = wrapn(i, nx), jw = wrapn(j, ny);
    constexpr unsigned ES = sizeof(T);  // byte offsets within a plane
    const unsigned col = (unsigned)(jw * nx + iw) * ES;
    const unsigned col_xp = (unsigned)(jw * nx + wrapn(i + 1, nx)) * ES;
    const unsigned col_yp = (unsigned)(wrapn(j + 1, ny) * nx + iw) * ES;
    // plane-load index maps: periodic wrap, or the mirror across walls
    const bool wx = WALLS && (a.walls & 1), wy = WALLS && (a.walls & 2), wz = WALLS && (a.walls & 4);
    auto mapx = [&](int v) { return WALLS && wx ? reflectn(v, nx) : wrapn(v, nx); };
    auto mapy = [&](int v) { return WALLS && wy ? reflectn(v, ny) : wrapn(v, ny); };
    auto mapz = [&](int v) { return WALLS && wz ? reflectz(v, nz) : wrapz(v, nz); };

    if constexpr (NU) {  // read by the first iteration, after its barriers
        if (tid < PW) {
            const T* r = a.nu[0] + (size_t)mapx(i0 - 2 + tid) * kNuCols;
#pragma unroll
            for (int c = 0; c < kNuCols; ++c) scx[c * PW + tid] = r[c];
        } else if (tid < PW + PH) {
            const int t = tid - PW;
            const T* r = a.nu[1] + (size_t)mapy(j0 - 2 + t) * kNuCols;
#pragma unroll
            for (int c = 0; c < kNuCols; ++c) scy[c * PH + t] = r[c];
        }
    }
    auto CX = [&](int col, int c) -> T { return scx[col * PW + c]; };
    auto CY = [&](int col, int r) -> T { return scy[col * PH + r]; };
    // FP64 on 64x8 tiles keeps the coefficients of the thread's own column and row, and those of
    // planes k-1 .. k+2, in registers along the march (it runs two waves per SIMD either way;
    // 512^3 NU adjoint 19.2 against 21.6 ms reading them per iteration); FP32, and the smaller
    // FP64 tiles (where 256 registers would leave one wave per SIMD), read them per iteration
    // (LDS and uniform loads), which keeps FP32 at four waves per SIMD (10.9 against 13.1 ms)
    constexpr bool HOIST = NU && sizeof(T) == 8 && TX * TY >= 512;
    struct NuRow {
        T v[kNuCols];
    };
    auto load_row = [&](const T* tab, int m) -> NuRow {
        NuRow r;
#pragma unroll
        for (int c = 0; c < kNuCols; ++c) r.v[c] = tab[(size_t)m * kNuCols + c];
        return r;
    };
    NuRow ox[3], oy[3];  // columns i-1, i, i+1 and rows j-1, j, j+1
    if constexpr (HOIST) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ox[d] = load_row(a.nu[0], mapx(i0 + tid % TX - 1 + d));
            oy[d] = load_row(a.nu[1], mapy(j0 + tid / TX - 1 + d));
        }
    }
    // coefficient col of the thread's own column i-1+d, row j-1+d
    auto OX = [&](int col, int d) -> T {
        if constexpr (HOIST) return ox[d].v[col];
        else return CX(col, tid % TX + 1 + d);
    };
    auto OY = [&](int col, int d) -> T {
        if constexpr (HOIST) return oy[d].v[col];
        else return CY(col, tid / TX + 1 + d);
    };

    unsigned loff[NL];
    int lpos[NL];
#pragma unroll
    for (int s = 0; s < NL; ++s) {
        const int e = tid + s * NT;
        lpos[s] = e < PS ? e : -1;
        const int r = e / PW, c = e - r * PW;
        loff[s] = e < PS ? (unsigned)(mapy(j0 - 2 + r) * nx + mapx(i0 - 2 + c)) * ES : 0u;
    }
    // buffer descriptors for the stencil and velocity arrays; the cotangent and gradient arrays,
    // touched once per cell, go through a scalar plane pointer and a vector byte offset (which
    // keeps the scalar registers for the descriptors). The stores name T explicitly: inside the
    // generic lambda below, deduction from an fma() argument would see its host overload.
    const FieldRef<T, BIG> fy(a.y, plane, nz), fk(a.kap_in, plane, nz), fU(a.U, plane, nz),
        fV(a.V, plane, nz), fW(a.W, plane, nz);

    T pre_y[NL], pre_k[NL];
    auto fetch = [&](int kk) {
        const int kw = mapz(kk);
#pragma unroll
        for (int s = 0; s < NL; ++s)
            if (lpos[s] >= 0) {
                pre_y[s] = fy.load(kw, loff[s]);
                pre_k[s] = a.kap_scale * fk.load(kw, loff[s]);
            }
    };
    auto commit = [&](int slot) {
#pragma unroll
        for (int s = 0; s < NL; ++s)
            if (lpos[s] >= 0) {
                sy[slot * PS + lpos[s]] = pre_y[s];
                sk[slot * PS + lpos[s]] = pre_k[s];
            }
    };
    int h_o = -1, h_dst = 0, h_axis = 0;
    if (tid < 2 * TY) {
        const int side = tid / TY, r = tid - side * TY;
        h_o = (r + 2) * PW + (side ? TX + 2 : 1);
        h_dst = r * GXW + (side ? TX + 1 : 0);
        h_axis = 0;
    } else if (tid < 2 * TY + 2 * TX) {
        const int t2 = tid - 2 * TY;
        const int side = t2 / TX, c = t2 - side * TX;
        h_o = (side ? TY + 2 : 1) * PW + c + 2;
        h_dst = (side ? TY + 1 : 0) * TX + c;
        h_axis = 1;
    }
    const T inv_dx = a.inv_dx, inv_2dx = a.inv_2dx, d2 = a.delta2, hs = a.hs, hg = a.hg, ge = a.ge;
    const int o = (ty + 2) * PW + (tx + 2);

    // gbar and local term of the cell at LDS offset q of plane k+1
    auto cell = [&](const T* Y0, const T* Y1, const T* Y2, const T* K0, const T* K1, const T* K2,
                    int q, T gb[3]) -> T {
        T g[3], qb[3];
        g[0] = grad1(Y1[q + 1], Y1[q - 1], inv_2dx);
        g[1] = grad1(Y1[q + PW], Y1[q - PW], inv_2dx);
        g[2] = grad1(Y2[q], Y0[q], inv_2dx);
        qb[0] = -hg * (adj_face(K1[q - 1], K1[q], inv_dx) + adj_face(K1[q], K1[q + 1], inv_dx));
        qb[1] = -hg * (adj_face(K1[q - PW], K1[q], inv_dx) + adj_face(K1[q], K1[q + PW], inv_dx));
        qb[2] = -hg * (adj_face(K0[q], K1[q], inv_dx) + adj_face(K1[q], K2[q], inv_dx));
        return adj_cell(Y1[q], g, qb, d2, gb);
    };
    // the same on a non-uniform mesh, the cell at LDS offset q: sx, sy, sz1 the inverse gradient
    // spans of its column, row and plane k+1; wxm..wxp, wym..wyp the inverse widths of the
    // columns and rows around it, iz0..iz2 those of planes k, k+1, k+2
    auto cell_nu = [&](const T* Y0, const T* Y1, const T* Y2, const T* K0, const T* K1,
                       const T* K2, int q, T sx, T sy, T wxm, T wxc, T wxp, T wym, T wyc, T wyp,
                       T sz1, T iz0, T iz1, T iz2, T gb[3]) -> T {
        T g[3], qb[3];
        g[0] = (Y1[q + 1] - Y1[q - 1]) * sx;
        g[1] = (Y1[q + PW] - Y1[q - PW]) * sy;
        g[2] = (Y2[q] - Y0[q]) * sz1;
        qb[0] = -a.nu_hg * (nu_face(K1[q - 1], wxm, K1[q], wxc) + nu_face(K1[q], wxc, K1[q + 1], wxp));
        qb[1] = -a.nu_hg *
                (nu_face(K1[q - PW], wym, K1[q], wyc) + nu_face(K1[q], wyc, K1[q + PW], wyp));
        qb[2] = -a.nu_hg * (nu_face(K0[q], iz0, K1[q], iz1) + nu_face(K1[q], iz1, K2[q], iz2));
        return adj_cell(Y1[q], g, qb, d2, gb);
    };
    const int h_r = h_o >= 0 ? h_o / PW : 0, h_c = h_o >= 0 ? h_o - h_r * PW : 0;

    fetch(k0 - 2);
    commit(0);
    fetch(k0 - 1);
    commit(1);
    fetch(k0);
    // FP64: the z-plane coefficients of planes k-1 .. k+2 of iteration k, handed down the march
    NuRow zr[4];
    if constexpr (HOIST) {
#pragma unroll
        for (int d = 0; d < 4; ++d) zr[d] = load_row(a.nu[2], mapz(k0 - 3 + d));
    }
    // handed from plane to plane: gbar_z at k-1 and k, the local term and z-face cotangent of
    // plane k, W at k
    T gz_prev = T(0), gz_cur = T(0), loc_cur = T(0), fbz_cur = T(0), w0 = T(0);
    // the per-cell operands of iteration k (velocities, gradient and cotangent values of plane k,
    // the z-face gradient of plane k+1, W at k+1), loaded one iteration ahead so that their
    // latency spans a whole iteration; each is read only where the iteration uses it, and every
    // cell's values are written by this thread alone, at the iteration that reads them
    T nu0, nu1, nv0, nv1, ngu, ngv, ngw, nlb, nlp, nw1;
    auto load_ops = [&](int k) {
        const bool out_plane = k >= k0 && k < k1;
        const bool zplane = k + 1 >= k0 && k + 1 < k1;
        nw1 = fW.load(wrapz(k + 1, nz), col);
        const size_t ok = (size_t)(k < 0 ? 0 : k) * plane, ok1 = ok + (k < 0 ? 0 : plane);
        if (out_plane) {
            nu0 = fU.load(k, col);
            nu1 = fU.load(k, col_xp);
            nv0 = fV.load(k, col);
            nv1 = fV.load(k, col_yp);
            if (a.gU) ngu = ldg(a.gU + ok, col);
            if (a.gV) ngv = ldg(a.gV + ok, col);
            if (a.lam_out) nlb = ldg(a.lam_base + ok, col);
            if (a.kap_out) nlp = ldg(a.lamp + ok, col);
        }
        if (zplane && a.gW) ngw = ldg(a.gW + ok1, col);
    };
    load_ops(k0 - 2);
    // R = (k - k0 + 2) mod 6 fixes the ring slots at compile time; iterations past the chunk end
    // compute on wrapped planes and store nothing
    auto iteration = [&](auto RC, int k) {
        constexpr int R = decltype(RC)::value;
        constexpr int s0 = R % 3, s1 = (R + 1) % 3, s2 = (R + 2) % 3;  // planes k, k+1, k+2
        constexpr int q0 = R & 1, q1 = (R + 1) & 1;
        __syncthreads();
        commit(s2);
        fetch(k + 3);
        const bool out_plane = k >= k0 && k < k1;
        const bool zplane = k + 1 >= k0 && k + 1 < k1;  // plane k+1, whose low z-face is done here
        // element offsets of planes k and k+1, used only where those planes are in the chunk
        const size_t ok = (size_t)(k < 0 ? 0 : k) * plane, ok1 = ok + (k < 0 ? 0 : plane);
        const T w1 = nw1, u0 = nu0, u1 = nu1, v0 = nv0, v1 = nv1, gu = ngu, gv = ngv, gw = ngw,
                lb = nlb, lp = nlp;
        load_ops(k + 1);
        __syncthreads();

        const T *Y0 = sy + s0 * PS, *Y1 = sy + s1 * PS, *Y2 = sy + s2 * PS;
        const T *K0 = sk + s0 * PS, *K1 = sk + s1 * PS, *K2 = sk + s2 * PS;
        T gb[3];
        T loc_next, fbz_next;  // fbz_next: the z-face between planes k and k+1
        // coefficient col of plane k+dk (dk = -1 .. 2)
        auto ZC = [&](int col, int dk) -> T {
            if constexpr (HOIST) return zr[dk + 1].v[col];
            else return a.nu[2][(size_t)mapz(k + dk) * kNuCols + col];
        };
        NuRow z3;
        if constexpr (HOIST) z3 = load_row(a.nu[2], mapz(k + 3));  // for the next iteration
        // inverse widths of planes k, k+1, k+2 and inverse gradient span of plane k+1
        T iz0 = T(0), iz1 = T(0), iz2 = T(0), sz1 = T(0);
        if constexpr (NU) {
            iz0 = ZC(kNuInvW, 0);
            iz1 = ZC(kNuInvW, 1);
            iz2 = ZC(kNuInvW, 2);
            sz1 = ZC(kNuInvSpan, 1);
            loc_next = cell_nu(Y0, Y1, Y2, K0, K1, K2, o, OX(kNuInvSpan, 1), OY(kNuInvSpan, 1),
                               OX(kNuInvW, 0), OX(kNuInvW, 1), OX(kNuInvW, 2), OY(kNuInvW, 0),
                               OY(kNuInvW, 1), OY(kNuInvW, 2), sz1, iz0, iz1, iz2, gb);
            fbz_next = nu_face(K0[o], iz0, K1[o], iz1);
        } else {
            loc_next = cell(Y0, Y1, Y2, K0, K1, K2, o, gb);
            fbz_next = adj_face(K0[o], K1[o], inv_dx);
        }
        sgx[q1 * GXS + ty * GXW + tx + 1] = gb[0];
        sgy[q1 * GYS + (ty + 1) * TX + tx] = gb[1];
        const T gz_next = gb[2];
        if (h_o >= 0) {
            T hb[3];
            if constexpr (NU)
                (void)cell_nu(Y0, Y1, Y2, K0, K1, K2, h_o, CX(kNuInvSpan, h_c), CY(kNuInvSpan, h_r),
                              CX(kNuInvW, h_c - 1), CX(kNuInvW, h_c), CX(kNuInvW, h_c + 1),
                              CY(kNuInvW, h_r - 1), CY(kNuInvW, h_r), CY(kNuInvW, h_r + 1),
                              sz1, iz0, iz1, iz2, hb);
            else
                (void)cell(Y0, Y1, Y2, K0, K1, K2, h_o, hb);
            if (h_axis == 0)
                sgx[q1 * GXS + h_dst] = hb[0];
            else
                sgy[q1 * GYS + h_dst] = hb[1];
        }
        if (zplane && active && a.gW) stg<T>(a.gW + ok1, col, fma(-hs * (Y0[o] + Y1[o]), fbz_next, gw));
        if constexpr (NU) {
            if (out_plane && active) {
                // diffusive coefficients of the six faces: gamma eps_face / centre distance
                const T dzl = ZC(kNuInvDist, 0), dzh = ZC(kNuInvDist, 1);
                T exl, exh, eyl, eyh, ezl, ezh;
                if (a.nu_eps_mode == 1) {  // eps of a cell ~ its largest width
                    const T wx = OX(kNuWidth, 1), wy = OY(kNuWidth, 1), wz = ZC(kNuWidth, 0);
                    const T mc = fmax(wx, fmax(wy, wz));
                    const T hh = a.nu_ge * T(0.5);
                    exl = hh * (fmax(OX(kNuWidth, 0), fmax(wy, wz)) + mc) * OX(kNuInvDist, 1);
                    exh = hh * (mc + fmax(OX(kNuWidth, 2), fmax(wy, wz))) * OX(kNuInvDist, 2);
                    eyl = hh * (fmax(wx, fmax(OY(kNuWidth, 0), wz)) + mc) * OY(kNuInvDist, 1);
                    eyh = hh * (mc + fmax(wx, fmax(OY(kNuWidth, 2), wz))) * OY(kNuInvDist, 2);
                    ezl = hh * (fmax(wx, fmax(wy, ZC(kNuWidth, -1))) + mc) * dzl;
                    ezh = hh * (mc + fmax(wx, fmax(wy, ZC(kNuWidth, 1)))) * dzh;
                } else {
                    exl = a.nu_ge * OX(kNuInvDist, 1);
                    exh = a.nu_ge * OX(kNuInvDist, 2);
                    eyl = a.nu_ge * OY(kNuInvDist, 1);
                    eyh = a.nu_ge * OY(kNuInvDist, 2);
                    ezl = a.nu_ge * dzl;
                    ezh = a.nu_ge * dzh;
                }
                T ybar = loc_cur;
                // x faces
                const T wxm = OX(kNuInvW, 0), wxc = OX(kNuInvW, 1), wxp = OX(kNuInvW, 2);
                T lo = nu_face(K0[o - 1], wxm, K0[o], wxc), hi = nu_face(K0[o], wxc, K0[o + 1], wxp);
                ybar = fma(lo, fma(-hs, u0, exl), ybar);
                ybar = fma(hi, fma(-hs, u1, -exh), ybar);
                if (a.gU) stg<T>(a.gU + ok, col, fma(-hs * (Y0[o - 1] + Y0[o]), lo, gu));
                const T* GX = sgx + q0 * GXS + ty * GXW + tx;
                ybar = fma(GX[0], OX(kNuInvSpan, 0), ybar);
                ybar = fma(-GX[2], OX(kNuInvSpan, 2), ybar);
                // y faces
                const T wym = OY(kNuInvW, 0), wyc = OY(kNuInvW, 1), wyp = OY(kNuInvW, 2);
                lo = nu_face(K0[o - PW], wym, K0[o], wyc);
                hi = nu_face(K0[o], wyc, K0[o + PW], wyp);
                ybar = fma(lo, fma(-hs, v0, eyl), ybar);
                ybar = fma(hi, fma(-hs, v1, -eyh), ybar);
                if (a.gV) stg<T>(a.gV + ok, col, fma(-hs * (Y0[o - PW] + Y0[o]), lo, gv));
                const T* GY = sgy + q0 * GYS + ty * TX + tx;
                ybar = fma(GY[0], OY(kNuInvSpan, 0), ybar);
                ybar = fma(-GY[2 * TX], OY(kNuInvSpan, 2), ybar);
                // z faces
                ybar = fma(fbz_cur, fma(-hs, w0, ezl), ybar);
                ybar = fma(fbz_next, fma(-hs, w1, -ezh), ybar);
                ybar = fma(gz_prev, ZC(kNuInvSpan, -1), ybar);
                ybar = fma(-gz_next, ZC(kNuInvSpan, 1), ybar);
                if (a.lam_out) stg<T>(a.lam_out + ok, col, lb + ybar);
                if (a.kap_out) stg<T>(a.kap_out + ok, col, fma(a.ka, ybar, a.kb * lp));
            }
        } else if (out_plane && active) {
            T ybar = loc_cur;
            // x faces
            T lo = adj_face(K0[o - 1], K0[o], inv_dx), hi = adj_face(K0[o], K0[o + 1], inv_dx);
            ybar = fma(lo, fma(-hs, u0, ge), ybar);
            ybar = fma(hi, fma(-hs, u1, -ge), ybar);
            if (a.gU) stg<T>(a.gU + ok, col, fma(-hs * (Y0[o - 1] + Y0[o]), lo, gu));
            const T* GX = sgx + q0 * GXS + ty * GXW + tx;
            ybar = fma(GX[0] - GX[2], inv_2dx, ybar);
            // y faces
            lo = adj_face(K0[o - PW], K0[o], inv_dx);
            hi = adj_face(K0[o], K0[o + PW], inv_dx);
            ybar = fma(lo, fma(-hs, v0, ge), ybar);
            ybar = fma(hi, fma(-hs, v1, -ge), ybar);
            if (a.gV) stg<T>(a.gV + ok, col, fma(-hs * (Y0[o - PW] + Y0[o]), lo, gv));
            const T* GY = sgy + q0 * GYS + ty * TX + tx;
            ybar = fma(GY[0] - GY[2 * TX], inv_2dx, ybar);
            // z faces
            ybar = fma(fbz_cur, fma(-hs, w0, ge), ybar);
            ybar = fma(fbz_next, fma(-hs, w1, -ge), ybar);
            ybar = fma(gz_prev - gz_next, inv_2dx, ybar);
            if (a.lam_out) stg<T>(a.lam_out + ok, col, lb + ybar);
            if (a.kap_out) stg<T>(a.kap_out + ok, col, fma(a.ka, ybar, a.kb * lp));
        }
        gz_prev = gz_cur;
        gz_cur = gz_next;
        loc_cur = loc_next;
        fbz_cur = fbz_next;
        w0 = w1;
        if constexpr (HOIST) {
            zr[0] = zr[1];
            zr[1] = zr[2];
            zr[2] = zr[3];
            zr[3] = z3;
        }
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

// Non-uniform mesh form of the gather above (a.nu set), one thread per cell: the same steps with
// the mesh's per-axis coefficients, read from the forward's tables at the wrapped or mirrored
// index of each cell: the flux cotangent on the low face of cell X is kap[X-e] / h[X-e] -
// kap[X] / h[X]; the diffusive coefficient of that face gamma eps_face / (distance between the
// two cells' centres), eps_face the mean of the two cells' eps (mode 1: eps of a cell ~ its
// largest width over the axes longer than one cell); the gradient of cell X divides by the
// distance between its two neighbours' centres, and its transpose gathers
// gbar[c - e] / span[c - e] - gbar[c + e] / span[c + e]. Across a wall the mirror reads make the
// wall face's flux cotangent vanish and a ghost's gradient cotangent the negative of its
// partner's, as in the uniform form (the tables are mirror-symmetric).
template <typename T>
__global__ void __launch_bounds__(256) adjoint_stage_nu_kernel(AdjArgs<T> a)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z;
    if (i >= a.nx || j >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    auto mx = [&](int v) { return (a.walls & 1) ? reflectn(v, nx) : wrapn(v, nx); };
    auto my = [&](int v) { return (a.walls & 2) ? reflectn(v, ny) : wrapn(v, ny); };
    auto mz = [&](int v) { return (a.walls & 4) ? reflectn(v, nz) : wrapn(v, nz); };
    auto idx = [&](int di, int dj, int dk) -> size_t {
        return ((size_t)mz(k + dk) * ny + my(j + dj)) * nx + mx(i + di);
    };
    auto Y = [&](int di, int dj, int dk) -> T { return a.y[idx(di, dj, dk)]; };
    auto K = [&](int di, int dj, int dk) -> T { return a.kap_scale * a.kap_in[idx(di, dj, dk)]; };
    // column col of the table of axis ax at the cell (di, dj, dk)
    auto tab = [&](int ax, int di, int dj, int dk, int col) -> T {
        const int m = ax == 0 ? mx(i + di) : (ax == 1 ? my(j + dj) : mz(k + dk));
        return a.nu[ax][(size_t)m * kNuCols + col];
    };
    // largest width of a cell over the axes longer than one cell (a one-cell axis has width 0)
    auto wmax = [&](int di, int dj, int dk) -> T {
        return fmax(tab(0, di, dj, dk, kNuWidth), fmax(tab(1, di, dj, dk, kNuWidth), tab(2, di, dj, dk, kNuWidth)));
    };
    // cotangent of the flux on the low ax-face of cell (di, dj, dk)
    auto Fb = [&](int di, int dj, int dk, int ax) -> T {
        const int ex = ax == 0, ey = ax == 1, ez = ax == 2;
        return nu_face(K(di - ex, dj - ey, dk - ez), tab(ax, di - ex, dj - ey, dk - ez, kNuInvW),
                       K(di, dj, dk), tab(ax, di, dj, dk, kNuInvW));
    };
    // diffusive coefficient of the low ax-face of cell (di, dj, dk)
    auto gef = [&](int di, int dj, int dk, int ax) -> T {
        const int ex = ax == 0, ey = ax == 1, ez = ax == 2;
        const T d = tab(ax, di, dj, dk, kNuInvDist);
        if (a.nu_eps_mode == 1)
            return a.nu_ge * T(0.5) * (wmax(di - ex, dj - ey, dk - ez) + wmax(di, dj, dk)) * d;
        return a.nu_ge * d;
    };
    auto cell = [&](int di, int dj, int dk, T gb[3], T& local) {
        const T p = Y(di, dj, dk);
        T g[3];
        g[0] = (Y(di + 1, dj, dk) - Y(di - 1, dj, dk)) * tab(0, di, dj, dk, kNuInvSpan);
        g[1] = (Y(di, dj + 1, dk) - Y(di, dj - 1, dk)) * tab(1, di, dj, dk, kNuInvSpan);
        g[2] = (Y(di, dj, dk + 1) - Y(di, dj, dk - 1)) * tab(2, di, dj, dk, kNuInvSpan);
        T qb[3];
        qb[0] = -a.nu_hg * (Fb(di, dj, dk, 0) + Fb(di + 1, dj, dk, 0));
        qb[1] = -a.nu_hg * (Fb(di, dj, dk, 1) + Fb(di, dj + 1, dk, 1));
        qb[2] = -a.nu_hg * (Fb(di, dj, dk, 2) + Fb(di, dj, dk + 1, 2));
        local = adj_cell(p, g, qb, a.delta2, gb);
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
        const T fb_lo = Fb(0, 0, 0, ax);
        const T fb_hi = Fb(ex, ey, ez, ax);
        const T u_lo = vel[ax][c];
        const T u_hi = vel[ax][idx(ex, ey, ez)];
        ybar = fma(fb_lo, fma(-a.hs, u_lo, gef(0, 0, 0, ax)), ybar);
        ybar = fma(fb_hi, fma(-a.hs, u_hi, -gef(ex, ey, ez, ax)), ybar);
        if (velbar[ax]) velbar[ax][c] = fma(-a.hs * (Y(-ex, -ey, -ez) + yc), fb_lo, velbar[ax][c]);
        T gbm[3], gbp[3], dummy;
        cell(-ex, -ey, -ez, gbm, dummy);
        cell(ex, ey, ez, gbp, dummy);
        ybar = fma(gbm[ax], tab(ax, -ex, -ey, -ez, kNuInvSpan), ybar);
        ybar = fma(-gbp[ax], tab(ax, ex, ey, ez, kNuInvSpan), ybar);
    }
    const T lb = a.lam_out ? a.lam_base[c] : T(0), lp = a.kap_out ? a.lamp[c] : T(0);
    if (a.lam_out) a.lam_out[c] = lb + ybar;
    if (a.kap_out) a.kap_out[c] = fma(a.ka, ybar, a.kb * lp);
}

template <typename T>
hipError_t launch_adjoint_stage_nu(const AdjArgs<T>& a, hipStream_t st)
{
    if (!a.nu[0] || !a.nu[1] || !a.nu[2]) return hipErrorInvalidValue;
    dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4, a.nz);
    hipLaunchKernelGGL(adjoint_stage_nu_kernel<T>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}
template hipError_t launch_adjoint_stage_nu<float>(const AdjArgs<float>&, hipStream_t);
template hipError_t launch_adjoint_stage_nu<double>(const AdjArgs<double>&, hipStream_t);

template <typename T>
hipError_t launch_adjoint_stage_global(const AdjArgs<T>& a, hipStream_t st)
{
    dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4, a.nz);
    hipLaunchKernelGGL(adjoint_stage_kernel<T>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename T, int TX, int TY>
static hipError_t launch_adjoint_tiled(const AdjArgs<T>& a, int kz, bool big, hipStream_t st)
{
    const int tiles_x = (a.nx + TX - 1) / TX;
    const int tiles_y = (a.ny + TY - 1) / TY;
    if (a.nz <= 0 || tiles_x <= 0 || tiles_y <= 0 || kz < 0) return hipErrorInvalidValue;
    big = big || field_needs_big(a.nx, a.ny, a.nz, sizeof(T));
    using Kernel = void (*)(AdjArgs<T>, int, int, int);
    Kernel kern;
    if (a.nu[0]) {
        if (big) return launch_adjoint_stage_nu<T>(a, st);  // the plain form indexes 64-bit
        kern = a.walls ? adjoint_tiled_kernel<T, TX, TY, false, true, true>
                       : adjoint_tiled_kernel<T, TX, TY, false, false, true>;
    } else {
        kern = a.walls ? (big ? adjoint_tiled_kernel<T, TX, TY, true, true>
                              : adjoint_tiled_kernel<T, TX, TY, false, true>)
                       : (big ? adjoint_tiled_kernel<T, TX, TY, true, false>
                              : adjoint_tiled_kernel<T, TX, TY, false, false>);
    }
    if (kz == 0) {
        kz = launch_chunk_planes((const void*)kern, TX * TY, (long long)tiles_x * tiles_y, a.nz, 1);
        if (kz <= 0) return hipErrorInvalidDevice;
    }
    const long long blocks = (long long)tiles_x * tiles_y * ((a.nz + kz - 1) / kz);
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(TX * TY), 0, st, a, tiles_x, tiles_y, kz);
    return hipGetLastError();
}

// Tile shapes (x, y) of the tiled adjoint, widest first.
static const int kAdjTiles[][2] = {{64, 8}, {64, 4}, {32, 4}};
constexpr int kNumAdjTiles = (int)(sizeof(kAdjTiles) / sizeof(kAdjTiles[0]));

int adjoint_tile_index(int tx, int ty)
{
    for (int t = 0; t < kNumAdjTiles; ++t)
        if (kAdjTiles[t][0] == tx && kAdjTiles[t][1] == ty) return t;
    return -1;
}

// 64x8 unless 64-wide tiles pad more columns than 32-wide ones (then 32x4); chunks per launch.
// At 128^3 (MI355X) 64x8 is the fastest shape in FP32 and FP64 (an adjoint step 15 % faster
// than on 64x4).
int adjoint_default_tile(int nx, int ny, int nz)
{
    (void)ny;
    (void)nz;
    const int p64 = (nx + 63) / 64 * 64, p32 = (nx + 31) / 32 * 32;
    return p64 <= p32 ? 0 : 2;
}

template <typename T>
hipError_t launch_adjoint_stage(const AdjArgs<T>& a, int tile, int kz, bool big, hipStream_t st)
{
    switch (tile) {
    case 0: return launch_adjoint_tiled<T, 64, 8>(a, kz, big, st);
    case 1: return launch_adjoint_tiled<T, 64, 4>(a, kz, big, st);
    case 2: return launch_adjoint_tiled<T, 32, 4>(a, kz, big, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_adjoint_stage<float>(const AdjArgs<float>&, int, int, bool, hipStream_t);
template hipError_t launch_adjoint_stage<double>(const AdjArgs<double>&, int, int, bool, hipStream_t);
template hipError_t launch_adjoint_stage_global<float>(const AdjArgs<float>&, hipStream_t);
template hipError_t launch_adjoint_stage_global<double>(const AdjArgs<double>&, hipStream_t);

}  // namespace pf
