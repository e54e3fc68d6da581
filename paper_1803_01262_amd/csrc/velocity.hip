// Face velocity from separable Fourier modes of an edge vector potential, and the transpose.
//
// The potential component A_c(x, y, z) = sum_{m3,m2,m1} C[m3][m2][m1][c] X_c(m1, x) Y_c(m2, y)
// Z_c(m3, z) is evaluated by sum factorisation (contract x, then y, then z) instead of the
// M^3-term direct sum, and the last contraction is fused with the discrete curl so the edge
// potential is never stored. All arithmetic is double; the faces are written in the storage
// type. The transpose runs the same steps backwards: curl^T gathered per edge and projected
// onto the x sine tables in one pass, then projected along y and z, each output a plain serial
// sum (fixed order, deterministic).
#include <cmath>

#include "pf_cell.h"
#include "pf_internal.h"

namespace pf {

struct VelGeom {
    int n[3];
    int M;
    int nmax;
    double dx;
};

// sin(2 pi (m+1) (i + pos/2) / n_axis + phase[axis][m]): mode m along an axis at the nodes
// (pos 0) or mid-points (pos 1)
__device__ __forceinline__ double sine_value(const VelGeom& g, const double* phases, int axis,
                                             int pos, int m, int i)
{
    const double off = pos ? 0.5 : 0.0;
    return sin(2.0 * M_PI * (double)(m + 1) * ((double)i + off) / (double)g.n[axis] +
               phases[axis * g.M + m]);
}

// tab[((axis * 2 + pos) * M + m) * nmax + i] = sine_value(axis, pos, m, i), 0 past the axis end
__global__ void sine_table_kernel(VelGeom g, const double* __restrict__ phases, double* __restrict__ tab)
{
    const size_t total = (size_t)6 * g.M * g.nmax, nm = (size_t)g.nmax * g.M;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.nmax);
        const int m = (int)((e / g.nmax) % g.M);
        const int pos = (int)((e / nm) % 2);
        const int axis = (int)(e / (nm * 2));
        tab[e] = i < g.n[axis] ? sine_value(g, phases, axis, pos, m, i) : 0.0;
    }
}

// The x tables mode-fastest for the projection: xT[(pos * nx + i) * M + m] = sine_value(0, pos, m, i)
__global__ void sine_table_xT_kernel(VelGeom g, const double* __restrict__ phases, double* __restrict__ xT)
{
    const size_t total = (size_t)2 * g.n[0] * g.M, nm = (size_t)g.n[0] * g.M;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(e % g.M);
        const int i = (int)((e / g.M) % g.n[0]);
        const int pos = (int)(e / nm);
        xT[e] = sine_value(g, phases, 0, pos, m, i);
    }
}

__device__ __forceinline__ const double* table(const VelGeom& g, const double* tab, int axis,
                                               int pos, int m)
{
    return tab + ((size_t)(axis * 2 + pos) * g.M + m) * g.nmax;
}

// T1[c][m3][m2][i] = sum_m1 C[m3][m2][m1][c] X_c(m1, i);  X_c on the mid-points for c = 0
__global__ void contract_x_kernel(VelGeom g, const double* __restrict__ coef,
                                  const double* __restrict__ tab, double* __restrict__ T1)
{
    const int M = g.M, nx = g.n[0];
    const size_t total = (size_t)3 * M * M * nx;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % nx);
        const int m2 = (int)((e / nx) % M);
        const int m3 = (int)((e / ((size_t)nx * M)) % M);
        const int c = (int)(e / ((size_t)nx * M * M));
        double s = 0.0;
        for (int m1 = 0; m1 < M; ++m1)
            s = fma(coef[(((size_t)m3 * M + m2) * M + m1) * 3 + c], table(g, tab, 0, c == 0, m1)[i], s);
        T1[e] = s;
    }
}

// T2[c][m3][j][i] = sum_m2 T1[c][m3][m2][i] Y_c(m2, j);  Y_c on the mid-points for c = 1
__global__ void contract_y_kernel(VelGeom g, const double* __restrict__ T1,
                                  const double* __restrict__ tab, double* __restrict__ T2)
{
    const int M = g.M, nx = g.n[0], ny = g.n[1];
    const size_t total = (size_t)3 * M * ny * nx;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % nx);
        const int j = (int)((e / nx) % ny);
        const int m3 = (int)((e / ((size_t)nx * ny)) % M);
        const int c = (int)(e / ((size_t)nx * ny * M));
        const double* t1 = T1 + (((size_t)c * M + m3) * M) * nx + i;
        double s = 0.0;
        for (int m2 = 0; m2 < M; ++m2) s = fma(t1[(size_t)m2 * nx], table(g, tab, 1, c == 1, m2)[j], s);
        T2[e] = s;
    }
}

// A_c at edge (i, j, k) = sum_m3 T2[c][m3][j][i] Z_c(m3, k) (Z_c on the mid-points for c = 2),
// fused with the discrete curl. A thread owns one (i, j) column and KB consecutive planes (the
// workgroup's plane block): it
// loads the seven T2 columns its curl needs (A_x, A_y, A_z at (i, j); A_x, A_z at (i, j+1); A_y,
// A_z at (i+1, j)) once per mode and reuses them for all KB planes, and keeps A_x and A_y one
// plane further for the k+1 edges. Each edge potential is the same m3-ordered fma chain as a
// direct per-edge sum.
template <typename T, int KB>
__global__ void __launch_bounds__(256) curl_kernel(VelGeom g, const double* __restrict__ T2,
                                                   const double* __restrict__ tab,
                                                   T* __restrict__ U, T* __restrict__ V,
                                                   T* __restrict__ W)
{
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2], M = g.M;
    const size_t ms = (size_t)ny * nx, cs = (size_t)M * ms;
    const double* zn = table(g, tab, 2, 0, 0);  // Z_x and Z_y: nodes
    const double* zm = table(g, tab, 2, 1, 0);  // Z_z: mid-points
    // blockIdx.y picks the plane block, so the table reads below are uniform across the workgroup
    const int k0 = (int)blockIdx.y * KB;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < ms) {
        const int i = (int)(e % nx);
        const int j = (int)(e / nx);
        const int ip = wrap1(i + 1, nx), jp = wrap1(j + 1, ny);
        const size_t o = (size_t)j * nx + i, o_jp = (size_t)jp * nx + i, o_ip = (size_t)j * nx + ip;
        int kq[KB + 1];  // plane of slot q; slots past the grid wrap and are not stored
#pragma unroll
        for (int q = 0; q <= KB; ++q) kq[q] = (k0 + q) % nz;
        double ax[KB + 1], ay[KB + 1], az[KB], ax_jp[KB], az_jp[KB], ay_ip[KB], az_ip[KB];
#pragma unroll
        for (int q = 0; q <= KB; ++q) ax[q] = ay[q] = 0.0;
#pragma unroll
        for (int q = 0; q < KB; ++q) az[q] = ax_jp[q] = az_jp[q] = ay_ip[q] = az_ip[q] = 0.0;
        for (int m3 = 0; m3 < M; ++m3) {
            const double* t = T2 + (size_t)m3 * ms;
            const double a0 = t[o], a0_jp = t[o_jp];
            const double a1 = t[cs + o], a1_ip = t[cs + o_ip];
            const double a2 = t[2 * cs + o], a2_jp = t[2 * cs + o_jp], a2_ip = t[2 * cs + o_ip];
            const double* zn_m = zn + (size_t)m3 * g.nmax;
            const double* zm_m = zm + (size_t)m3 * g.nmax;
#pragma unroll
            for (int q = 0; q <= KB; ++q) {
                const double z = zn_m[kq[q]];
                ax[q] = fma(a0, z, ax[q]);
                ay[q] = fma(a1, z, ay[q]);
                if (q < KB) {
                    ax_jp[q] = fma(a0_jp, z, ax_jp[q]);
                    ay_ip[q] = fma(a1_ip, z, ay_ip[q]);
                    const double zz = zm_m[kq[q]];
                    az[q] = fma(a2, zz, az[q]);
                    az_jp[q] = fma(a2_jp, zz, az_jp[q]);
                    az_ip[q] = fma(a2_ip, zz, az_ip[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < KB; ++q)
            if (k0 + q < nz) {
                const size_t c = (size_t)(k0 + q) * ms + o;
                U[c] = (T)((((az_jp[q] - az[q]) - ay[q + 1]) + ay[q]) / g.dx);
                V[c] = (T)((((ax[q + 1] - ax[q]) - az_ip[q]) + az[q]) / g.dx);
                W[c] = (T)((((ay_ip[q] - ay[q]) - ax_jp[q]) + ax[q]) / g.dx);
            }
    }
}

// ------------------------------------------------------------------ transpose
// Edge cotangent Abar = curl^T (Ubar, Vbar, Wbar) gathered on the fly and projected onto the x
// sine tables: P1[c][k][j][m1] = sum_i X_c(m1, i) Abar_c[k][j][i], a serial sum over i per
// output. A group of MC lanes takes one (k, j) row, one lane per mode of the current chunk of MC
// modes, so a wave covers 64 / MC rows. For each run of 64 x-positions the wave first gathers
// Abar of its rows with one coalesced load per array and row (lane = x-position) into LDS, then
// every lane adds the run to its three sums; the table is mode-fastest (xT), so a group's table
// reads are consecutive.
template <typename T, int MC>
__global__ void __launch_bounds__(256) curl_T_project_x_kernel(VelGeom g, const T* __restrict__ gU,
                                                              const T* __restrict__ gV,
                                                              const T* __restrict__ gW,
                                                              const double* __restrict__ xT,
                                                              double* __restrict__ P1)
{
    constexpr int RPW = 64 / MC;  // rows per wave
    constexpr int RS = 3 * 64 + 1;  // LDS doubles per row (padded: the groups hit distinct banks)
    __shared__ double sab[4][RPW][RS];
    __shared__ double sxt[2][64 * MC];  // the run's x tables for the mode chunk, mid-points / nodes
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2], M = g.M;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane / MC, mm = lane % MC;
    const long long rows = (long long)nz * ny;
    const long long row0 = ((long long)blockIdx.x * 4 + wave) * RPW;  // first row of this wave
    const long long row = row0 + grp;                                   // this lane's row
    const double inv = 1.0 / g.dx;
    const double* xmid = xT + (size_t)nx * M;  // X_x: mid-points; X_y, X_z: nodes (xT itself)
    double* my = sab[wave][0];
    for (int m0 = 0; m0 < M; m0 += MC) {
        const int m = m0 + mm < M ? m0 + mm : M - 1;  // lanes past the last mode idle along
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int i0 = 0; i0 < nx; i0 += 64) {
            const int i = i0 + lane;
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                double ab0 = 0.0, ab1 = 0.0, ab2 = 0.0;
                const long long rr = row0 + r;
                if (rr < rows && i < nx) {
                    const int j = (int)(rr % ny), k = (int)(rr / ny);
                    const int jm = wrap1(j - 1, ny), km = wrap1(k - 1, nz), im = i == 0 ? nx - 1 : i - 1;
                    const size_t o = ((size_t)k * ny + j) * nx;
                    const size_t o_km = ((size_t)km * ny + j) * nx;
                    const size_t o_jm = ((size_t)k * ny + jm) * nx;
                    // Ax(k) enters V(k-1) with +1 and V(k) with -1; W(j-1) with -1 and W(j) with +1
                    ab0 = ((((double)gV[o_km + i] - (double)gV[o + i]) - (double)gW[o_jm + i]) +
                           (double)gW[o + i]) * inv;
                    // Ay(k) enters U(k-1) with -1 and U(k) with +1; W(i-1) with +1 and W(i) with -1
                    ab1 = ((-(double)gU[o_km + i] + (double)gU[o + i]) + (double)gW[o + im] -
                           (double)gW[o + i]) * inv;
                    // Az(j) enters U(j-1) with +1 and U(j) with -1; V(i-1) with -1 and V(i) with +1
                    ab2 = ((((double)gU[o_jm + i] - (double)gU[o + i]) - (double)gV[o + im]) +
                           (double)gV[o + i]) * inv;
                }
                my[r * RS + lane] = ab0;
                my[r * RS + 64 + lane] = ab1;
                my[r * RS + 128 + lane] = ab2;
            }
            const int cnt = nx - i0 < 64 ? nx - i0 : 64;
            // the workgroup stages the x tables of this run and mode chunk (padded modes repeat
            // the last one, as the lanes past it do)
            for (int e = threadIdx.x; e < 64 * MC; e += 256) {
                const int ii = e / MC, mc = m0 + e % MC < M ? m0 + e % MC : M - 1;
                const size_t t = (size_t)(i0 + (ii < cnt ? ii : 0)) * M + mc;
                sxt[0][e] = xmid[t];
                sxt[1][e] = xT[t];
            }
            __syncthreads();
            if (row < rows) {
                const double* A = my + grp * RS;
                for (int ii = 0; ii < cnt; ++ii) {
                    const double xn = sxt[1][ii * MC + mm];
                    s0 = fma(sxt[0][ii * MC + mm], A[ii], s0);
                    s1 = fma(xn, A[64 + ii], s1);
                    s2 = fma(xn, A[128 + ii], s2);
                }
            }
            __syncthreads();
        }
        if (row < rows && m0 + mm < M) {
            const int j = (int)(row % ny), k = (int)(row / ny);
            P1[(((size_t)0 * nz + k) * ny + j) * M + m] = s0;
            P1[(((size_t)1 * nz + k) * ny + j) * M + m] = s1;
            P1[(((size_t)2 * nz + k) * ny + j) * M + m] = s2;
        }
    }
}

// P2[c][k][m2][m1] = sum_j Y_c(m2, j) P1[c][k][j][m1]
__global__ void project_y_kernel(VelGeom g, const double* __restrict__ P1,
                                 const double* __restrict__ tab, double* __restrict__ P2)
{
    const int M = g.M, ny = g.n[1], nz = g.n[2];
    const size_t total = (size_t)3 * nz * M * M;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int m1 = (int)(e % M);
        const int m2 = (int)((e / M) % M);
        const size_t ck = e / ((size_t)M * M);  // (c, k)
        const int c = (int)(ck / nz);
        const double* y = table(g, tab, 1, c == 1, m2);
        const double* p1 = P1 + ck * (size_t)ny * M + m1;
        double s = 0.0;
        for (int j = 0; j < ny; ++j) s = fma(y[j], p1[(size_t)j * M], s);
        P2[e] = s;
    }
}

// coef_grad[m3][m2][m1][c] += sum_k Z_c(m3, k) P2[c][k][m2][m1]
__global__ void project_z_kernel(VelGeom g, const double* __restrict__ P2,
                                 const double* __restrict__ tab, double* __restrict__ cg)
{
    const int M = g.M, nz = g.n[2];
    const int total = 3 * M * M * M;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int c = e % 3;
        const int m1 = (e / 3) % M;
        const int m2 = (e / (3 * M)) % M;
        const int m3 = e / (3 * M * M);
        const double* z = table(g, tab, 2, c == 2, m3);
        const double* p2 = P2 + (size_t)c * nz * M * M + (size_t)m2 * M + m1;
        double s = 0.0;
        for (int k = 0; k < nz; ++k) s = fma(z[k], p2[(size_t)k * M * M], s);
        cg[e] += s;
    }
}

static VelGeom geom(int nx, int ny, int nz, double dx, int M)
{
    VelGeom g;
    g.n[0] = nx;
    g.n[1] = ny;
    g.n[2] = nz;
    g.M = M;
    g.nmax = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);
    g.dx = dx;
    return g;
}

static size_t table_doubles(const VelGeom& g) { return (size_t)6 * g.M * g.nmax; }

size_t velocity_scratch_doubles(int nx, int ny, int nz, int M)
{
    const VelGeom g = geom(nx, ny, nz, 1.0, M);
    const size_t synth = (size_t)3 * M * M * nx + (size_t)3 * M * ny * nx;
    const size_t grad = (size_t)2 * nx * M + (size_t)3 * nz * ny * M + (size_t)3 * nz * M * M;
    return table_doubles(g) + (synth > grad ? synth : grad);
}

static unsigned blocks_for(size_t n)
{
    size_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    return (unsigned)(b ? b : 1);
}

template <typename T>
hipError_t launch_velocity(int nx, int ny, int nz, double dx, int M, const double* phases,
                           const double* coeffs, T* U, T* V, T* W, double* scratch, hipStream_t st)
{
    const VelGeom g = geom(nx, ny, nz, dx, M);
    double* tab = scratch;
    double* T1 = tab + table_doubles(g);
    double* T2 = T1 + (size_t)3 * M * M * nx;
    hipLaunchKernelGGL(sine_table_kernel, dim3(blocks_for(table_doubles(g))), dim3(256), 0, st, g,
                       phases, tab);
    hipLaunchKernelGGL(contract_x_kernel, dim3(blocks_for((size_t)3 * M * M * nx)), dim3(256), 0,
                       st, g, coeffs, tab, T1);
    hipLaunchKernelGGL(contract_y_kernel, dim3(blocks_for((size_t)3 * M * ny * nx)), dim3(256), 0,
                       st, g, T1, tab, T2);
    constexpr int KB = 8;
    const size_t cols = (size_t)nx * ny;
    if ((cols + 255) / 256 > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL((curl_kernel<T, KB>), dim3((unsigned)((cols + 255) / 256), (nz + KB - 1) / KB),
                       dim3(256), 0, st, g, T2, tab, U, V, W);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_velocity_grad(int nx, int ny, int nz, double dx, int M, const double* phases,
                                const T* gU, const T* gV, const T* gW, double* coeff_grad,
                                double* scratch, hipStream_t st)
{
    const VelGeom g = geom(nx, ny, nz, dx, M);
    double* tab = scratch;
    double* xT = tab + table_doubles(g);
    double* P1 = xT + (size_t)2 * nx * M;
    double* P2 = P1 + (size_t)3 * nz * ny * M;
    hipLaunchKernelGGL(sine_table_kernel, dim3(blocks_for(table_doubles(g))), dim3(256), 0, st, g,
                       phases, tab);
    hipLaunchKernelGGL(sine_table_xT_kernel, dim3(blocks_for((size_t)2 * nx * M)), dim3(256), 0, st,
                       g, phases, xT);
    const long long rows = (long long)nz * ny;
    if (M <= 8) {  // 8 rows per wave, 32 per workgroup
        const long long blocks = (rows + 31) / 32;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
        hipLaunchKernelGGL((curl_T_project_x_kernel<T, 8>), dim3((unsigned)blocks), dim3(256), 0, st,
                           g, gU, gV, gW, xT, P1);
    } else {  // 4 rows per wave, 16 per workgroup
        const long long blocks = (rows + 15) / 16;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
        hipLaunchKernelGGL((curl_T_project_x_kernel<T, 16>), dim3((unsigned)blocks), dim3(256), 0, st,
                           g, gU, gV, gW, xT, P1);
    }
    hipLaunchKernelGGL(project_y_kernel, dim3(blocks_for((size_t)3 * nz * M * M)), dim3(256), 0,
                       st, g, P1, tab, P2);
    hipLaunchKernelGGL(project_z_kernel, dim3(blocks_for((size_t)3 * M * M * M)), dim3(256), 0, st,
                       g, P2, tab, coeff_grad);
    return hipGetLastError();
}

template hipError_t launch_velocity<float>(int, int, int, double, int, const double*, const double*,
                                           float*, float*, float*, double*, hipStream_t);
template hipError_t launch_velocity<double>(int, int, int, double, int, const double*,
                                            const double*, double*, double*, double*, double*,
                                            hipStream_t);
template hipError_t launch_velocity_grad<float>(int, int, int, double, int, const double*,
                                                const float*, const float*, const float*, double*,
                                                double*, hipStream_t);
template hipError_t launch_velocity_grad<double>(int, int, int, double, int, const double*,
                                                 const double*, const double*, const double*,
                                                 double*, double*, hipStream_t);

}  // namespace pf
