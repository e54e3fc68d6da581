// Face velocity from separable Fourier modes of an edge vector potential, and the transpose.
//
// The potential component A_c(x, y, z) = sum_{m3,m2,m1} C[m3][m2][m1][c] X_c(m1, x) Y_c(m2, y)
// Z_c(m3, z) is evaluated by sum factorisation (contract x, then y, then z) instead of the
// M^3-term direct sum, and the last contraction is fused with the discrete curl so the edge
// potential is never stored. All arithmetic is double; the faces are written in the storage
// type. The transpose runs the same steps backwards: curl^T gathered per edge, then projection
// onto the 1-D sine tables along x, y and z, each as a plain serial sum per output (fixed
// order, deterministic).
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

// tab[((axis * 2 + pos) * M + m) * nmax + i] = sin(2 pi (m+1) (i + pos/2) / n_axis + phase)
__global__ void sine_table_kernel(VelGeom g, const double* __restrict__ phases, double* __restrict__ tab)
{
    const int total = 6 * g.M * g.nmax;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int i = e % g.nmax;
        const int m = (e / g.nmax) % g.M;
        const int pos = (e / (g.nmax * g.M)) % 2;
        const int axis = e / (g.nmax * g.M * 2);
        const int n = g.n[axis];
        if (i >= n) {
            tab[e] = 0.0;
            continue;
        }
        const double off = pos ? 0.5 : 0.0;
        tab[e] = sin(2.0 * M_PI * (double)(m + 1) * ((double)i + off) / (double)n +
                     phases[axis * g.M + m]);
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

// A_c at edge (i, j, k) = sum_m3 T2[c][m3][j][i] Z_c(m3, k);  Z_c on the mid-points for c = 2
__device__ __forceinline__ double edge_pot(const VelGeom& g, const double* T2, const double* tab,
                                           int c, int i, int j, int k)
{
    const int M = g.M, nx = g.n[0], ny = g.n[1];
    const double* t2 = T2 + (size_t)c * M * ny * nx + (size_t)j * nx + i;
    const double* z = table(g, tab, 2, c == 2, 0) + k;
    double s = 0.0;
    for (int m3 = 0; m3 < M; ++m3) s = fma(t2[(size_t)m3 * ny * nx], z[(size_t)m3 * g.nmax], s);
    return s;
}

template <typename T>
__global__ void curl_kernel(VelGeom g, const double* __restrict__ T2, const double* __restrict__ tab,
                            T* __restrict__ U, T* __restrict__ V, T* __restrict__ W)
{
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const size_t total = (size_t)nx * ny * nz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % nx);
        const int j = (int)((e / nx) % ny);
        const int k = (int)(e / ((size_t)nx * ny));
        const int ip = wrap1(i + 1, nx), jp = wrap1(j + 1, ny), kp = wrap1(k + 1, nz);
        const double ax = edge_pot(g, T2, tab, 0, i, j, k);
        const double ay = edge_pot(g, T2, tab, 1, i, j, k);
        const double az = edge_pot(g, T2, tab, 2, i, j, k);
        const double az_jp = edge_pot(g, T2, tab, 2, i, jp, k);
        const double ay_kp = edge_pot(g, T2, tab, 1, i, j, kp);
        const double ax_kp = edge_pot(g, T2, tab, 0, i, j, kp);
        const double az_ip = edge_pot(g, T2, tab, 2, ip, j, k);
        const double ay_ip = edge_pot(g, T2, tab, 1, ip, j, k);
        const double ax_jp = edge_pot(g, T2, tab, 0, i, jp, k);
        U[e] = (T)((((az_jp - az) - ay_kp) + ay) / g.dx);
        V[e] = (T)((((ax_kp - ax) - az_ip) + az) / g.dx);
        W[e] = (T)((((ay_ip - ay) - ax_jp) + ax) / g.dx);
    }
}

// ------------------------------------------------------------------ transpose
// Edge cotangent Abar = curl^T (Ubar, Vbar, Wbar), gathered per edge (c, i, j, k).
template <typename T>
__global__ void curl_T_kernel(VelGeom g, const T* __restrict__ gU, const T* __restrict__ gV,
                              const T* __restrict__ gW, double* __restrict__ Ab)
{
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const size_t N = (size_t)nx * ny * nz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % nx);
        const int j = (int)((e / nx) % ny);
        const int k = (int)(e / ((size_t)nx * ny));
        auto at = [&](int ii, int jj, int kk) -> size_t {
            return ((size_t)wrap1(kk, nz) * ny + wrap1(jj, ny)) * nx + wrap1(ii, nx);
        };
        const double inv = 1.0 / g.dx;
        // Ax(k) enters V(k-1) with +1 and V(k) with -1; W(j-1) with -1 and W(j) with +1
        Ab[e] = (((double)gV[at(i, j, k - 1)] - (double)gV[e]) - (double)gW[at(i, j - 1, k)] +
                 (double)gW[e]) * inv;
        // Ay(k) enters U(k-1) with -1 and U(k) with +1; W(i-1) with +1 and W(i) with -1
        Ab[N + e] = ((-(double)gU[at(i, j, k - 1)] + (double)gU[e]) + (double)gW[at(i - 1, j, k)] -
                     (double)gW[e]) * inv;
        // Az(j) enters U(j-1) with +1 and U(j) with -1; V(i-1) with -1 and V(i) with +1
        Ab[2 * N + e] = (((double)gU[at(i, j - 1, k)] - (double)gU[e]) - (double)gV[at(i - 1, j, k)] +
                         (double)gV[e]) * inv;
    }
}

// P1[c][k][j][m1] = sum_i X_c(m1, i) Abar_c[k][j][i]
__global__ void project_x_kernel(VelGeom g, const double* __restrict__ Ab,
                                 const double* __restrict__ tab, double* __restrict__ P1)
{
    const int M = g.M, nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const size_t total = (size_t)3 * nz * ny * M;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int m1 = (int)(e % M);
        const size_t row = e / M;  // (c, k, j)
        const int c = (int)(row / ((size_t)nz * ny));
        const double* x = table(g, tab, 0, c == 0, m1);
        const double* ab = Ab + row * nx;
        double s = 0.0;
        for (int i = 0; i < nx; ++i) s = fma(x[i], ab[i], s);
        P1[e] = s;
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
    const size_t N = (size_t)nx * ny * nz;
    const size_t grad = 3 * N + (size_t)3 * nz * ny * M + (size_t)3 * nz * M * M;
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
    hipLaunchKernelGGL(curl_kernel<T>, dim3(blocks_for((size_t)nx * ny * nz)), dim3(256), 0, st, g,
                       T2, tab, U, V, W);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_velocity_grad(int nx, int ny, int nz, double dx, int M, const double* phases,
                                const T* gU, const T* gV, const T* gW, double* coeff_grad,
                                double* scratch, hipStream_t st)
{
    const VelGeom g = geom(nx, ny, nz, dx, M);
    const size_t N = (size_t)nx * ny * nz;
    double* tab = scratch;
    double* Ab = tab + table_doubles(g);
    double* P1 = Ab + 3 * N;
    double* P2 = P1 + (size_t)3 * nz * ny * M;
    hipLaunchKernelGGL(sine_table_kernel, dim3(blocks_for(table_doubles(g))), dim3(256), 0, st, g,
                       phases, tab);
    hipLaunchKernelGGL(curl_T_kernel<T>, dim3(blocks_for(N)), dim3(256), 0, st, g, gU, gV, gW, Ab);
    hipLaunchKernelGGL(project_x_kernel, dim3(blocks_for((size_t)3 * nz * ny * M)), dim3(256), 0,
                       st, g, Ab, tab, P1);
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
