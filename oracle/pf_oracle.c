/*
 * Oracle for the conservative, bounded phase-field step — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, deliberately slow FP64 statement of what the GPU library computes. Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load it; the product
 * path never does. It shares no source, header, table or helper with the HIP library.
 *
 * Paper: Mirjalili, Ivey & Mani, "A conservative diffuse interface method for two-phase flows
 * with provable boundedness properties" (arXiv:1803.01262).
 *
 * Model (Sec. 1, Eq. 1):  d(phi)/dt + div(u phi) = div[ gamma ( eps grad(phi)
 *                                                    - phi (1-phi) grad(phi)/|grad(phi)| ) ].
 * Discretisation (Sec. 2.2, the five-step recipe): phi at cell centres, velocity on faces;
 * unit normal and the sharpening product phi(1-phi)n at centres, interpolated (arithmetic mean)
 * to faces; diffusive flux from the two cells sharing the face; advective flux from the
 * face-interpolated phi; the update is the divergence of the face fluxes. All derivatives are
 * second-order central differences on a uniform isotropic mesh.
 *
 * Layout: arrays are [nz][ny][nx] (x fastest), periodic in every axis. U[k][j][i] is the
 * x-velocity on the LEFT x-face of cell (i,j,k) (x = i*dx); V and W likewise on the low y- and
 * z-faces. Face flux F_a[c] lives on the low a-face of cell c, between c-e_a and c.
 *
 * Readings of the paper where it is silent or garbled (each is also stated in the design notes):
 *  - n = g/|g| with g the 2dx central gradient at the centre; n = 0 where |g| = 0 (sgn(0) = 0).
 *    With delta > 0 the regularised n = g/sqrt(|g|^2 + delta^2) is used everywhere.
 *  - The i-1 sharpening term of Eq. 11/12 carries (phi^2 - phi), as Eq. 13 and Eq. 21 require.
 *  - Velocity with a time factor: u(x,t) = u0(x) s(t), s = 1 (steady) or cos(pi t / T);
 *    classic RK4 evaluates s at t, t+dt/2, t+dt/2, t+dt; the explicit midpoint RK2 at t, t+dt/2;
 *    the RK3 at t, t+8dt/15, t+2dt/3.
 *  - RK3 (the paper names Wray's low-storage third-order scheme and its limit, Eq. 27, but not its
 *    coefficients): u1 = u0 + dt g1 k1, u2 = u1 + dt (g2 k2 + z2 k1), u3 = u2 + dt (g3 k3 + z3 k2)
 *    with g = (8/15, 5/12, 3/4), z2 = -17/60, z3 = -5/12, k_s = f(u_{s-1}). Third order; its
 *    stability polynomial 1 + z + z^2/2 + z^3/6 reaches -2.51 on the real axis, Eq. 27's factor.
 *  - FP32-storage mode: every RK stage input and the new phi are rounded to float32 at the
 *    points where a value must be materialised; arithmetic stays FP64.
 *  - Walls (the paper names slip walls for its 2D random-field test but gives no discrete
 *    form): an axis flagged as walled has solid walls at x_a = 0 and x_a = n dx. The total flux
 *    through a wall face is zero (no normal velocity, no diffusive or sharpening flux), and the
 *    central gradient of a cell next to a wall takes the wall-side value from a mirror ghost
 *    (ghost of cell 0 = cell 0, of cell n-1 = cell n-1). The velocity stored on a wall face is
 *    ignored. The adjoint transposes exactly this: a wall face contributes nothing, and the
 *    gradient's read of a mirror ghost scatters back into the cell itself.
 *  - Non-uniform rectilinear meshes (the closing remarks say the method extends to non-uniform
 *    anisotropic Cartesian grids, with eps either fixed by the worst case or tuned to the local
 *    mesh, and give no discrete form; orc_rhs_nu and the functions after it): cell widths
 *    h_a[idx] per axis; the width index wraps on a periodic axis and mirrors across walls. The
 *    centre distance across the low a-face of cell idx is d_a(idx) = (h_a(idx-1) + h_a(idx))/2;
 *    the central gradient divides the difference of the two neighbours by the distance between
 *    their centres, d_a(idx) + d_a(idx+1); the diffusive flux uses the centre distance of its
 *    face; the face value of phi and of the sharpening product stays the mean of the two cells;
 *    the divergence divides by the cell's own width. eps is either the given value everywhere
 *    (mode 0) or, per cell, eps * max(h_x, h_y, h_z) / dx (mode 1, dx the reference spacing the
 *    given eps belongs to; the maximum over the axes longer than one cell), averaged onto each
 *    face. Mass is sum(phi * cell volume), the volume over the axes longer than one cell.
 */
#define _GNU_SOURCE
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t nx, ny, nz;
    double dx, eps, gamma, delta;
    int32_t wall[3]; /* per axis (x, y, z): 0 periodic, 1 walls at both ends */
} orc_grid;

static inline int64_t wrap(int64_t i, int64_t n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

/* linear index of cell (i,j,k) with periodic wrap */
static inline int64_t at(const orc_grid *g, int64_t i, int64_t j, int64_t k)
{
    return (wrap(k, g->nz) * g->ny + wrap(j, g->ny)) * g->nx + wrap(i, g->nx);
}

static inline int64_t ncell(const orc_grid *g) { return g->nx * g->ny * g->nz; }

/* offset of neighbour c + d*e_a */
static inline int64_t nb(const orc_grid *g, int64_t i, int64_t j, int64_t k, int a, int d)
{
    return at(g, i + (a == 0 ? d : 0), j + (a == 1 ? d : 0), k + (a == 2 ? d : 0));
}

static inline double round_storage(double v, int fp32) { return fp32 ? (double)(float)v : v; }

/* offset of neighbour c + d*e_a (|d| = 1) for the central gradient: across a wall, the mirror
 * ghost, i.e. the cell itself */
static inline int64_t nb_grad(const orc_grid *g, int64_t i, int64_t j, int64_t k, int a, int d)
{
    const int64_t n = a == 0 ? g->nx : (a == 1 ? g->ny : g->nz);
    const int64_t idx = (a == 0 ? i : (a == 1 ? j : k)) + d;
    if (g->wall[a] && (idx < 0 || idx >= n)) return at(g, i, j, k);
    return nb(g, i, j, k, a, d);
}

/* whether the low a-face of cell (i,j,k) is a wall face */
static inline int low_face_is_wall(const orc_grid *g, int64_t i, int64_t j, int64_t k, int a)
{
    return g->wall[a] && (a == 0 ? i : (a == 1 ? j : k)) == 0;
}

/* Threads of the OpenMP loops (for timing the oracle on a stated number of cores). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* Steps 1-3 of the recipe: central gradient, unit normal and sharpening product at centres.
 * Fills gr[3N] (gradient), nrm[3N] (normal), q[3N] = phi(1-phi) n. */
static void centre_fields(const orc_grid *g, const double *phi, double *gr, double *nrm,
                          double *q)
{
    const int64_t N = ncell(g);
    (void)N;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                double gv[3], mag2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    gv[a] = (phi[nb_grad(g, i, j, k, a, +1)] - phi[nb_grad(g, i, j, k, a, -1)]) /
                            (2.0 * g->dx);
                    mag2 += gv[a] * gv[a];
                }
                const double mag = sqrt(mag2 + g->delta * g->delta);
                const double p = phi[c];
                for (int a = 0; a < 3; ++a) {
                    const double n = mag > 0.0 ? gv[a] / mag : 0.0;
                    gr[3 * c + a] = gv[a];
                    nrm[3 * c + a] = n;
                    q[3 * c + a] = p * (1.0 - p) * n;
                }
            }
}

/* Right-hand side f = d(phi)/dt of the semi-discrete Eq. 1 (steps 1-5 of the recipe).
 * s multiplies the face velocities. */
void orc_rhs(const orc_grid *g, double s, const double *phi, const double *U, const double *V,
             const double *W, double *f)
{
    const int64_t N = ncell(g);
    double *gr = malloc(sizeof(double) * 3 * N);
    double *nrm = malloc(sizeof(double) * 3 * N);
    double *q = malloc(sizeof(double) * 3 * N);
    double *F = malloc(sizeof(double) * 3 * N);
    const double *vel[3] = {U, V, W};
    centre_fields(g, phi, gr, nrm, q);

    /* step 4: fluxes on the low face of every cell, F = -u phi_f + gamma eps dphi/dx - gamma q_f */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                for (int a = 0; a < 3; ++a) {
                    if (low_face_is_wall(g, i, j, k, a)) {
                        F[3 * c + a] = 0.0; /* no flux through a wall */
                        continue;
                    }
                    const int64_t m = nb(g, i, j, k, a, -1);
                    const double adv = -s * vel[a][c] * 0.5 * (phi[m] + phi[c]);
                    const double dif = g->gamma * g->eps * (phi[c] - phi[m]) / g->dx;
                    const double shp = -g->gamma * 0.5 * (q[3 * m + a] + q[3 * c + a]);
                    F[3 * c + a] = adv + dif + shp;
                }
            }

    /* step 5: divergence of the face fluxes (with walls, the high face of the last cell is the
     * wall face stored at index 0, whose flux is zero) */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                double acc = 0.0;
                for (int a = 0; a < 3; ++a)
                    acc += (F[3 * nb(g, i, j, k, a, +1) + a] - F[3 * c + a]) / g->dx;
                f[c] = acc;
            }
    free(gr);
    free(nrm);
    free(q);
    free(F);
}

static double time_factor(int vel_mode, double vel_T, double t)
{
    return vel_mode == 1 ? cos(M_PI * t / vel_T) : 1.0;
}

/* nsteps explicit steps of Eq. 1 in place on phi (Sec. 2.3).
 * scheme 1: forward Euler (Eq. 25 regime); scheme 2: the explicit midpoint rule (RK2, Eq. 26
 * regime); scheme 3: the low-storage RK3 above (Eq. 27 regime); scheme 4: classic RK4 (Eq. 28,
 * used for every experiment of Sec. 3). Step n starts at t0 + n*dt. */
typedef struct orc_mesh orc_mesh;
static void rhs_any(const orc_grid *g, const orc_mesh *m, double s, const double *phi,
                    const double *U, const double *V, const double *W, double *f);

static void step_impl(const orc_grid *g, const orc_mesh *mesh, int scheme, int fp32, double dt,
                      double t0, int vel_mode, double vel_T, int64_t nsteps, double *phi,
                      const double *U, const double *V, const double *W)
{
    const int64_t N = ncell(g);
    double *k1 = malloc(sizeof(double) * N), *k2 = malloc(sizeof(double) * N);
    double *k3 = malloc(sizeof(double) * N), *k4 = malloc(sizeof(double) * N);
    double *y = malloc(sizeof(double) * N);
    for (int64_t n = 0; n < nsteps; ++n) {
        const double t = t0 + (double)n * dt;
        if (scheme == 1) {
            rhs_any(g, mesh, time_factor(vel_mode, vel_T, t), phi, U, V, W, k1);
            for (int64_t c = 0; c < N; ++c) phi[c] = round_storage(phi[c] + dt * k1[c], fp32);
            continue;
        }
        if (scheme == 3) {
            const double g1 = 8.0 / 15.0, g2 = 5.0 / 12.0, g3 = 0.75, z2 = -17.0 / 60.0,
                         z3 = -5.0 / 12.0;
            double *u2 = k4;
            rhs_any(g, mesh, time_factor(vel_mode, vel_T, t), phi, U, V, W, k1);
            for (int64_t c = 0; c < N; ++c) y[c] = round_storage(phi[c] + dt * g1 * k1[c], fp32);
            rhs_any(g, mesh, time_factor(vel_mode, vel_T, t + g1 * dt), y, U, V, W, k2);
            for (int64_t c = 0; c < N; ++c)
                u2[c] = round_storage(y[c] + dt * (g2 * k2[c] + z2 * k1[c]), fp32);
            rhs_any(g, mesh, time_factor(vel_mode, vel_T, t + (g1 + g2 + z2) * dt), u2, U, V, W, k3);
            for (int64_t c = 0; c < N; ++c)
                phi[c] = round_storage(u2[c] + dt * (g3 * k3[c] + z3 * k2[c]), fp32);
            continue;
        }
        if (scheme == 2) {
            /* half an Euler step to the midpoint, then the whole step with the midpoint slope */
            rhs_any(g, mesh, time_factor(vel_mode, vel_T, t), phi, U, V, W, k1);
            for (int64_t c = 0; c < N; ++c) y[c] = round_storage(phi[c] + 0.5 * dt * k1[c], fp32);
            rhs_any(g, mesh, time_factor(vel_mode, vel_T, t + 0.5 * dt), y, U, V, W, k2);
            for (int64_t c = 0; c < N; ++c) phi[c] = round_storage(phi[c] + dt * k2[c], fp32);
            continue;
        }
        rhs_any(g, mesh, time_factor(vel_mode, vel_T, t), phi, U, V, W, k1);
        for (int64_t c = 0; c < N; ++c) y[c] = round_storage(phi[c] + 0.5 * dt * k1[c], fp32);
        rhs_any(g, mesh, time_factor(vel_mode, vel_T, t + 0.5 * dt), y, U, V, W, k2);
        for (int64_t c = 0; c < N; ++c) y[c] = round_storage(phi[c] + 0.5 * dt * k2[c], fp32);
        rhs_any(g, mesh, time_factor(vel_mode, vel_T, t + 0.5 * dt), y, U, V, W, k3);
        for (int64_t c = 0; c < N; ++c) y[c] = round_storage(phi[c] + dt * k3[c], fp32);
        rhs_any(g, mesh, time_factor(vel_mode, vel_T, t + dt), y, U, V, W, k4);
        for (int64_t c = 0; c < N; ++c)
            phi[c] = round_storage(
                phi[c] + dt / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]), fp32);
    }
    free(k1);
    free(k2);
    free(k3);
    free(k4);
    free(y);
}

void orc_step(const orc_grid *g, int scheme, int fp32, double dt, double t0, int vel_mode,
              double vel_T, int64_t nsteps, double *phi, const double *U, const double *V,
              const double *W)
{
    step_impl(g, NULL, scheme, fp32, dt, t0, vel_mode, vel_T, nsteps, phi, U, V, W);
}

/* One forward-Euler step written in the printed 1D coefficient form (Sec. 2.2.1, Eq. 13):
 * phi_i' = C_{i-1} phi_{i-1} + C_i phi_i + C_{i+1} phi_{i+1}, with A = dt gamma eps / dx^2,
 * B = dx / (2 eps), n_i = sgn(phi_{i+1} - phi_{i-1}) and a uniform velocity u. */
void orc_euler_coeff_1d(int64_t nx, double dx, double eps, double gamma, double u, double dt,
                        const double *phi, double *out)
{
    const double A = dt * gamma * eps / (dx * dx);
    const double B = dx / (2.0 * eps);
    for (int64_t i = 0; i < nx; ++i) {
        const int64_t im = wrap(i - 1, nx), ip = wrap(i + 1, nx);
        const int64_t imm = wrap(i - 2, nx), ipp = wrap(i + 2, nx);
        const double dm = phi[i] - phi[imm];  /* sign of the central difference at i-1 */
        const double dp = phi[ipp] - phi[i];  /* ... and at i+1 */
        const double nm = (dm > 0) - (dm < 0);
        const double np = (dp > 0) - (dp < 0);
        const double Cm = A * (1.0 + B * (nm * (1.0 - phi[im]) + u / gamma));
        const double Cc = 1.0 - 2.0 * A;
        const double Cp = A * (1.0 + B * (-np * (1.0 - phi[ip]) - u / gamma));
        out[i] = Cm * phi[im] + Cc * phi[i] + Cp * phi[ip];
    }
}

/* One forward-Euler step in the multi-dimensional coefficient form of Sec. 2.2.2
 * (Eqs. 18, 19, 21, 22), extended to three axes by symmetry:
 *   C_c      = 1 - 6A - (B A / gamma) s * (discrete divergence of the face velocity, times dx)
 *   C_{c-ea} = A [1 + B ( n_a(c-ea) (1 - phi(c-ea)) + s U_a(c)    / gamma)]
 *   C_{c+ea} = A [1 + B (-n_a(c+ea) (1 - phi(c+ea)) - s U_a(c+ea) / gamma)]
 * where n is the centre normal of the flux form. Degenerate axes (n_a = 1) contribute zero. */
void orc_euler_coeff(const orc_grid *g, double s, double dt, const double *phi, const double *U,
                     const double *V, const double *W, double *out)
{
    const int64_t N = ncell(g);
    double *gr = malloc(sizeof(double) * 3 * N);
    double *nrm = malloc(sizeof(double) * 3 * N);
    double *q = malloc(sizeof(double) * 3 * N);
    const double *vel[3] = {U, V, W};
    centre_fields(g, phi, gr, nrm, q);
    const double A = dt * g->gamma * g->eps / (g->dx * g->dx);
    const double B = g->dx / (2.0 * g->eps);
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                double div = 0.0;
                for (int a = 0; a < 3; ++a)
                    div += vel[a][nb(g, i, j, k, a, +1)] - vel[a][c];
                double v = (1.0 - 6.0 * A - B * A / g->gamma * s * div) * phi[c];
                for (int a = 0; a < 3; ++a) {
                    const int64_t m = nb(g, i, j, k, a, -1), p = nb(g, i, j, k, a, +1);
                    const double Cm =
                        A * (1.0 + B * (nrm[3 * m + a] * (1.0 - phi[m]) + s * vel[a][c] / g->gamma));
                    const double Cp =
                        A * (1.0 + B * (-nrm[3 * p + a] * (1.0 - phi[p]) - s * vel[a][p] / g->gamma));
                    v += Cm * phi[m] + Cp * phi[p];
                }
                out[c] = v;
            }
    free(gr);
    free(nrm);
    free(q);
}

/* Mass, extrema and non-finite count of a field: out4 = {sum(phi)*dV, min, max, #nonfinite}.
 * dV = dx^D with D the number of axes longer than one cell (Sec. 2.2.2 uses a D_f-dimensional
 * uniform mesh). Non-finite cells are excluded from the sum and the extrema. */
void orc_reduce(const orc_grid *g, const double *phi, double *out4)
{
    const int64_t N = ncell(g);
    int D = (g->nx > 1) + (g->ny > 1) + (g->nz > 1);
    if (D == 0) D = 1;
    double dV = 1.0;
    for (int d = 0; d < D; ++d) dV *= g->dx;
    double sum = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
    for (int64_t c = 0; c < N; ++c) {
        const double v = phi[c];
        if (!isfinite(v)) {
            bad += 1.0;
            continue;
        }
        sum += v;
        if (v < mn) mn = v;
        if (v > mx) mx = v;
    }
    out4[0] = sum * dV;
    out4[1] = mn;
    out4[2] = mx;
    out4[3] = bad;
}

/* ---------------------------------------------------------------------------------------
 * Non-uniform rectilinear meshes (the reading in the header): the recipe's five steps with
 * per-axis cell widths.
 * ------------------------------------------------------------------------------------- */
struct orc_mesh {
    const double *h[3]; /* cell widths along x, y, z: h[0][nx], h[1][ny], h[2][nz] */
    int32_t eps_mode;   /* 0: eps everywhere; 1: eps * max(h_x, h_y, h_z) / dx per cell */
};

/* width of cell idx along axis a (index wrapped on a periodic axis, mirrored across walls) */
static double width(const orc_grid *g, const orc_mesh *m, int a, int64_t idx)
{
    const int64_t n = a == 0 ? g->nx : (a == 1 ? g->ny : g->nz);
    if (g->wall[a]) {
        const int64_t p = 2 * n;
        int64_t r = idx % p;
        if (r < 0) r += p;
        idx = r < n ? r : p - 1 - r;
    } else {
        idx = wrap(idx, n);
    }
    return m->h[a][idx];
}

/* distance between the centres of cells idx-1 and idx along axis a */
static double centre_dist(const orc_grid *g, const orc_mesh *m, int a, int64_t idx)
{
    return 0.5 * (width(g, m, a, idx - 1) + width(g, m, a, idx));
}

/* interface thickness at cell (i, j, k) */
static double eps_cell(const orc_grid *g, const orc_mesh *m, int64_t i, int64_t j, int64_t k)
{
    if (m->eps_mode == 0) return g->eps;
    /* the largest width over the axes longer than one cell (a one-cell axis is not resolved) */
    const int64_t n[3] = {g->nx, g->ny, g->nz}, idx[3] = {i, j, k};
    double hmax = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double h = n[a] > 1 ? width(g, m, a, idx[a]) : 0.0;
        if (h > hmax) hmax = h;
    }
    return g->eps * hmax / g->dx;
}

static void rhs_nu(const orc_grid *g, const orc_mesh *m, double s, const double *phi,
                   const double *U, const double *V, const double *W, double *f)
{
    const int64_t N = ncell(g);
    double *q = malloc(sizeof(double) * 3 * N);
    double *F = malloc(sizeof(double) * 3 * N);
    const double *vel[3] = {U, V, W};
    /* steps 1-3: gradient over the distance between the two neighbours' centres, normal,
     * sharpening product */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                const int64_t idx[3] = {i, j, k};
                double gv[3], mag2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double span = centre_dist(g, m, a, idx[a]) + centre_dist(g, m, a, idx[a] + 1);
                    gv[a] = (phi[nb_grad(g, i, j, k, a, +1)] - phi[nb_grad(g, i, j, k, a, -1)]) / span;
                    mag2 += gv[a] * gv[a];
                }
                const double mag = sqrt(mag2 + g->delta * g->delta);
                const double p = phi[c];
                for (int a = 0; a < 3; ++a) q[3 * c + a] = p * (1.0 - p) * (mag > 0.0 ? gv[a] / mag : 0.0);
            }
    /* step 4: low-face fluxes */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                const int64_t idx[3] = {i, j, k};
                for (int a = 0; a < 3; ++a) {
                    if (low_face_is_wall(g, i, j, k, a)) {
                        F[3 * c + a] = 0.0;
                        continue;
                    }
                    const int64_t mc = nb(g, i, j, k, a, -1);
                    const double eps_f =
                        0.5 * (eps_cell(g, m, i - (a == 0), j - (a == 1), k - (a == 2)) +
                               eps_cell(g, m, i, j, k));
                    const double adv = -s * vel[a][c] * 0.5 * (phi[mc] + phi[c]);
                    const double dif = g->gamma * eps_f * (phi[c] - phi[mc]) / centre_dist(g, m, a, idx[a]);
                    const double shp = -g->gamma * 0.5 * (q[3 * mc + a] + q[3 * c + a]);
                    F[3 * c + a] = adv + dif + shp;
                }
            }
    /* step 5: divergence over the cell's widths */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                const int64_t idx[3] = {i, j, k};
                double acc = 0.0;
                for (int a = 0; a < 3; ++a)
                    acc += (F[3 * nb(g, i, j, k, a, +1) + a] - F[3 * c + a]) / width(g, m, a, idx[a]);
                f[c] = acc;
            }
    free(q);
    free(F);
}

static void rhs_any(const orc_grid *g, const orc_mesh *m, double s, const double *phi,
                    const double *U, const double *V, const double *W, double *f)
{
    if (m)
        rhs_nu(g, m, s, phi, U, V, W, f);
    else
        orc_rhs(g, s, phi, U, V, W, f);
}

/* f = d(phi)/dt on a non-uniform mesh: hx[nx], hy[ny], hz[nz] cell widths. */
void orc_rhs_nu(const orc_grid *g, const double *hx, const double *hy, const double *hz,
                int eps_mode, double s, const double *phi, const double *U, const double *V,
                const double *W, double *f)
{
    const orc_mesh m = {{hx, hy, hz}, eps_mode};
    rhs_nu(g, &m, s, phi, U, V, W, f);
}

/* orc_step on a non-uniform mesh */
void orc_step_nu(const orc_grid *g, const double *hx, const double *hy, const double *hz,
                 int eps_mode, int scheme, int fp32, double dt, double t0, int vel_mode,
                 double vel_T, int64_t nsteps, double *phi, const double *U, const double *V,
                 const double *W)
{
    const orc_mesh m = {{hx, hy, hz}, eps_mode};
    step_impl(g, &m, scheme, fp32, dt, t0, vel_mode, vel_T, nsteps, phi, U, V, W);
}

/* Mass on a non-uniform mesh: sum of phi times the cell volume (the product of the widths of
 * the axes longer than one cell); extrema and non-finite count as orc_reduce. */
void orc_reduce_nu(const orc_grid *g, const double *hx, const double *hy, const double *hz,
                   const double *phi, double *out4)
{
    const double *h[3] = {hx, hy, hz};
    const int64_t n[3] = {g->nx, g->ny, g->nz};
    double sum = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const double v = phi[at(g, i, j, k)];
                if (!isfinite(v)) {
                    bad += 1.0;
                    continue;
                }
                const int64_t idx[3] = {i, j, k};
                double vol = 1.0;
                for (int a = 0; a < 3; ++a)
                    if (n[a] > 1) vol *= h[a][idx[a]];
                sum += v * vol;
                if (v < mn) mn = v;
                if (v > mx) mx = v;
            }
    out4[0] = sum;
    out4[1] = mn;
    out4[2] = mx;
    out4[3] = bad;
}

/* ---------------------------------------------------------------------------------------
 * Discrete adjoint. The paper has no adjoint; what is computed here is the plain definition
 * of a vector-Jacobian product: the transpose of the derivative of the step above, obtained by
 * running the recipe's five steps backwards, each step scattered to the values it read.
 * ------------------------------------------------------------------------------------- */

/* phibar += (df/dphi)^T lam and Ubar/Vbar/Wbar += (df/dU)^T lam, for f = orc_rhs(phi, s).
 * Any of Ubar, Vbar, Wbar may be NULL. */
void orc_rhs_vjp(const orc_grid *g, double s, const double *phi, const double *U,
                 const double *V, const double *W, const double *lam, double *phibar,
                 double *Ubar, double *Vbar, double *Wbar)
{
    const int64_t N = ncell(g);
    double *gr = malloc(sizeof(double) * 3 * N);
    double *nrm = malloc(sizeof(double) * 3 * N);
    double *q = malloc(sizeof(double) * 3 * N);
    double *qbar = calloc(3 * N, sizeof(double));
    const double *vel[3] = {U, V, W};
    double *velbar[3] = {Ubar, Vbar, Wbar};
    centre_fields(g, phi, gr, nrm, q);

    /* reverse of steps 5 and 4 (serial scatter: obviously correct, no races) */
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                for (int a = 0; a < 3; ++a) {
                    /* a wall face carries the constant flux zero: nothing to transpose */
                    if (low_face_is_wall(g, i, j, k, a)) continue;
                    const int64_t m = nb(g, i, j, k, a, -1);
                    /* F_a[c] enters f[m] with +1/dx and f[c] with -1/dx */
                    const double Fbar = (lam[m] - lam[c]) / g->dx;
                    if (velbar[a]) velbar[a][c] += -s * 0.5 * (phi[m] + phi[c]) * Fbar;
                    phibar[c] += Fbar * (-s * vel[a][c] * 0.5 + g->gamma * g->eps / g->dx);
                    phibar[m] += Fbar * (-s * vel[a][c] * 0.5 - g->gamma * g->eps / g->dx);
                    qbar[3 * c + a] += -g->gamma * 0.5 * Fbar;
                    qbar[3 * m + a] += -g->gamma * 0.5 * Fbar;
                }
            }
    /* reverse of steps 3, 2 and 1 */
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                const double p = phi[c];
                double nbar[3], wbar = 0.0, mag2 = 0.0, gn = 0.0;
                for (int a = 0; a < 3; ++a) {
                    /* q_a = w n_a with w = p (1 - p) */
                    wbar += nrm[3 * c + a] * qbar[3 * c + a];
                    nbar[a] = p * (1.0 - p) * qbar[3 * c + a];
                    mag2 += gr[3 * c + a] * gr[3 * c + a];
                    gn += gr[3 * c + a] * nbar[a];
                }
                phibar[c] += (1.0 - 2.0 * p) * wbar;
                const double mag = sqrt(mag2 + g->delta * g->delta);
                if (!(mag > 0.0)) continue; /* n = 0 there, with zero derivative */
                for (int a = 0; a < 3; ++a) {
                    /* n_a = g_a / mag:  d n_a / d g_b = delta_ab / mag - g_a g_b / mag^3 */
                    const double gbar = nbar[a] / mag - gr[3 * c + a] * gn / (mag * mag * mag);
                    /* the gradient read the mirror ghost (the cell itself) across a wall */
                    phibar[nb_grad(g, i, j, k, a, +1)] += gbar / (2.0 * g->dx);
                    phibar[nb_grad(g, i, j, k, a, -1)] -= gbar / (2.0 * g->dx);
                }
            }
    free(gr);
    free(nrm);
    free(q);
    free(qbar);
}

/* The same vector-Jacobian product for rhs_nu (the non-uniform mesh m): rhs_nu's steps run
 * backwards with the mesh's coefficients, each scattered to the values it read. */
static void rhs_vjp_nu(const orc_grid *g, const orc_mesh *m, double s, const double *phi,
                       const double *U, const double *V, const double *W, const double *lam,
                       double *phibar, double *Ubar, double *Vbar, double *Wbar)
{
    const int64_t N = ncell(g);
    double *gr = malloc(sizeof(double) * 3 * N);
    double *qbar = calloc(3 * N, sizeof(double));
    const double *vel[3] = {U, V, W};
    double *velbar[3] = {Ubar, Vbar, Wbar};
    /* the forward's gradient (over the distance between the two neighbours' centres) */
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                const int64_t idx[3] = {i, j, k};
                for (int a = 0; a < 3; ++a) {
                    const double span = centre_dist(g, m, a, idx[a]) + centre_dist(g, m, a, idx[a] + 1);
                    gr[3 * c + a] =
                        (phi[nb_grad(g, i, j, k, a, +1)] - phi[nb_grad(g, i, j, k, a, -1)]) / span;
                }
            }
    /* reverse of steps 5 and 4 */
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                const int64_t idx[3] = {i, j, k};
                for (int a = 0; a < 3; ++a) {
                    if (low_face_is_wall(g, i, j, k, a)) continue;
                    const int64_t mc = nb(g, i, j, k, a, -1);
                    /* F_a[c] enters f[mc] with +1/h(mc) and f[c] with -1/h(c) */
                    const double Fbar = lam[mc] / width(g, m, a, idx[a] - 1) - lam[c] / width(g, m, a, idx[a]);
                    const double eps_f = 0.5 * (eps_cell(g, m, i - (a == 0), j - (a == 1), k - (a == 2)) +
                                                eps_cell(g, m, i, j, k));
                    const double dcoef = g->gamma * eps_f / centre_dist(g, m, a, idx[a]);
                    if (velbar[a]) velbar[a][c] += -s * 0.5 * (phi[mc] + phi[c]) * Fbar;
                    phibar[c] += Fbar * (-s * vel[a][c] * 0.5 + dcoef);
                    phibar[mc] += Fbar * (-s * vel[a][c] * 0.5 - dcoef);
                    qbar[3 * c + a] += -g->gamma * 0.5 * Fbar;
                    qbar[3 * mc + a] += -g->gamma * 0.5 * Fbar;
                }
            }
    /* reverse of steps 3, 2 and 1 */
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                const int64_t idx[3] = {i, j, k};
                const double p = phi[c];
                double mag2 = 0.0;
                for (int a = 0; a < 3; ++a) mag2 += gr[3 * c + a] * gr[3 * c + a];
                const double mag = sqrt(mag2 + g->delta * g->delta);
                double nbar[3], wbar = 0.0, gn = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double n_a = mag > 0.0 ? gr[3 * c + a] / mag : 0.0;
                    wbar += n_a * qbar[3 * c + a];
                    nbar[a] = p * (1.0 - p) * qbar[3 * c + a];
                    gn += gr[3 * c + a] * nbar[a];
                }
                phibar[c] += (1.0 - 2.0 * p) * wbar;
                if (!(mag > 0.0)) continue;
                for (int a = 0; a < 3; ++a) {
                    const double gbar = nbar[a] / mag - gr[3 * c + a] * gn / (mag * mag * mag);
                    const double span = centre_dist(g, m, a, idx[a]) + centre_dist(g, m, a, idx[a] + 1);
                    phibar[nb_grad(g, i, j, k, a, +1)] += gbar / span;
                    phibar[nb_grad(g, i, j, k, a, -1)] -= gbar / span;
                }
            }
    free(gr);
    free(qbar);
}

static void rhs_vjp_any(const orc_grid *g, const orc_mesh *m, double s, const double *phi,
                        const double *U, const double *V, const double *W, const double *lam,
                        double *phibar, double *Ubar, double *Vbar, double *Wbar)
{
    if (m)
        rhs_vjp_nu(g, m, s, phi, U, V, W, lam, phibar, Ubar, Vbar, Wbar);
    else
        orc_rhs_vjp(g, s, phi, U, V, W, lam, phibar, Ubar, Vbar, Wbar);
}

/* orc_rhs_vjp on a non-uniform mesh (widths and eps_mode as orc_rhs_nu) */
void orc_rhs_vjp_nu(const orc_grid *g, const double *hx, const double *hy, const double *hz,
                    int eps_mode, double s, const double *phi, const double *U, const double *V,
                    const double *W, const double *lam, double *phibar, double *Ubar,
                    double *Vbar, double *Wbar)
{
    const orc_mesh m = {{hx, hy, hz}, eps_mode};
    rhs_vjp_nu(g, &m, s, phi, U, V, W, lam, phibar, Ubar, Vbar, Wbar);
}

static void adjoint_impl(const orc_grid *g, const orc_mesh *mesh, int scheme, double dt,
                         double t, int vel_mode, double vel_T, const double *phi, const double *U,
                         const double *V, const double *W, double *lam, double *Ubar, double *Vbar,
                         double *Wbar);

/* Adjoint of one step of orc_step (FP64): on entry lam holds dL/dphi_{n+1}; on exit dL/dphi_n.
 * Ubar/Vbar/Wbar (may be NULL) accumulate dL/dU0 etc. for u = u0 s(t). */
void orc_adjoint_step(const orc_grid *g, int scheme, double dt, double t, int vel_mode,
                      double vel_T, const double *phi, const double *U, const double *V,
                      const double *W, double *lam, double *Ubar, double *Vbar, double *Wbar)
{
    adjoint_impl(g, NULL, scheme, dt, t, vel_mode, vel_T, phi, U, V, W, lam, Ubar, Vbar, Wbar);
}

/* orc_adjoint_step on a non-uniform mesh (widths and eps_mode as orc_rhs_nu) */
void orc_adjoint_step_nu(const orc_grid *g, const double *hx, const double *hy, const double *hz,
                         int eps_mode, int scheme, double dt, double t, int vel_mode,
                         double vel_T, const double *phi, const double *U, const double *V,
                         const double *W, double *lam, double *Ubar, double *Vbar, double *Wbar)
{
    const orc_mesh m = {{hx, hy, hz}, eps_mode};
    adjoint_impl(g, &m, scheme, dt, t, vel_mode, vel_T, phi, U, V, W, lam, Ubar, Vbar, Wbar);
}

static void adjoint_impl(const orc_grid *g, const orc_mesh *mesh, int scheme, double dt,
                         double t, int vel_mode, double vel_T, const double *phi, const double *U,
                         const double *V, const double *W, double *lam, double *Ubar, double *Vbar,
                         double *Wbar)
{
    const int64_t N = ncell(g);
    double *kb = malloc(sizeof(double) * N);
    double *yb = calloc(N, sizeof(double));
    double *out = malloc(sizeof(double) * N);
    if (scheme == 1) {
        for (int64_t c = 0; c < N; ++c) kb[c] = dt * lam[c];
        rhs_vjp_any(g, mesh, time_factor(vel_mode, vel_T, t), phi, U, V, W, kb, yb, Ubar, Vbar,
                    Wbar);
        for (int64_t c = 0; c < N; ++c) lam[c] += yb[c];
        free(kb);
        free(yb);
        free(out);
        return;
    }
    /* Explicit Runge-Kutta in Butcher form: y_s = phi + dt sum_{j<s} a[s][j] k_j,
     * phi' = phi + dt sum_s b[s] k_s, k_s = f(y_s, t + c[s] dt). Reverse: with
     * kbar_s = dt (b[s] lam' + sum_{i>s} a[i][s] ybar_i) and ybar_s = (df/dy at y_s)^T kbar_s,
     * phibar = lam' + sum_s ybar_s.
     *   RK2 (explicit midpoint): a21 = 1/2; b = (0, 1); c = (0, 1/2).
     *   RK3 (low storage, see the header): a21 = 8/15, a31 = 1/4, a32 = 5/12; b = (1/4, 0, 3/4);
     *                                      c = (0, 8/15, 2/3).
     *   RK4 (classic): a21 = a32 = 1/2, a43 = 1; b = (1/6, 1/3, 1/3, 1/6); c = (0, 1/2, 1/2, 1). */
    double a[4][4] = {{0}}, b[4] = {0}, cs[4] = {0};
    int ns;
    if (scheme == 2) {
        ns = 2;
        a[1][0] = 0.5;
        b[1] = 1.0;
        cs[1] = 0.5;
    } else if (scheme == 3) {
        ns = 3;
        a[1][0] = 8.0 / 15.0;
        a[2][0] = 0.25;
        a[2][1] = 5.0 / 12.0;
        b[0] = 0.25;
        b[2] = 0.75;
        cs[1] = 8.0 / 15.0;
        cs[2] = 2.0 / 3.0;
    } else {
        ns = 4;
        a[1][0] = a[2][1] = 0.5;
        a[3][2] = 1.0;
        b[0] = b[3] = 1.0 / 6.0;
        b[1] = b[2] = 1.0 / 3.0;
        cs[1] = cs[2] = 0.5;
        cs[3] = 1.0;
    }
    /* recompute the stage inputs and slopes of the forward step */
    double *y[4], *kk[4];
    for (int s = 0; s < ns; ++s) {
        y[s] = malloc(sizeof(double) * N);
        kk[s] = malloc(sizeof(double) * N);
    }
    for (int s = 0; s < ns; ++s) {
        for (int64_t c = 0; c < N; ++c) {
            double v = phi[c];
            for (int j = 0; j < s; ++j) v += dt * a[s][j] * kk[j][c];
            y[s][c] = v;
        }
        if (s < ns - 1) /* the last slope enters no stage input */
            rhs_any(g, mesh, time_factor(vel_mode, vel_T, t + cs[s] * dt), y[s], U, V, W, kk[s]);
    }
    /* reverse sweep over the stages, newest first */
    for (int64_t c = 0; c < N; ++c) out[c] = lam[c];
    double *ybar[4];
    for (int s = 0; s < ns; ++s) ybar[s] = calloc(N, sizeof(double));
    for (int s = ns - 1; s >= 0; --s) {
        for (int64_t c = 0; c < N; ++c) {
            double v = b[s] * lam[c];
            for (int i = s + 1; i < ns; ++i) v += a[i][s] * ybar[i][c];
            kb[c] = dt * v;
        }
        rhs_vjp_any(g, mesh, time_factor(vel_mode, vel_T, t + cs[s] * dt), y[s], U, V, W, kb,
                    ybar[s], Ubar, Vbar, Wbar);
    }
    /* every stage input is phi + (something), so phibar collects all the ybar */
    for (int64_t c = 0; c < N; ++c) {
        double sum = out[c];
        for (int s = 0; s < ns; ++s) sum += ybar[s][c];
        lam[c] = sum;
    }
    for (int s = 0; s < ns; ++s) {
        free(y[s]);
        free(ybar[s]);
        free(kk[s]);
    }
    free(kb);
    free(yb);
    free(out);
}

/* ---------------------------------------------------------------------------------------
 * Face velocity from a vector potential of separable Fourier modes, and its transpose.
 * The paper requires a discretely incompressible face velocity (the divergence term of
 * Eq. 19 must vanish); the discrete curl of an edge potential has zero discrete divergence
 * identically. Potential component a at its edge position x:
 *   A_a(x) = sum_{m1,m2,m3=1..M} c[m3-1][m2-1][m1-1][a]
 *            sin(2 pi m1 x/Lx + th[0][m1-1]) sin(2 pi m2 y/Ly + th[1][m2-1]) sin(2 pi m3 z/Lz + th[2][m3-1])
 * Edge positions (cell (i,j,k) spans [i dx,(i+1) dx] etc.):
 *   Ax at ((i+1/2) dx, j dx, k dx);  Ay at (i dx, (j+1/2) dx, k dx);  Az at (i dx, j dx, (k+1/2) dx).
 * Curl on the faces:
 *   U = (Az[j+1]-Az[j] - Ay[k+1]+Ay[k]) / dx,  V = (Ax[k+1]-Ax[k] - Az[i+1]+Az[i]) / dx,
 *   W = (Ay[i+1]-Ay[i] - Ax[j+1]+Ax[j]) / dx.
 * ------------------------------------------------------------------------------------- */

/* 1-D sine tables: tab[m*n + i] = sin(2 pi (m+1) (i + off)/n + th[m]) */
static double *sine_table(int64_t n, int M, const double *th, double off)
{
    double *tab = malloc(sizeof(double) * n * M);
    for (int m = 0; m < M; ++m)
        for (int64_t i = 0; i < n; ++i)
            tab[m * n + i] = sin(2.0 * M_PI * (double)(m + 1) * ((double)i + off) / (double)n + th[m]);
    return tab;
}

/* the three edge potentials, by direct summation over all M^3 modes */
static void edge_potential(const orc_grid *g, int M, const double *th, const double *coef,
                           double *A[3])
{
    double *node[3], *mid[3];
    const int64_t n[3] = {g->nx, g->ny, g->nz};
    for (int a = 0; a < 3; ++a) {
        node[a] = sine_table(n[a], M, th + a * M, 0.0);
        mid[a] = sine_table(n[a], M, th + a * M, 0.5);
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                for (int a = 0; a < 3; ++a) {
                    /* component a sits at the mid-point along axis a, nodes along the others */
                    const double *tx = a == 0 ? mid[0] : node[0];
                    const double *ty = a == 1 ? mid[1] : node[1];
                    const double *tz = a == 2 ? mid[2] : node[2];
                    double sum = 0.0;
                    for (int m3 = 0; m3 < M; ++m3)
                        for (int m2 = 0; m2 < M; ++m2)
                            for (int m1 = 0; m1 < M; ++m1)
                                sum += coef[(((int64_t)m3 * M + m2) * M + m1) * 3 + a] *
                                       tx[m1 * g->nx + i] * ty[m2 * g->ny + j] * tz[m3 * g->nz + k];
                    A[a][c] = sum;
                }
            }
    for (int a = 0; a < 3; ++a) {
        free(node[a]);
        free(mid[a]);
    }
}

void orc_velocity_from_coeffs(const orc_grid *g, int M, const double *th, const double *coef,
                              double *U, double *V, double *W)
{
    const int64_t N = ncell(g);
    double *A[3];
    for (int a = 0; a < 3; ++a) A[a] = malloc(sizeof(double) * N);
    edge_potential(g, M, th, coef, A);
    const double *Ax = A[0], *Ay = A[1], *Az = A[2];
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                U[c] = (Az[at(g, i, j + 1, k)] - Az[c] - Ay[at(g, i, j, k + 1)] + Ay[c]) / g->dx;
                V[c] = (Ax[at(g, i, j, k + 1)] - Ax[c] - Az[at(g, i + 1, j, k)] + Az[c]) / g->dx;
                W[c] = (Ay[at(g, i + 1, j, k)] - Ay[c] - Ax[at(g, i, j + 1, k)] + Ax[c]) / g->dx;
            }
    for (int a = 0; a < 3; ++a) free(A[a]);
}

/* coefbar += (d(U,V,W)/d coef)^T (Ubar,Vbar,Wbar): transpose of the curl (scatter form),
 * then projection of each edge cotangent onto the separable modes. */
void orc_velocity_from_coeffs_T(const orc_grid *g, int M, const double *th, const double *Ubar,
                                const double *Vbar, const double *Wbar, double *coefbar)
{
    const int64_t N = ncell(g);
    double *Ab[3];
    for (int a = 0; a < 3; ++a) Ab[a] = calloc(N, sizeof(double));
    double *Axb = Ab[0], *Ayb = Ab[1], *Azb = Ab[2];
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                const int64_t c = at(g, i, j, k);
                const double u = Ubar[c] / g->dx, v = Vbar[c] / g->dx, w = Wbar[c] / g->dx;
                Azb[at(g, i, j + 1, k)] += u;
                Azb[c] -= u;
                Ayb[at(g, i, j, k + 1)] -= u;
                Ayb[c] += u;
                Axb[at(g, i, j, k + 1)] += v;
                Axb[c] -= v;
                Azb[at(g, i + 1, j, k)] -= v;
                Azb[c] += v;
                Ayb[at(g, i + 1, j, k)] += w;
                Ayb[c] -= w;
                Axb[at(g, i, j + 1, k)] -= w;
                Axb[c] += w;
            }
    double *node[3], *mid[3];
    const int64_t n[3] = {g->nx, g->ny, g->nz};
    for (int a = 0; a < 3; ++a) {
        node[a] = sine_table(n[a], M, th + a * M, 0.0);
        mid[a] = sine_table(n[a], M, th + a * M, 0.5);
    }
    const int64_t nm = (int64_t)M * M * M;
#pragma omp parallel for schedule(static)
    for (int64_t mm = 0; mm < nm; ++mm) {
        const int m1 = (int)(mm % M), m2 = (int)((mm / M) % M), m3 = (int)(mm / ((int64_t)M * M));
        for (int a = 0; a < 3; ++a) {
            const double *tx = a == 0 ? mid[0] : node[0];
            const double *ty = a == 1 ? mid[1] : node[1];
            const double *tz = a == 2 ? mid[2] : node[2];
            double sum = 0.0;
            for (int64_t k = 0; k < g->nz; ++k)
                for (int64_t j = 0; j < g->ny; ++j)
                    for (int64_t i = 0; i < g->nx; ++i)
                        sum += Ab[a][at(g, i, j, k)] * tx[m1 * g->nx + i] * ty[m2 * g->ny + j] *
                               tz[m3 * g->nz + k];
            coefbar[mm * 3 + a] += sum;
        }
    }
    for (int a = 0; a < 3; ++a) {
        free(node[a]);
        free(mid[a]);
        free(Ab[a]);
    }
}
