/*
 * FP64 CPU oracle for the MAC-grid liquid step.  TEST INFRASTRUCTURE ONLY:
 * the product path never links, loads or calls this file.
 *
 * What it computes, with the passage each part follows (paper sections of
 * arXiv 2503.00868; the readings where the paper is silent are marked R#):
 *   - the incompressible momentum equation with gravity, viscosity and the
 *     pressure gradient (Section 3.2.2, Eq. (v)), split into sub-steps in the
 *     style of Chorin (Section 3.2.2);
 *   - semi-Lagrangian back-tracing for the convection term (Section 3.4.1,
 *     after Stam's stable fluids);
 *   - viscosity as nu * Laplacian per component (R5: the strain-rate form of
 *     Eq. (v) reduces to it for constant nu and divergence-free velocity);
 *   - the pressure Poisson equation over liquid cells, p = 0 in air (R7),
 *     no flux through solid walls (Section 3.2.2 "Poisson Pressure Equation");
 *   - MIC(0) as in the fluid-simulation text the paper points to for its
 *     solver details (Section 3.2.2, [bridson2015fluid]).
 * Conventions are in oracle.h.  Every function here is a plain loop in double
 * precision; parallel-for pragmas only split independent iterations.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- layout */

static void face_dims(int n, int comp, int d[3]) {
    d[0] = n + (comp == 0);
    d[1] = n + (comp == 1);
    d[2] = n + (comp == 2);
}

long orc_face_count(int n, int comp) {
    int d[3];
    face_dims(n, comp, d);
    return (long)d[0] * d[1] * d[2];
}

static long fidx(const int d[3], int i, int j, int k) {
    return i + (long)d[0] * (j + (long)d[1] * k);
}

static long cidx(int n, int i, int j, int k) { return i + (long)n * (j + (long)n * k); }

static int cell_type(int n, const uint8_t* cell, int i, int j, int k) {
    if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) return ORC_SOLID;
    return cell[cidx(n, i, j, k)];
}

/* The face (i,j,k) of component comp separates cell (i,j,k) - e_comp ("minus")
 * from cell (i,j,k) ("plus"). */
static int face_class(int n, const uint8_t* cell, int comp, int i, int j, int k) {
    int d[3];
    face_dims(n, comp, d);
    if (i < 0 || j < 0 || k < 0 || i >= d[0] || j >= d[1] || k >= d[2]) return ORC_WALL;
    int im = i - (comp == 0), jm = j - (comp == 1), km = k - (comp == 2);
    int a = cell_type(n, cell, im, jm, km);
    int b = cell_type(n, cell, i, j, k);
    if (a == ORC_SOLID || b == ORC_SOLID) return ORC_WALL;
    if (a == ORC_LIQUID || b == ORC_LIQUID) return ORC_ACTIVE;
    return ORC_INACTIVE;
}

void orc_face_classes(int n, const uint8_t* cell, int comp, uint8_t* out) {
    int d[3];
    face_dims(n, comp, d);
    for (int k = 0; k < d[2]; ++k)
        for (int j = 0; j < d[1]; ++j)
            for (int i = 0; i < d[0]; ++i)
                out[fidx(d, i, j, k)] = (uint8_t)face_class(n, cell, comp, i, j, k);
}

/* Every face that is not active holds zero (R2: walls are no-flux, air-air
 * faces carry no velocity; no extrapolation into air). */
void orc_mask_faces(int n, const uint8_t* cell, int comp, double* f) {
    int d[3];
    face_dims(n, comp, d);
    for (int k = 0; k < d[2]; ++k)
        for (int j = 0; j < d[1]; ++j)
            for (int i = 0; i < d[0]; ++i)
                if (face_class(n, cell, comp, i, j, k) != ORC_ACTIVE) f[fidx(d, i, j, k)] = 0.0;
}

/* ------------------------------------------------------------ sampling */

/* Trilinear interpolation on the node lattice of one velocity component.
 * The lattice of comp has nodes at integer grid units along its own axis and
 * at half units along the other two.  Each axis is clamped to the node range;
 * the lower node index is floor(t), capped so the upper node exists (R4). */
double orc_sample(int n, int comp, const double* f, const double g[3], double grad[3]) {
    int d[3];
    face_dims(n, comp, d);
    int i0[3];
    double fr[3];
    int clamped[3];
    for (int a = 0; a < 3; ++a) {
        double off = (a == comp) ? 0.0 : 0.5;
        double t = g[a] - off;
        double hi = (double)(d[a] - 1);
        clamped[a] = (t < 0.0 || t > hi);
        if (t < 0.0) t = 0.0;
        if (t > hi) t = hi;
        int b = (int)floor(t);
        if (b > d[a] - 2) b = d[a] - 2;
        i0[a] = b;
        fr[a] = t - b;
    }
    double c[2][2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                c[dz][dy][dx] = f[fidx(d, i0[0] + dx, i0[1] + dy, i0[2] + dz)];
    double wx[2] = {1.0 - fr[0], fr[0]};
    double wy[2] = {1.0 - fr[1], fr[1]};
    double wz[2] = {1.0 - fr[2], fr[2]};
    double val = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) val += wx[dx] * wy[dy] * wz[dz] * c[dz][dy][dx];
    if (grad) {
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy) gx += wy[dy] * wz[dz] * (c[dz][dy][1] - c[dz][dy][0]);
        for (int dz = 0; dz < 2; ++dz)
            for (int dx = 0; dx < 2; ++dx) gy += wx[dx] * wz[dz] * (c[dz][1][dx] - c[dz][0][dx]);
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) gz += wx[dx] * wy[dy] * (c[1][dy][dx] - c[0][dy][dx]);
        grad[0] = clamped[0] ? 0.0 : gx;
        grad[1] = clamped[1] ? 0.0 : gy;
        grad[2] = clamped[2] ? 0.0 : gz;
    }
    return val;
}

/* Scatter s * (trilinear weights at g) onto the nodes of comp (adjoint of
 * orc_sample's value with respect to the field). */
static void scatter_sample(int n, int comp, double* f, const double g[3], double s) {
    int d[3];
    face_dims(n, comp, d);
    int i0[3];
    double fr[3];
    for (int a = 0; a < 3; ++a) {
        double off = (a == comp) ? 0.0 : 0.5;
        double t = g[a] - off;
        double hi = (double)(d[a] - 1);
        if (t < 0.0) t = 0.0;
        if (t > hi) t = hi;
        int b = (int)floor(t);
        if (b > d[a] - 2) b = d[a] - 2;
        i0[a] = b;
        fr[a] = t - b;
    }
    double wx[2] = {1.0 - fr[0], fr[0]};
    double wy[2] = {1.0 - fr[1], fr[1]};
    double wz[2] = {1.0 - fr[2], fr[2]};
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                f[fidx(d, i0[0] + dx, i0[1] + dy, i0[2] + dz)] += s * wx[dx] * wy[dy] * wz[dz];
}

static const double* pick(int comp, const double* u, const double* v, const double* w) {
    return comp == 0 ? u : (comp == 1 ? v : w);
}

/* ----------------------------------------------------------- advection */

/* Semi-Lagrangian advection (Section 3.4.1, Stam's back-tracing): every
 * active face samples the velocity at its own position, steps back by dt
 * along it (one explicit Euler step, R3) and takes the trilinear sample of
 * its own component there.  Non-active faces get zero.  dt_over_h = dt / h. */
void orc_advect(int n, const uint8_t* cell, const double* u, const double* v, const double* w,
                double dt_over_h, double* au, double* av, double* aw) {
    for (int comp = 0; comp < 3; ++comp) {
        int d[3];
        face_dims(n, comp, d);
        const double* src = pick(comp, u, v, w);
        double* dst = comp == 0 ? au : (comp == 1 ? av : aw);
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < d[2]; ++k)
            for (int j = 0; j < d[1]; ++j)
                for (int i = 0; i < d[0]; ++i) {
                    long id = fidx(d, i, j, k);
                    if (face_class(n, cell, comp, i, j, k) != ORC_ACTIVE) {
                        dst[id] = 0.0;
                        continue;
                    }
                    double gf[3] = {i + (comp == 0 ? 0.0 : 0.5), j + (comp == 1 ? 0.0 : 0.5),
                                    k + (comp == 2 ? 0.0 : 0.5)};
                    double U[3];
                    for (int a = 0; a < 3; ++a) U[a] = orc_sample(n, a, pick(a, u, v, w), gf, NULL);
                    double gd[3];
                    for (int a = 0; a < 3; ++a) gd[a] = gf[a] - dt_over_h * U[a];
                    dst[id] = orc_sample(n, comp, src, gd, NULL);
                }
    }
}

/* Derivative of the advected value of every active face with respect to the
 * time step (the advection's own dependence on dt; the body force is
 * separate).  The departure point x_d = x_f - dt U(x_f) moves by -U(x_f) per
 * unit of dt, so d a_f / d dt = -grad I_c(x_d) . U(x_f).  In grid units
 * (X = x / h) the sample gradient is per cell and dX_d / d dt = -U / h.
 * Non-active faces get zero. */
void orc_advect_ddt(int n, const uint8_t* cell, const double* u, const double* v, const double* w,
                    double dt_over_h, double* du, double* dv, double* dw) {
    for (int comp = 0; comp < 3; ++comp) {
        int d[3];
        face_dims(n, comp, d);
        const double* src = pick(comp, u, v, w);
        double* dst = comp == 0 ? du : (comp == 1 ? dv : dw);
        for (int k = 0; k < d[2]; ++k)
            for (int j = 0; j < d[1]; ++j)
                for (int i = 0; i < d[0]; ++i) {
                    long id = fidx(d, i, j, k);
                    dst[id] = 0.0;
                    if (face_class(n, cell, comp, i, j, k) != ORC_ACTIVE) continue;
                    double gf[3] = {i + (comp == 0 ? 0.0 : 0.5), j + (comp == 1 ? 0.0 : 0.5),
                                    k + (comp == 2 ? 0.0 : 0.5)};
                    double U[3];
                    for (int a = 0; a < 3; ++a) U[a] = orc_sample(n, a, pick(a, u, v, w), gf, NULL);
                    double gd[3];
                    for (int a = 0; a < 3; ++a) gd[a] = gf[a] - dt_over_h * U[a];
                    double grad[3];
                    orc_sample(n, comp, src, gd, grad);
                    double s = 0.0;
                    for (int a = 0; a < 3; ++a) s -= grad[a] * U[a] * (double)n;
                    dst[id] = s;
                }
    }
}

/* Body force applied explicitly on active faces (Section 3.2.2). */
void orc_add_force(int n, const uint8_t* cell, double* u, double* v, double* w, double dt,
                   const double g[3]) {
    for (int comp = 0; comp < 3; ++comp) {
        int d[3];
        face_dims(n, comp, d);
        double* f = comp == 0 ? u : (comp == 1 ? v : w);
        for (int k = 0; k < d[2]; ++k)
            for (int j = 0; j < d[1]; ++j)
                for (int i = 0; i < d[0]; ++i)
                    if (face_class(n, cell, comp, i, j, k) == ORC_ACTIVE)
                        f[fidx(d, i, j, k)] += dt * g[comp];
    }
}

/* ----------------------------------------------------------- diffusion */

/* Componentwise 7-point Laplacian on active faces, scaled by 1/h^2 (R5, R6):
 *  - an active neighbour contributes (f_nbr - f);
 *  - along the component's own axis a wall neighbour is a Dirichlet zero and
 *    contributes (0 - f) (no flux through the wall);
 *  - a tangential neighbour that is a wall or lies outside the grid, and any
 *    inactive neighbour, is left out (free slip at walls, no traction at the
 *    liquid surface).
 * Non-active faces get zero. */
void orc_laplacian(int n, const uint8_t* cell, int comp, const double* f, double* out) {
    int d[3];
    face_dims(n, comp, d);
    double inv_h2 = (double)n * (double)n;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < d[2]; ++k)
        for (int j = 0; j < d[1]; ++j)
            for (int i = 0; i < d[0]; ++i) {
                long id = fidx(d, i, j, k);
                if (face_class(n, cell, comp, i, j, k) != ORC_ACTIVE) {
                    out[id] = 0.0;
                    continue;
                }
                double acc = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int s = -1; s <= 1; s += 2) {
                        int ii = i + (a == 0 ? s : 0), jj = j + (a == 1 ? s : 0),
                            kk = k + (a == 2 ? s : 0);
                        int cls = face_class(n, cell, comp, ii, jj, kk);
                        if (cls == ORC_ACTIVE)
                            acc += f[fidx(d, ii, jj, kk)] - f[id];
                        else if (cls == ORC_WALL && a == comp)
                            acc += -f[id];
                    }
                out[id] = acc * inv_h2;
            }
}

/* Explicit viscosity step: out = f + nu*dt*L f on active faces. */
void orc_diffuse_explicit(int n, const uint8_t* cell, int comp, double nu_dt, const double* f,
                          double* out) {
    long m = orc_face_count(n, comp);
    double* lf = (double*)malloc(sizeof(double) * m);
    orc_laplacian(n, cell, comp, f, lf);
    int d[3];
    face_dims(n, comp, d);
    for (int k = 0; k < d[2]; ++k)
        for (int j = 0; j < d[1]; ++j)
            for (int i = 0; i < d[0]; ++i) {
                long id = fidx(d, i, j, k);
                out[id] = face_class(n, cell, comp, i, j, k) == ORC_ACTIVE ? f[id] + nu_dt * lf[id]
                                                                           : 0.0;
            }
    free(lf);
}

static double dot(long m, const double* a, const double* b) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long q = 0; q < m; ++q) s += a[q] * b[q];
    return s;
}

/* Implicit viscosity step: solve (I - nu*dt*L) out = f on active faces by
 * plain conjugate gradients, to a relative residual tol. */
int orc_diffuse_implicit(int n, const uint8_t* cell, int comp, double nu_dt, const double* f,
                         double* out, double tol, int max_iter, double* relres) {
    long m = orc_face_count(n, comp);
    double* b = (double*)malloc(sizeof(double) * m);
    double* r = (double*)malloc(sizeof(double) * m);
    double* p = (double*)malloc(sizeof(double) * m);
    double* q = (double*)malloc(sizeof(double) * m);
    memcpy(b, f, sizeof(double) * m);
    orc_mask_faces(n, cell, comp, b);
    memset(out, 0, sizeof(double) * m);
    memcpy(r, b, sizeof(double) * m);
    memcpy(p, r, sizeof(double) * m);
    double bn = sqrt(dot(m, b, b));
    double rr = dot(m, r, r);
    int it = 0;
    if (bn == 0.0) {
        if (relres) *relres = 0.0;
        free(b); free(r); free(p); free(q);
        return 0;
    }
    while (sqrt(rr) / bn > tol && it < max_iter) {
        orc_laplacian(n, cell, comp, p, q);
        for (long t = 0; t < m; ++t) q[t] = p[t] - nu_dt * q[t];
        orc_mask_faces(n, cell, comp, q);
        double alpha = rr / dot(m, p, q);
        for (long t = 0; t < m; ++t) {
            out[t] += alpha * p[t];
            r[t] -= alpha * q[t];
        }
        double rr_new = dot(m, r, r);
        double beta = rr_new / rr;
        rr = rr_new;
        for (long t = 0; t < m; ++t) p[t] = r[t] + beta * p[t];
        ++it;
    }
    /* true residual */
    orc_laplacian(n, cell, comp, out, q);
    for (long t = 0; t < m; ++t) q[t] = b[t] - (out[t] - nu_dt * q[t]);
    orc_mask_faces(n, cell, comp, q);
    if (relres) *relres = sqrt(dot(m, q, q)) / bn;
    free(b); free(r); free(p); free(q);
    return it;
}

/* ---------------------------------------------------------- projection */

/* Diagonal of the Poisson matrix: for a liquid cell, the number of its six
 * faces that are not walls; zero for air and solid cells. */
void orc_poisson_diag(int n, const uint8_t* cell, double* diag) {
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long c = cidx(n, i, j, k);
                if (cell[c] != ORC_LIQUID) {
                    diag[c] = 0.0;
                    continue;
                }
                int cnt = 0;
                cnt += face_class(n, cell, 0, i, j, k) != ORC_WALL;
                cnt += face_class(n, cell, 0, i + 1, j, k) != ORC_WALL;
                cnt += face_class(n, cell, 1, i, j, k) != ORC_WALL;
                cnt += face_class(n, cell, 1, i, j + 1, k) != ORC_WALL;
                cnt += face_class(n, cell, 2, i, j, k) != ORC_WALL;
                cnt += face_class(n, cell, 2, i, j, k + 1) != ORC_WALL;
                diag[c] = (double)cnt;
            }
}

/* (A p)_c = n_c p_c - sum of p over liquid neighbours, for liquid c; the
 * pressure of air cells is zero (R7) so they drop out; zero off-liquid. */
void orc_poisson_apply(int n, const uint8_t* cell, const double* p, double* out) {
    static const int nb[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    double* diag = (double*)malloc(sizeof(double) * (long)n * n * n);
    orc_poisson_diag(n, cell, diag);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long c = cidx(n, i, j, k);
                if (cell[c] != ORC_LIQUID) {
                    out[c] = 0.0;
                    continue;
                }
                double s = diag[c] * p[c];
                for (int q = 0; q < 6; ++q) {
                    int ii = i + nb[q][0], jj = j + nb[q][1], kk = k + nb[q][2];
                    if (cell_type(n, cell, ii, jj, kk) == ORC_LIQUID) s -= p[cidx(n, ii, jj, kk)];
                }
                out[c] = s;
            }
    free(diag);
}

/* Right-hand side b_c = -h * (net outward flux of c) for liquid c; this is
 * -h^2 times the discrete divergence (Poisson pressure equation with the
 * pressure scaled by dt/rho, R8). */
void orc_divergence_rhs(int n, const uint8_t* cell, const double* u, const double* v,
                        const double* w, double* b) {
    int du[3], dv[3], dw[3];
    face_dims(n, 0, du);
    face_dims(n, 1, dv);
    face_dims(n, 2, dw);
    double h = 1.0 / n;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long c = cidx(n, i, j, k);
                if (cell[c] != ORC_LIQUID) {
                    b[c] = 0.0;
                    continue;
                }
                double flux = u[fidx(du, i + 1, j, k)] - u[fidx(du, i, j, k)] +
                              v[fidx(dv, i, j + 1, k)] - v[fidx(dv, i, j, k)] +
                              w[fidx(dw, i, j, k + 1)] - w[fidx(dw, i, j, k)];
                b[c] = -h * flux;
            }
}

/* u_f -= (p_plus - p_minus)/h on active faces, p = 0 off liquid; every other
 * face is set to zero. */
void orc_pressure_update(int n, const uint8_t* cell, const double* p, double* u, double* v,
                         double* w) {
    for (int comp = 0; comp < 3; ++comp) {
        int d[3];
        face_dims(n, comp, d);
        double* f = comp == 0 ? u : (comp == 1 ? v : w);
        for (int k = 0; k < d[2]; ++k)
            for (int j = 0; j < d[1]; ++j)
                for (int i = 0; i < d[0]; ++i) {
                    long id = fidx(d, i, j, k);
                    if (face_class(n, cell, comp, i, j, k) != ORC_ACTIVE) {
                        f[id] = 0.0;
                        continue;
                    }
                    int im = i - (comp == 0), jm = j - (comp == 1), km = k - (comp == 2);
                    double pp = cell_type(n, cell, i, j, k) == ORC_LIQUID ? p[cidx(n, i, j, k)] : 0.0;
                    double pm =
                        cell_type(n, cell, im, jm, km) == ORC_LIQUID ? p[cidx(n, im, jm, km)] : 0.0;
                    f[id] -= (pp - pm) * (double)n;
                }
    }
}

/* ------------------------------------------------------------- MIC(0) */

/* Coupling of liquid cell (i,j,k) to its + neighbour along axis a: the
 * off-diagonal entry of the Poisson matrix, -1 when both are liquid. */
static double aplus(int n, const uint8_t* cell, int a, int i, int j, int k) {
    if (cell_type(n, cell, i, j, k) != ORC_LIQUID) return 0.0;
    int ii = i + (a == 0), jj = j + (a == 1), kk = k + (a == 2);
    return cell_type(n, cell, ii, jj, kk) == ORC_LIQUID ? -1.0 : 0.0;
}

static double prec_at(int n, const uint8_t* cell, const double* precon, int i, int j, int k) {
    if (cell_type(n, cell, i, j, k) != ORC_LIQUID) return 0.0;
    return precon[cidx(n, i, j, k)];
}

/* Modified incomplete Cholesky, level 0, in lexicographic order (x fastest):
 * E_c = A_cc - sum over the three lower neighbours m of (A_mc precon_m)^2
 *       - tau * sum over m of A_mc (sum of m's other two upper couplings) precon_m^2,
 * replaced by A_cc when E_c < sigma * A_cc; precon_c = 1/sqrt(E_c). */
void orc_mic0_setup(int n, const uint8_t* cell, double tau, double sigma, double* precon) {
    double* diag = (double*)malloc(sizeof(double) * (long)n * n * n);
    orc_poisson_diag(n, cell, diag);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long c = cidx(n, i, j, k);
                if (cell[c] != ORC_LIQUID) {
                    precon[c] = 0.0;
                    continue;
                }
                double ax = aplus(n, cell, 0, i - 1, j, k), px = prec_at(n, cell, precon, i - 1, j, k);
                double ay = aplus(n, cell, 1, i, j - 1, k), py = prec_at(n, cell, precon, i, j - 1, k);
                double az = aplus(n, cell, 2, i, j, k - 1), pz = prec_at(n, cell, precon, i, j, k - 1);
                double e = diag[c] - (ax * px) * (ax * px) - (ay * py) * (ay * py) - (az * pz) * (az * pz);
                double ox = aplus(n, cell, 1, i - 1, j, k) + aplus(n, cell, 2, i - 1, j, k);
                double oy = aplus(n, cell, 0, i, j - 1, k) + aplus(n, cell, 2, i, j - 1, k);
                double oz = aplus(n, cell, 0, i, j, k - 1) + aplus(n, cell, 1, i, j, k - 1);
                e -= tau * (ax * ox * px * px + ay * oy * py * py + az * oz * pz * pz);
                if (e < sigma * diag[c]) e = diag[c];
                precon[c] = 1.0 / sqrt(e);
            }
    free(diag);
}

/* z = (L L^T)^-1 r with L from orc_mic0_setup: forward substitution in
 * lexicographic order, then back substitution in reverse order. */
void orc_mic0_apply(int n, const uint8_t* cell, const double* precon, const double* r,
                    double* z) {
    long nc = (long)n * n * n;
    double* q = (double*)calloc(nc, sizeof(double));
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long c = cidx(n, i, j, k);
                if (cell[c] != ORC_LIQUID) continue;
                double t = r[c];
                if (i > 0) t -= aplus(n, cell, 0, i - 1, j, k) * prec_at(n, cell, precon, i - 1, j, k) * q[cidx(n, i - 1, j, k)];
                if (j > 0) t -= aplus(n, cell, 1, i, j - 1, k) * prec_at(n, cell, precon, i, j - 1, k) * q[cidx(n, i, j - 1, k)];
                if (k > 0) t -= aplus(n, cell, 2, i, j, k - 1) * prec_at(n, cell, precon, i, j, k - 1) * q[cidx(n, i, j, k - 1)];
                q[c] = t * precon[c];
            }
    for (long c = 0; c < nc; ++c) z[c] = 0.0;
    for (int k = n - 1; k >= 0; --k)
        for (int j = n - 1; j >= 0; --j)
            for (int i = n - 1; i >= 0; --i) {
                long c = cidx(n, i, j, k);
                if (cell[c] != ORC_LIQUID) continue;
                double t = q[c];
                if (i + 1 < n) t -= aplus(n, cell, 0, i, j, k) * precon[c] * z[cidx(n, i + 1, j, k)];
                if (j + 1 < n) t -= aplus(n, cell, 1, i, j, k) * precon[c] * z[cidx(n, i, j + 1, k)];
                if (k + 1 < n) t -= aplus(n, cell, 2, i, j, k) * precon[c] * z[cidx(n, i, j, k + 1)];
                z[c] = t * precon[c];
            }
    free(q);
}

/* ----------------------------------------------------------------- PCG */

double orc_true_relres(int n, const uint8_t* cell, const double* b, const double* x) {
    long nc = (long)n * n * n;
    double* ax = (double*)malloc(sizeof(double) * nc);
    orc_poisson_apply(n, cell, x, ax);
    double rr = 0.0, bb = 0.0;
    for (long c = 0; c < nc; ++c) {
        double r = b[c] - ax[c];
        rr += r * r;
        bb += b[c] * b[c];
    }
    free(ax);
    return bb > 0.0 ? sqrt(rr / bb) : 0.0;
}

/* Preconditioned conjugate gradients on the Poisson matrix, from the given
 * x, stopping when the relative residual (recursive, FP64) reaches tol.
 * Returns the iteration count; relres receives the true relative residual. */
int orc_pcg(int n, const uint8_t* cell, const double* b, double* x, int precond, double tol,
            int max_iter, double* relres) {
    long nc = (long)n * n * n;
    double* r = (double*)malloc(sizeof(double) * nc);
    double* z = (double*)malloc(sizeof(double) * nc);
    double* d = (double*)malloc(sizeof(double) * nc);
    double* q = (double*)malloc(sizeof(double) * nc);
    double* diag = (double*)malloc(sizeof(double) * nc);
    double* precon = NULL;
    orc_poisson_diag(n, cell, diag);
    if (precond == ORC_PRECOND_MIC0) {
        precon = (double*)malloc(sizeof(double) * nc);
        orc_mic0_setup(n, cell, 0.97, 0.25, precon);
    }
    orc_poisson_apply(n, cell, x, q);
    for (long c = 0; c < nc; ++c) r[c] = b[c] - q[c];
    double bn = sqrt(dot(nc, b, b));
    int it = 0;
    if (bn == 0.0) {
        for (long c = 0; c < nc; ++c) x[c] = 0.0;
        if (relres) *relres = 0.0;
        goto done;
    }
#define APPLY_M(rv, zv)                                                               \
    do {                                                                              \
        if (precond == ORC_PRECOND_MIC0)                                              \
            orc_mic0_apply(n, cell, precon, rv, zv);                                  \
        else if (precond == ORC_PRECOND_JACOBI)                                       \
            for (long c = 0; c < nc; ++c) zv[c] = diag[c] > 0 ? rv[c] / diag[c] : 0.0; \
        else                                                                          \
            for (long c = 0; c < nc; ++c) zv[c] = rv[c];                              \
    } while (0)
    APPLY_M(r, z);
    memcpy(d, z, sizeof(double) * nc);
    double rz = dot(nc, r, z);
    while (sqrt(dot(nc, r, r)) / bn > tol && it < max_iter) {
        orc_poisson_apply(n, cell, d, q);
        double alpha = rz / dot(nc, d, q);
        for (long c = 0; c < nc; ++c) {
            x[c] += alpha * d[c];
            r[c] -= alpha * q[c];
        }
        APPLY_M(r, z);
        double rz_new = dot(nc, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
        for (long c = 0; c < nc; ++c) d[c] = z[c] + beta * d[c];
        ++it;
    }
#undef APPLY_M
    if (relres) *relres = orc_true_relres(n, cell, b, x);
done:
    free(r); free(z); free(d); free(q); free(diag);
    free(precon);
    return it;
}

/* ------------------------------------------------------------ adjoints */

/* Transpose of the Jacobian of orc_advect with respect to (u, v, w), applied
 * to (lu, lv, lw) and ADDED to (gu, gv, gw).  The sampled value depends on
 * the field through the trilinear weights at the departure point and on the
 * departure point through the face velocity, which is itself a trilinear
 * sample of the three components at the face (exact discrete adjoint,
 * R13).  Sequential, so the scatter order is fixed. */
void orc_advect_adjoint(int n, const uint8_t* cell, const double* u, const double* v,
                        const double* w, double dt_over_h, const double* lu, const double* lv,
                        const double* lw, double* gu, double* gv, double* gw) {
    for (int comp = 0; comp < 3; ++comp) {
        int d[3];
        face_dims(n, comp, d);
        const double* lam = pick(comp, lu, lv, lw);
        double* gc = comp == 0 ? gu : (comp == 1 ? gv : gw);
        for (int k = 0; k < d[2]; ++k)
            for (int j = 0; j < d[1]; ++j)
                for (int i = 0; i < d[0]; ++i) {
                    long id = fidx(d, i, j, k);
                    if (face_class(n, cell, comp, i, j, k) != ORC_ACTIVE) continue;
                    double l = lam[id];
                    if (l == 0.0) continue;
                    double gf[3] = {i + (comp == 0 ? 0.0 : 0.5), j + (comp == 1 ? 0.0 : 0.5),
                                    k + (comp == 2 ? 0.0 : 0.5)};
                    double U[3];
                    for (int a = 0; a < 3; ++a) U[a] = orc_sample(n, a, pick(a, u, v, w), gf, NULL);
                    double gd[3];
                    for (int a = 0; a < 3; ++a) gd[a] = gf[a] - dt_over_h * U[a];
                    double grad[3];
                    orc_sample(n, comp, pick(comp, u, v, w), gd, grad);
                    scatter_sample(n, comp, gc, gd, l);
                    for (int a = 0; a < 3; ++a) {
                        double s = l * (-dt_over_h) * grad[a];
                        if (s != 0.0) scatter_sample(n, a, a == 0 ? gu : (a == 1 ? gv : gw), gf, s);
                    }
                }
    }
}
