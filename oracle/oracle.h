/*
 * FP64 CPU oracle for the MAC-grid liquid step (test infrastructure only).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this library.  It shares no code with the GPU path.  Every routine is a
 * plain loop over the grid in double precision, written to be read against
 * the definitions, not to be fast.
 *
 * Grid: unit box, n cells per axis, h = 1/n.  Arrays are flat, x fastest.
 *   cell (i,j,k)           -> i + n*(j + n*k)
 *   u face (i,j,k), i<=n   -> i + (n+1)*(j + n*k)      at (i h, (j+.5)h, (k+.5)h)
 *   v face (i,j,k), j<=n   -> i + n*(j + (n+1)*k)      at ((i+.5)h, j h, (k+.5)h)
 *   w face (i,j,k), k<=n   -> i + n*(j + n*k)          at ((i+.5)h, (j+.5)h, k h)
 * Cell types: 0 air, 1 liquid, 2 solid; outside the box counts as solid.
 * Face classes: wall (touches a solid cell), active (not wall, touches
 * liquid), inactive (air on both sides).
 */
#ifndef FLUID_ORACLE_H
#define FLUID_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_AIR = 0, ORC_LIQUID = 1, ORC_SOLID = 2 };
enum { ORC_INACTIVE = 0, ORC_ACTIVE = 1, ORC_WALL = 2 };
enum { ORC_PRECOND_NONE = 0, ORC_PRECOND_JACOBI = 1, ORC_PRECOND_MIC0 = 2 };

long orc_face_count(int n, int comp);
void orc_face_classes(int n, const uint8_t* cell, int comp, uint8_t* out);
void orc_mask_faces(int n, const uint8_t* cell, int comp, double* f);

/* trilinear sample of component comp at grid-unit position g (x/h, y/h, z/h);
 * grad (nullable) receives d/dg of the sample, zero on clamped axes */
double orc_sample(int n, int comp, const double* f, const double g[3], double grad[3]);

void orc_advect(int n, const uint8_t* cell, const double* u, const double* v, const double* w,
                double dt_over_h, double* au, double* av, double* aw);
/* d(advected face value)/d(dt) on active faces (0 elsewhere) */
void orc_advect_ddt(int n, const uint8_t* cell, const double* u, const double* v, const double* w,
                    double dt_over_h, double* du, double* dv, double* dw);
void orc_add_force(int n, const uint8_t* cell, double* u, double* v, double* w,
                   double dt, const double g[3]);
void orc_laplacian(int n, const uint8_t* cell, int comp, const double* f, double* out);
void orc_diffuse_explicit(int n, const uint8_t* cell, int comp, double nu_dt,
                          const double* f, double* out);
int orc_diffuse_implicit(int n, const uint8_t* cell, int comp, double nu_dt, const double* f,
                         double* out, double tol, int max_iter, double* relres);

void orc_poisson_diag(int n, const uint8_t* cell, double* diag);
void orc_poisson_apply(int n, const uint8_t* cell, const double* p, double* out);
void orc_divergence_rhs(int n, const uint8_t* cell, const double* u, const double* v,
                        const double* w, double* b);
void orc_pressure_update(int n, const uint8_t* cell, const double* p, double* u, double* v,
                         double* w);
void orc_mic0_setup(int n, const uint8_t* cell, double tau, double sigma, double* precon);
void orc_mic0_apply(int n, const uint8_t* cell, const double* precon, const double* r,
                    double* z);
int orc_pcg(int n, const uint8_t* cell, const double* b, double* x, int precond, double tol,
            int max_iter, double* relres);
double orc_true_relres(int n, const uint8_t* cell, const double* b, const double* x);

void orc_advect_adjoint(int n, const uint8_t* cell, const double* u, const double* v,
                        const double* w, double dt_over_h, const double* lu, const double* lv,
                        const double* lw, double* gu, double* gv, double* gw);

#ifdef __cplusplus
}
#endif
#endif
