/*
 * gray_oracle.h -- plain FP64 CPU oracle for Kerr photon-geodesic ray tracing
 * as described by Chan, Psaltis & Ozel (2013), "GRay", Sec. 2.
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the GPU path. Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg load
 * it; the product library never includes this header, links this code or
 * calls it, and the two share no source.
 *
 * Conventions: G = c = M = 1, Boyer-Lindquist coordinates, index order
 * 0 = t, 1 = r, 2 = theta, 3 = phi. A photon state is the 8-vector
 * (t, r, theta, phi, k^t, k^r, k^theta, k^phi); k is the tangent that is
 * integrated (the photon's physical momentum p = -k, traced backwards).
 */
#ifndef GRAY_ORACLE_H
#define GRAY_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_METRIC_KERR = 0, ORACLE_METRIC_JP = 1 };

enum { ORACLE_RUNNING = 0, ORACLE_CAPTURED = 1, ORACLE_ESCAPED = 2,
       ORACLE_UNFINISHED = 3, ORACLE_NONFINITE = 4 };

typedef struct {
    double step_frac;   /* Delta of the step-size rule, Sec. 2 eq. (2); ~1/32     */
    double horizon_eps; /* capture once r < r_bh (1 + horizon_eps)                */
    double r_escape;    /* escape once r > r_escape while moving outward          */
    double xi_eps;      /* epsilon of the null-condition monitor, Sec. 2 eq. (4)  */
    double euler_div;   /* fallback Euler step is h / euler_div (9 in Sec. 2)     */
    double disk_rmin;   /* equatorial recorder window; < 0 means r_ISCO(a)        */
    double disk_rmax;
    int32_t max_steps;  /* total accepted steps before UNFINISHED                 */
    int32_t record_disk;/* nonzero: record the first in-window equatorial crossing */
    int32_t pole_mode;  /* treatment of the polar axis (Sec. 2, Fig. 2):
                           0 production: null monitor eq. (4), Euler at h/euler_div;
                           1 earlier scheme: one Euler step of the same h whenever
                             the RK4 step crosses a pole;
                           2 none: RK4 and the remap of eq. (3) only             */
    int32_t metric;     /* ORACLE_METRIC_KERR, or ORACLE_METRIC_JP: the deformed
                           Kerr metric of oracle_metric_jp with deviation eps3
                           (camera states for it come from oracle_camera_jp)   */
    double eps3;
} oracle_params;

typedef struct {
    double a, r_obs, incl;          /* spin, observer distance, inclination (rad) */
    int32_t nx, ny;                 /* pixels; pixel id = iy * nx + ix            */
    double alpha_lo, alpha_hi;      /* cell-centred image-plane grid (M)          */
    double beta_lo, beta_hi;
} oracle_camera_t;

/* Spacetime. */
double oracle_horizon(double a);
double oracle_r_isco(double a);
void oracle_metric(double a, double r, double th, double g[16]);
void oracle_metric_deriv(double a, double r, double th, double dgr[16], double dgth[16]);
void oracle_christoffel(double a, double r, double th, double G[64]);
void oracle_rhs(double a, const double x[8], double f[8]);

/* Deformed Kerr metric (Johannsen & Psaltis 2011, deviation eps3; eps3 = 0 is
 * Kerr): metric, complex-step derivatives, Christoffel symbols, RHS, null
 * monitor, camera and constants (E, L_z; Q in its Kerr form). */
void oracle_metric_jp(double a, double eps3, double r, double th, double g[16]);
void oracle_metric_deriv_jp(double a, double eps3, double r, double th, double dgr[16], double dgth[16]);
void oracle_christoffel_jp(double a, double eps3, double r, double th, double G[64]);
void oracle_rhs_jp(double a, double eps3, const double x[8], double f[8]);
double oracle_xi_jp(double a, double eps3, const double x[8]);
void oracle_camera_jp(double a, double eps3, double r_obs, double incl, double alpha, double beta, double x[8]);
void oracle_conserved_jp(double a, double eps3, const double x[8], double out[3]);

/* Image plane. */
void oracle_camera(double a, double r_obs, double incl, double alpha, double beta, double x[8]);
void oracle_camera_grid(const oracle_camera_t *cam, double *x /* nx*ny*8, pixel-major */);

/* Integrator pieces (Sec. 2). */
double oracle_step_size(double rbh, double step_frac, const double x[8]);
double oracle_xi(double a, const double x[8]);
int oracle_remap(double x[8]);
int oracle_step(const oracle_params *p, double a, double x[8], double *h_used);

/* Diagnostics. */
void oracle_conserved(double a, const double x[8], double out[3]);
double oracle_disk_redshift(double a, double rc, double E, double L);

/* Whole trajectories. */
int oracle_trace(const oracle_params *p, double a, double x[8], int32_t *steps,
                 int32_t *n_euler, int32_t *n_remap, double disk[3]);
int oracle_trace_mark(const oracle_params *p, double a, double x[8], int32_t *steps,
                      int32_t *n_euler, int32_t *n_remap, double disk[3], double mark[8]);
int oracle_trace_path(const oracle_params *p, double a, double x[8], int32_t max_pts,
                      double *path, int32_t *flags, int32_t *n_pts);
void oracle_run(const oracle_params *p, int64_t n, const double *a, double *x,
                int32_t *status, int32_t *steps, int32_t *n_euler, int32_t *n_remap,
                double *disk, double *mark, int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
