/*
 * gray_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for the
 * Kerr photon-geodesic integrator of Chan, Psaltis & Ozel (2013), "GRay".
 *
 * TEST INFRASTRUCTURE ONLY: see gray_oracle.h. Nothing in the product path
 * includes, links or calls this file.
 *
 * What it computes, and where each piece comes from:
 *   - Kerr spacetime in Boyer-Lindquist coordinates, G = c = M = 1, spin a,
 *     horizon r_bh = 1 + sqrt(1 - a^2) (Sec. 1 and Sec. 2).
 *   - The second-order geodesic equation dx/dl = k, dk^mu/dl =
 *     -Gamma^mu_{ab} k^a k^b, integrated for all eight components (Sec. 1
 *     motivates the second-order form; Sec. 2 integrates it). The paper
 *     defers the equations to an earlier paper; here the Christoffel symbols
 *     are assembled from their textbook definition out of the analytic
 *     metric derivatives and the inverse metric.
 *   - Classical fourth-order Runge-Kutta with the step-size rule of Sec. 2
 *     eq. (2), the horizon stop, the theta remap of eq. (3), and the
 *     null-condition monitor of eq. (4) with its forward-Euler re-integration
 *     at h/9.
 *   - The image plane at r_obs (Sec. 2 and Sec. 3; the paper defers its
 *     construction) read as a flat, plane-parallel screen; each ray is traced
 *     backwards, k = -p.
 *
 *   - Optionally a deformed Kerr metric (Johannsen & Psaltis 2011, one
 *     deviation parameter eps3), the kind of non-Kerr spacetime Sec. 1 gives
 *     as the reason to integrate the second-order equations: it has no
 *     Carter constant. The paper gives no formula for it; see
 *     oracle_metric_jp. Its metric derivatives are taken by the complex step
 *     (exact to rounding, no truncation error) and the Christoffel symbols
 *     by the same definition-based sum as for Kerr.
 *
 * Built with -O2 -ffp-contract=off and no fast-math, so every operation is
 * a separately rounded IEEE double operation in the order written here.
 */
#include "gray_oracle.h"

#include <complex.h>
#include <math.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IX(mu, nu) ((mu) * 4 + (nu))

static const double ORACLE_PI = 3.14159265358979323846;

/* Outer horizon of Kerr, r_bh = 1 + sqrt(1 - a^2) (Sec. 2). */
double oracle_horizon(double a) { return 1.0 + sqrt(1.0 - a * a); }

/* Prograde innermost stable circular orbit (Bardeen, Press & Teukolsky 1972):
 * only used for the equatorial-crossing window of the grid-projection
 * workload (Sec. 3), which the paper states without a formula. */
double oracle_r_isco(double a)
{
    double z1 = 1.0 + cbrt(1.0 - a * a) * (cbrt(1.0 + a) + cbrt(1.0 - a));
    double z2 = sqrt(3.0 * a * a + z1 * z1);
    return 3.0 + z2 - sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

/* Covariant Kerr metric g_{mu nu} at (r, theta), Boyer-Lindquist form. */
void oracle_metric(double a, double r, double th, double g[16])
{
    double s = sin(th), c = cos(th);
    double sig = r * r + a * a * c * c;
    double del = r * r - 2.0 * r + a * a;
    memset(g, 0, 16 * sizeof(double));
    g[IX(0, 0)] = -(1.0 - 2.0 * r / sig);
    g[IX(0, 3)] = -2.0 * a * r * s * s / sig;
    g[IX(3, 0)] = g[IX(0, 3)];
    g[IX(1, 1)] = sig / del;
    g[IX(2, 2)] = sig;
    g[IX(3, 3)] = (r * r + a * a + 2.0 * a * a * r * s * s / sig) * s * s;
}

/* Analytic partial derivatives of g_{mu nu} with respect to r and theta,
 * written out with the product and quotient rules term by term. The metric
 * does not depend on t or phi. */
void oracle_metric_deriv(double a, double r, double th, double dgr[16], double dgth[16])
{
    double s = sin(th), c = cos(th);
    double sig = r * r + a * a * c * c;
    double sig_r = 2.0 * r;
    double sig_th = -2.0 * a * a * c * s;
    double del = r * r - 2.0 * r + a * a;
    double del_r = 2.0 * r - 2.0;
    double sig2 = sig * sig;

    memset(dgr, 0, 16 * sizeof(double));
    memset(dgth, 0, 16 * sizeof(double));

    /* g_tt = -1 + 2 r / Sigma */
    dgr[IX(0, 0)] = 2.0 / sig - 2.0 * r * sig_r / sig2;
    dgth[IX(0, 0)] = -2.0 * r * sig_th / sig2;

    /* g_tphi = -2 a r sin^2 / Sigma */
    dgr[IX(0, 3)] = -2.0 * a * s * s / sig + 2.0 * a * r * s * s * sig_r / sig2;
    dgth[IX(0, 3)] = -4.0 * a * r * s * c / sig + 2.0 * a * r * s * s * sig_th / sig2;
    dgr[IX(3, 0)] = dgr[IX(0, 3)];
    dgth[IX(3, 0)] = dgth[IX(0, 3)];

    /* g_rr = Sigma / Delta */
    dgr[IX(1, 1)] = sig_r / del - sig * del_r / (del * del);
    dgth[IX(1, 1)] = sig_th / del;

    /* g_thth = Sigma */
    dgr[IX(2, 2)] = sig_r;
    dgth[IX(2, 2)] = sig_th;

    /* g_phph = F sin^2, F = r^2 + a^2 + 2 a^2 r sin^2 / Sigma */
    double F = r * r + a * a + 2.0 * a * a * r * s * s / sig;
    double F_r = 2.0 * r + 2.0 * a * a * s * s / sig - 2.0 * a * a * r * s * s * sig_r / sig2;
    double F_th = 4.0 * a * a * r * s * c / sig - 2.0 * a * a * r * s * s * sig_th / sig2;
    dgr[IX(3, 3)] = F_r * s * s;
    dgth[IX(3, 3)] = F_th * s * s + 2.0 * F * s * c;
}

/* Inverse metric: g^rr and g^thth are reciprocals; the t-phi block is the
 * inverse of a symmetric 2x2 matrix. */
static void inverse_metric(const double g[16], double gi[16])
{
    memset(gi, 0, 16 * sizeof(double));
    double det = g[IX(0, 0)] * g[IX(3, 3)] - g[IX(0, 3)] * g[IX(0, 3)];
    gi[IX(0, 0)] = g[IX(3, 3)] / det;
    gi[IX(0, 3)] = -g[IX(0, 3)] / det;
    gi[IX(3, 0)] = gi[IX(0, 3)];
    gi[IX(3, 3)] = g[IX(0, 0)] / det;
    gi[IX(1, 1)] = 1.0 / g[IX(1, 1)];
    gi[IX(2, 2)] = 1.0 / g[IX(2, 2)];
}

/* Christoffel symbols of the second kind from their definition,
 *   Gamma^mu_{ab} = 1/2 g^{mu nu} (d_a g_{nu b} + d_b g_{nu a} - d_nu g_{ab}),
 * stored as G[mu*16 + a*4 + b], given the metric and its r and theta
 * derivatives (the metrics here depend on neither t nor phi). */
static void christoffel_from(const double g[16], const double dgr[16], const double dgth[16], double G[64])
{
    double gi[16], dg[4][16];
    inverse_metric(g, gi);
    memset(dg, 0, sizeof dg);
    memcpy(dg[1], dgr, sizeof dg[1]);
    memcpy(dg[2], dgth, sizeof dg[2]);

    for (int mu = 0; mu < 4; ++mu)
        for (int al = 0; al < 4; ++al)
            for (int be = 0; be < 4; ++be) {
                double sum = 0.0;
                for (int nu = 0; nu < 4; ++nu)
                    sum += gi[IX(mu, nu)] *
                           (dg[al][IX(nu, be)] + dg[be][IX(nu, al)] - dg[nu][IX(al, be)]);
                G[mu * 16 + al * 4 + be] = 0.5 * sum;
            }
}

void oracle_christoffel(double a, double r, double th, double G[64])
{
    double g[16], dgr[16], dgth[16];
    oracle_metric(a, r, th, g);
    oracle_metric_deriv(a, r, th, dgr, dgth);
    christoffel_from(g, dgr, dgth, G);
}

/* Deformed Kerr metric of Johannsen & Psaltis (2011) with the deviation
 * function h = eps3 r / Sigma^2 (their leading parameter epsilon_3, M = 1):
 *   g_tt   = -(1 + h) (1 - 2 r / Sigma)
 *   g_tphi = -(2 a r sin^2 / Sigma) (1 + h)
 *   g_rr   = Sigma (1 + h) / (Delta + a^2 sin^2 h)
 *   g_thth = Sigma
 *   g_phph = sin^2 (r^2 + a^2 + 2 a^2 r sin^2 / Sigma) + h a^2 (Sigma + 2 r) sin^4 / Sigma
 * eps3 = 0 is the Kerr metric. It is stationary and axisymmetric (E and L_z
 * are conserved) but has no Carter constant for eps3 != 0. Evaluated in
 * complex arithmetic so that the same expression yields the derivatives by
 * the complex step (oracle_metric_deriv_jp). */
static void jp_metric_c(double a, double eps3, double complex r, double complex th, double complex g[16])
{
    double complex s = csin(th), c = ccos(th);
    double complex s2 = s * s;
    double complex sig = r * r + a * a * c * c;
    double complex del = r * r - 2.0 * r + a * a;
    double complex h = eps3 * r / (sig * sig);
    for (int k = 0; k < 16; ++k) g[k] = 0.0;
    g[IX(0, 0)] = -(1.0 + h) * (1.0 - 2.0 * r / sig);
    g[IX(0, 3)] = -(2.0 * a * r * s2 / sig) * (1.0 + h);
    g[IX(3, 0)] = g[IX(0, 3)];
    g[IX(1, 1)] = sig * (1.0 + h) / (del + a * a * s2 * h);
    g[IX(2, 2)] = sig;
    g[IX(3, 3)] = s2 * (r * r + a * a + 2.0 * a * a * r * s2 / sig) + h * a * a * (sig + 2.0 * r) * s2 * s2 / sig;
}

void oracle_metric_jp(double a, double eps3, double r, double th, double g[16])
{
    double complex gc[16];
    jp_metric_c(a, eps3, r, th, gc);
    for (int k = 0; k < 16; ++k) g[k] = creal(gc[k]);
}

/* d_r and d_theta of the deformed metric by the complex step: for f analytic
 * and real on the real axis, f'(x) = Im f(x + i eta) / eta + O(eta^2) with no
 * subtraction, so a tiny eta gives the derivative to rounding. */
void oracle_metric_deriv_jp(double a, double eps3, double r, double th, double dgr[16], double dgth[16])
{
    const double eta = 1e-20;
    double complex gr[16], gt[16];
    jp_metric_c(a, eps3, r + eta * I, th, gr);
    jp_metric_c(a, eps3, r, th + eta * I, gt);
    for (int k = 0; k < 16; ++k) {
        dgr[k] = cimag(gr[k]) / eta;
        dgth[k] = cimag(gt[k]) / eta;
    }
}

void oracle_christoffel_jp(double a, double eps3, double r, double th, double G[64])
{
    double g[16], dgr[16], dgth[16];
    oracle_metric_jp(a, eps3, r, th, g);
    oracle_metric_deriv_jp(a, eps3, r, th, dgr, dgth);
    christoffel_from(g, dgr, dgth, G);
}

/* Covariant metric of the spacetime the parameters select. */
static void metric_of(const oracle_params *p, double a, double r, double th, double g[16])
{
    if (p->metric == ORACLE_METRIC_JP)
        oracle_metric_jp(a, p->eps3, r, th, g);
    else
        oracle_metric(a, r, th, g);
}

/* Right-hand side of the geodesic equation for the 8-vector state:
 * dx^mu/dl = k^mu, dk^mu/dl = -Gamma^mu_{ab} k^a k^b. */
static void rhs_from(const double G[64], const double x[8], double f[8])
{
    for (int mu = 0; mu < 4; ++mu) f[mu] = x[4 + mu];
    for (int mu = 0; mu < 4; ++mu) {
        double acc = 0.0;
        for (int al = 0; al < 4; ++al)
            for (int be = 0; be < 4; ++be)
                acc += G[mu * 16 + al * 4 + be] * x[4 + al] * x[4 + be];
        f[4 + mu] = -acc;
    }
}

void oracle_rhs(double a, const double x[8], double f[8])
{
    double G[64];
    oracle_christoffel(a, x[1], x[2], G);
    rhs_from(G, x, f);
}

void oracle_rhs_jp(double a, double eps3, const double x[8], double f[8])
{
    double G[64];
    oracle_christoffel_jp(a, eps3, x[1], x[2], G);
    rhs_from(G, x, f);
}

static void rhs_of(const oracle_params *p, double a, const double x[8], double f[8])
{
    if (p->metric == ORACLE_METRIC_JP)
        oracle_rhs_jp(a, p->eps3, x, f);
    else
        oracle_rhs(a, x, f);
}

/* Initial state of one ray. The observer sits at distance D = r_obs in the
 * direction (theta = incl, phi = 0); the image plane is the flat plane through
 * the observer perpendicular to the line of sight, with alpha along +phi-hat
 * and beta along -theta-hat (towards the spin axis). The ray arriving at the
 * screen point (alpha, beta) travels along the line of sight n; its momentum p
 * has the flat-space spherical components of n at that point, and p^t > 0
 * follows from the null condition in the Kerr metric there. The state that is
 * integrated is k = -p (the ray is traced back towards the hole).
 * A ray exactly on the spin axis (incl = 0, alpha = beta = 0) has undefined
 * theta and phi directions; it is given p^theta = p^phi = 0 there. */
static void camera_in(int metric, double eps3, double a, double r_obs, double incl, double alpha, double beta,
                      double x[8])
{
    double D = r_obs;
    double si = sin(incl), ci = cos(incl);
    double X = D * si - beta * ci;
    double Y = alpha;
    double Z = D * ci + beta * si;
    double b2 = alpha * alpha + beta * beta;
    double r0 = sqrt(D * D + b2);
    double rho2 = X * X + Y * Y;
    double rho = sqrt(rho2);

    double th0 = atan2(rho, Z);
    double ph0 = atan2(Y, X);
    double pr = D / r0;
    double pth = 0.0, pph = 0.0;
    if (rho > 0.0) {
        /* d theta along n: (D Z / r0^2 - cos i) / rho, rewritten without the
         * cancellation between the two terms. */
        pth = (D * beta * si - b2 * ci) / (r0 * r0 * rho);
        /* d phi along n: (X n_y - Y n_x) / rho^2 with n = (sin i, 0, cos i). */
        pph = -alpha * si / rho2;
    }

    double g[16];
    if (metric == ORACLE_METRIC_JP)
        oracle_metric_jp(a, eps3, r0, th0, g);
    else
        oracle_metric(a, r0, th0, g);
    double S = g[IX(1, 1)] * pr * pr + g[IX(2, 2)] * pth * pth + g[IX(3, 3)] * pph * pph;
    double B = g[IX(0, 3)] * pph;
    /* g_tt (p^t)^2 + 2 B p^t + S = 0, root with p^t > 0 (g_tt < 0 far out). */
    double pt = (-B - sqrt(B * B - g[IX(0, 0)] * S)) / g[IX(0, 0)];

    x[0] = 0.0;
    x[1] = r0;
    x[2] = th0;
    x[3] = ph0;
    x[4] = -pt;
    x[5] = -pr;
    x[6] = -pth;
    x[7] = -pph;
}

void oracle_camera(double a, double r_obs, double incl, double alpha, double beta, double x[8])
{
    camera_in(ORACLE_METRIC_KERR, 0.0, a, r_obs, incl, alpha, beta, x);
}

/* The same screen in the deformed metric (p^t from its null condition). */
void oracle_camera_jp(double a, double eps3, double r_obs, double incl, double alpha, double beta, double x[8])
{
    camera_in(ORACLE_METRIC_JP, eps3, a, r_obs, incl, alpha, beta, x);
}

/* Regular cell-centred grid of rays; pixel id = iy * nx + ix. */
void oracle_camera_grid(const oracle_camera_t *cam, double *x)
{
    for (int32_t iy = 0; iy < cam->ny; ++iy)
        for (int32_t ix = 0; ix < cam->nx; ++ix) {
            double alpha = cam->alpha_lo + (cam->alpha_hi - cam->alpha_lo) * ((ix + 0.5) / cam->nx);
            double beta = cam->beta_lo + (cam->beta_hi - cam->beta_lo) * ((iy + 0.5) / cam->ny);
            oracle_camera(cam->a, cam->r_obs, cam->incl, alpha, beta,
                          x + ((int64_t)iy * cam->nx + ix) * 8);
        }
}

/* Step-size rule, Sec. 2 eq. (2):
 *   h = min( Delta / (|d ln r/dl| + |d theta/dl| + |d phi/dl|),
 *            (r - r_bh) / (2 |dr/dl|) ),
 * the second term being +infinity when dr/dl = 0. */
double oracle_step_size(double rbh, double step_frac, const double x[8])
{
    double r = x[1];
    double h1 = step_frac / (fabs(x[5]) / r + fabs(x[6]) + fabs(x[7]));
    double h2 = (x[5] != 0.0) ? (r - rbh) / (2.0 * fabs(x[5])) : INFINITY;
    return (h2 < h1) ? h2 : h1;
}

/* Null-condition monitor xi of Sec. 2 eq. (4); -1 on an exact null ray. */
static double xi_with(const double g[16], const double x[8])
{
    double kt = x[4], kr = x[5], kth = x[6], kph = x[7];
    double num = g[IX(1, 1)] * kr * kr + g[IX(3, 3)] * kph * kph + g[IX(2, 2)] * kth * kth +
                 2.0 * g[IX(0, 3)] * kt * kph;
    return num / (g[IX(0, 0)] * kt * kt);
}

double oracle_xi(double a, const double x[8])
{
    double g[16];
    oracle_metric(a, x[1], x[2], g);
    return xi_with(g, x);
}

double oracle_xi_jp(double a, double eps3, const double x[8])
{
    double g[16];
    oracle_metric_jp(a, eps3, x[1], x[2], g);
    return xi_with(g, x);
}

/* Remap of Sec. 2 eq. (3), keeping theta in [0, pi]. Returns 1 if applied. */
int oracle_remap(double x[8])
{
    if (x[2] > ORACLE_PI) {
        x[2] = 2.0 * ORACLE_PI - x[2];
        x[3] = x[3] + ORACLE_PI;
        x[6] = -x[6];
        return 1;
    }
    if (x[2] < 0.0) {
        x[2] = -x[2];
        x[3] = x[3] - ORACLE_PI;
        x[6] = -x[6];
        return 1;
    }
    return 0;
}

/* One accepted step of the production scheme of Sec. 2: a classical RK4
 * step of size h from eq. (2); if the result violates the null condition,
 * |xi + 1| > epsilon (eq. 4), the step is re-integrated from the same start
 * with one forward-Euler step of size h / 9; then the remap of eq. (3).
 * Returns a bit set (1: Euler fallback, 2: remap) or -1 if h is not a
 * positive finite number (state left unchanged). */
int oracle_step(const oracle_params *p, double a, double x[8], double *h_used)
{
    double rbh = oracle_horizon(a);
    double h = oracle_step_size(rbh, p->step_frac, x);
    if (h_used) *h_used = h;
    if (!(h > 0.0 && h < INFINITY)) return -1;

    double k1[8], k2[8], k3[8], k4[8], y[8], xn[8];
    rhs_of(p, a, x, k1);
    for (int i = 0; i < 8; ++i) y[i] = x[i] + 0.5 * h * k1[i];
    rhs_of(p, a, y, k2);
    for (int i = 0; i < 8; ++i) y[i] = x[i] + 0.5 * h * k2[i];
    rhs_of(p, a, y, k3);
    for (int i = 0; i < 8; ++i) y[i] = x[i] + h * k3[i];
    rhs_of(p, a, y, k4);
    for (int i = 0; i < 8; ++i)
        xn[i] = x[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);

    int flags = 0;
    if (p->pole_mode == 0) {
        /* production scheme: re-integrate with Euler at h / euler_div when
         * the step violates the null condition, eq. (4) */
        double gn[16];
        metric_of(p, a, xn[1], xn[2], gn);
        double xi = xi_with(gn, xn);
        if (fabs(xi + 1.0) > p->xi_eps) {
            double he = h / p->euler_div;
            for (int i = 0; i < 8; ++i) xn[i] = x[i] + he * k1[i];
            flags |= 1;
        }
    } else if (p->pole_mode == 1) {
        /* earlier scheme: a step whose end lies across a pole is replaced by
         * a forward Euler step of the same size */
        if (xn[2] < 0.0 || xn[2] > ORACLE_PI) {
            for (int i = 0; i < 8; ++i) xn[i] = x[i] + h * k1[i];
            flags |= 1;
        }
    }
    if (oracle_remap(xn)) flags |= 2;
    memcpy(x, xn, sizeof xn);
    return flags;
}

/* Conserved quantities of the photon's physical momentum p = -k:
 * energy E = -p_t, axial angular momentum L = p_phi and Carter's constant
 * Q = p_theta^2 + cos^2 theta (L^2 / sin^2 theta - a^2 E^2) (Sec. 1). */
static void conserved_with(double a, const double g[16], const double x[8], double out[3])
{
    double p[4] = {-x[4], -x[5], -x[6], -x[7]};
    double pl[4];
    for (int mu = 0; mu < 4; ++mu) {
        pl[mu] = 0.0;
        for (int nu = 0; nu < 4; ++nu) pl[mu] += g[IX(mu, nu)] * p[nu];
    }
    double E = -pl[0], L = pl[3];
    double s = sin(x[2]), c = cos(x[2]);
    out[0] = E;
    out[1] = L;
    out[2] = pl[2] * pl[2] + c * c * (L * L / (s * s) - a * a * E * E);
}

void oracle_conserved(double a, const double x[8], double out[3])
{
    double g[16];
    oracle_metric(a, x[1], x[2], g);
    conserved_with(a, g, x, out);
}

/* E and L_z in the deformed metric (still constants of motion); the third
 * entry is the Kerr expression for Q with this metric's p_theta, which is not
 * conserved when eps3 != 0. */
void oracle_conserved_jp(double a, double eps3, const double x[8], double out[3])
{
    double g[16];
    oracle_metric_jp(a, eps3, x[1], x[2], g);
    conserved_with(a, g, x, out);
}

/* Redshift factor g = 1 / (u^t (1 - Omega L/E)) of light emitted at radius rc
 * by gas on a prograde Keplerian circular orbit, Omega = 1/(rc^{3/2} + a),
 * received by a static observer at infinity. */
double oracle_disk_redshift(double a, double rc, double E, double L)
{
    double g[16];
    oracle_metric(a, rc, 0.5 * ORACLE_PI, g);
    double om = 1.0 / (pow(rc, 1.5) + a);
    double ut = 1.0 / sqrt(-(g[IX(0, 0)] + 2.0 * om * g[IX(0, 3)] + om * om * g[IX(3, 3)]));
    return 1.0 / (ut * (1.0 - om * L / E));
}

static int all_finite(const double x[8])
{
    for (int i = 0; i < 8; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

/* Status after an accepted step, tested in this order: non-finite state,
 * capture inside r_bh (1 + eps) (the horizon stop of Sec. 2), escape beyond
 * r_escape moving outward, step cap. */
static int classify_after_step(const oracle_params *p, double rcap, const double x[8], int32_t steps)
{
    if (!all_finite(x)) return ORACLE_NONFINITE;
    if (x[1] < rcap) return ORACLE_CAPTURED;
    if (x[1] > p->r_escape && x[5] > 0.0) return ORACLE_ESCAPED;
    if (steps >= p->max_steps) return ORACLE_UNFINISHED;
    return ORACLE_RUNNING;
}

/* First crossing of the equatorial plane between x_prev and x (theta through
 * pi/2), located by linear interpolation in theta; recorded when the crossing
 * radius lies in [rmin, rmax]. Returns 1 when recorded. */
static int disk_crossing(double a, double rmin, double rmax, const double *xp, const double *x,
                         double disk[3])
{
    const double half_pi = 0.5 * ORACLE_PI;
    if (!((xp[2] - half_pi) * (x[2] - half_pi) < 0.0)) return 0;
    double f = (half_pi - xp[2]) / (x[2] - xp[2]);
    double rc = xp[1] + f * (x[1] - xp[1]);
    double phc = xp[3] + f * (x[3] - xp[3]);
    if (!(rc >= rmin && rc <= rmax)) return 0;
    double cq[3];
    oracle_conserved(a, x, cq);
    disk[0] = rc;
    disk[1] = phc;
    disk[2] = oracle_disk_redshift(a, rc, cq[0], cq[1]);
    return 1;
}

/* Integrate one photon from its current state until it is captured, escapes,
 * turns non-finite or reaches max_steps. The state x is the last accepted
 * state on return. mark (optional) receives the last accepted state with
 * r >= 2 r_bh before the photon last fell below 2 r_bh (all zero if it never
 * did): where a captured photon's state is compared, since its components
 * in Boyer-Lindquist coordinates diverge at the horizon. */
int oracle_trace_mark(const oracle_params *p, double a, double x[8], int32_t *steps,
                      int32_t *n_euler, int32_t *n_remap, double disk[3], double mark[8])
{
    double rcap = oracle_horizon(a) * (1.0 + p->horizon_eps);
    double rmark = 2.0 * oracle_horizon(a);
    double rmin = p->disk_rmin < 0.0 ? oracle_r_isco(a) : p->disk_rmin;
    int32_t s = 0, ne = 0, nr = 0;
    int hit = 0;
    if (disk) disk[0] = disk[1] = disk[2] = 0.0;
    if (mark) memset(mark, 0, 8 * sizeof(double));

    int status = ORACLE_RUNNING;
    while (status == ORACLE_RUNNING) {
        double xp[8];
        memcpy(xp, x, sizeof xp);
        int fl = oracle_step(p, a, x, NULL);
        if (fl < 0) {
            status = ORACLE_NONFINITE;
            break;
        }
        ne += fl & 1;
        nr += (fl >> 1) & 1;
        ++s;
        if (p->record_disk && disk && !hit) hit = disk_crossing(a, rmin, p->disk_rmax, xp, x, disk);
        if (mark && xp[1] >= rmark && x[1] < rmark) memcpy(mark, xp, 8 * sizeof(double));
        status = classify_after_step(p, rcap, x, s);
    }
    if (steps) *steps = s;
    if (n_euler) *n_euler = ne;
    if (n_remap) *n_remap = nr;
    return status;
}

int oracle_trace(const oracle_params *p, double a, double x[8], int32_t *steps,
                 int32_t *n_euler, int32_t *n_remap, double disk[3])
{
    return oracle_trace_mark(p, a, x, steps, n_euler, n_remap, disk, NULL);
}

/* Same loop, recording every accepted state (path[i*8..]) and the step's
 * flags (bit 0 Euler, bit 1 remap) for up to max_pts steps. */
int oracle_trace_path(const oracle_params *p, double a, double x[8], int32_t max_pts,
                      double *path, int32_t *flags, int32_t *n_pts)
{
    double rcap = oracle_horizon(a) * (1.0 + p->horizon_eps);
    int32_t s = 0;
    int status = ORACLE_RUNNING;
    while (status == ORACLE_RUNNING) {
        int fl = oracle_step(p, a, x, NULL);
        if (fl < 0) {
            status = ORACLE_NONFINITE;
            break;
        }
        if (s < max_pts) {
            memcpy(path + (int64_t)s * 8, x, 8 * sizeof(double));
            flags[s] = fl;
        }
        ++s;
        status = classify_after_step(p, rcap, x, s);
    }
    *n_pts = s < max_pts ? s : max_pts;
    return status;
}

/* Batch driver: photon i starts from x[i*8..] with spin a[i]; the final state
 * overwrites x. OpenMP over photons; they never interact (Sec. 1, Sec. 2). */
void oracle_run(const oracle_params *p, int64_t n, const double *a, double *x,
                int32_t *status, int32_t *steps, int32_t *n_euler, int32_t *n_remap,
                double *disk, double *mark, int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int32_t s, ne, nr;
        status[i] = oracle_trace_mark(p, a[i], x + i * 8, &s, &ne, &nr, disk ? disk + i * 3 : NULL,
                                      mark ? mark + i * 8 : NULL);
        steps[i] = s;
        if (n_euler) n_euler[i] = ne;
        if (n_remap) n_remap[i] = nr;
    }
}
