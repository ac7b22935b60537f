// kerr.hpp -- Kerr geodesic right-hand side, camera and diagnostics for the
// GPU path (gfx950). Boyer-Lindquist coordinates, G = c = M = 1.
//
// The acceleration dk^mu/dl = -Gamma^mu_{ab} k^a k^b (the second-order
// geodesic equation integrated by Chan, Psaltis & Ozel 2013, Sec. 2) is
// evaluated in lowered form: A_mu = Gamma_{mu ab} k^a k^b
//   = k^r d_r(g_{mu b} k^b) + k^th d_th(g_{mu b} k^b) - 1/2 d_mu(g_{ab}) k^a k^b,
// then raised with the closed-form inverse metric. With
//   Sigma = r^2 + a^2 cos^2, Delta = r^2 - 2r + a^2, q = r / Sigma,
//   w = d_r q = 1/Sigma - 2 q^2, W = (r^2 + a^2) / Sigma,
//   F = g_phph / sin^2 = r^2 + a^2 + 2 a^2 q sin^2, P = k^t - a sin^2 k^phi,
// the four components collapse to
//   A_t          = 2 w k^r P + 4 a q sc k^th (a k^t / Sigma - W k^phi)
//   A_phi/sin^2  = k^r (2 r k^phi - 2 a w P)
//                  + k^th (2 F cot k^phi - 4 a q W (cot k^t - a sc k^phi))
//   A_r          = 1/2 d_r g_rr (k^r)^2 - 2 a^2 sc k^r k^th / Delta
//                  - r ((k^th)^2 + sin^2 (k^phi)^2) - w P^2
//   A_th         = 2 r k^r k^th + sc [a^2 ((k^r)^2 / Delta - (k^th)^2) - F (k^phi)^2
//                  - 2 q (a^2 (k^t)^2 / Sigma - 2 a W k^t k^phi + a^2 sin^2 W (k^phi)^2)]
// (sc = sin cos, cot = cos / sin), and
//   dk^t = (F A_t + 2 a q sin^2 A_phi/sin^2) / Delta,   dk^r = -A_r Delta / Sigma,
//   dk^th = -A_th / Sigma,   dk^phi = ((2q - 1) A_phi/sin^2 + 2 a q A_t) / Delta.
// The sin^2 of the t-phi block determinant cancels everywhere except the
// genuine 1/sin coordinate singularity in dk^phi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gray {

#define GRAY_HD __host__ __device__ __forceinline__

template <class T>
struct State {
    T t, r, th, ph, kt, kr, kth, kph;
};

template <class T>
GRAY_HD T get(const State<T> &s, int c)
{
    switch (c) {
    case 0: return s.t;
    case 1: return s.r;
    case 2: return s.th;
    case 3: return s.ph;
    case 4: return s.kt;
    case 5: return s.kr;
    case 6: return s.kth;
    default: return s.kph;
    }
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * 3.14159265358979323846;
constexpr double kHalfPi = 0.5 * 3.14159265358979323846;

// Geodesic acceleration given sin and cos of theta (see the file comment).
template <class T>
GRAY_HD void accel(T a, T a2, T r, T s, T c, T kt, T kr, T kth, T kph, T &dkt, T &dkr, T &dkth,
                   T &dkph)
{
    const T two = T(2);
    const T r2 = r * r;
    const T s2 = s * s;
    const T sc = s * c;
    const T sig = fma(a2, c * c, r2);
    const T del = fma(r, r - two, a2);
    const T rho2 = r2 + a2;
    const T isig = T(1) / sig;
    const T idel = T(1) / del;
    const T cot = c / s;
    const T q = r * isig;
    const T w = isig - two * q * q;
    const T W = rho2 * isig;
    const T F = fma(two * a2 * s2, q, rho2);
    const T grr = sig * idel;
    const T drgrr = idel * (two * r - grr * (two * r - two));
    const T P = kt - a * s2 * kph;

    const T At = two * w * kr * P + T(4) * a * q * sc * kth * (a * isig * kt - W * kph);
    const T Aph = kr * (two * r * kph - two * a * w * P) +
                  kth * (two * F * cot * kph - T(4) * a * q * W * (cot * kt - a * sc * kph));
    const T Ar = T(0.5) * drgrr * kr * kr - two * a2 * sc * idel * kr * kth -
                 r * (kth * kth + s2 * kph * kph) - w * P * P;
    const T Ath = two * r * kr * kth +
                  sc * (a2 * (idel * kr * kr - kth * kth) - F * kph * kph -
                        two * q * (a2 * isig * kt * kt - two * a * W * kt * kph + a2 * s2 * W * kph * kph));

    dkt = (F * At + two * a * q * s2 * Aph) * idel;
    dkr = -Ar * del * isig;
    dkth = -Ath * isig;
    dkph = ((two * q - T(1)) * Aph + two * a * q * At) * idel;
}

// sin and cos of an angle; overloaded per arithmetic type.
GRAY_HD void sin_cos(double x, double &s, double &c) { sincos(x, &s, &c); }

template <class T>
GRAY_HD void deriv(T a, T a2, const State<T> &y, State<T> &f)
{
    T s, c;
    sin_cos(y.th, s, c);
    f.t = y.kt;
    f.r = y.kr;
    f.th = y.kth;
    f.ph = y.kph;
    accel(a, a2, y.r, s, c, y.kt, y.kr, y.kth, y.kph, f.kt, f.kr, f.kth, f.kph);
}

template <class T>
GRAY_HD State<T> axpy(const State<T> &x, T h, const State<T> &k)
{
    State<T> y;
    y.t = fma(h, k.t, x.t);
    y.r = fma(h, k.r, x.r);
    y.th = fma(h, k.th, x.th);
    y.ph = fma(h, k.ph, x.ph);
    y.kt = fma(h, k.kt, x.kt);
    y.kr = fma(h, k.kr, x.kr);
    y.kth = fma(h, k.kth, x.kth);
    y.kph = fma(h, k.kph, x.kph);
    return y;
}

// Covariant metric components (g_tt, g_tphi, g_rr, g_thth, g_phph).
template <class T>
struct Metric {
    T tt, tph, rr, thth, phph;
};

template <class T>
GRAY_HD Metric<T> metric(T a, T a2, T r, T s, T c)
{
    const T s2 = s * s;
    const T sig = fma(a2, c * c, r * r);
    const T del = fma(r, r - T(2), a2);
    const T q = r / sig;
    Metric<T> g;
    g.tt = T(2) * q - T(1);
    g.tph = T(-2) * a * q * s2;
    g.rr = sig / del;
    g.thth = sig;
    g.phph = fma(T(2) * a2 * s2, q, r * r + a2) * s2;
    return g;
}

// Null-condition test of eq. (4) without the division:
// |xi + 1| > eps  <=>  |N + g_tt kt^2| > eps |g_tt kt^2|, N the numerator of xi.
template <class T>
GRAY_HD bool xi_violated(const Metric<T> &g, T kt, T kr, T kth, T kph, T eps)
{
    const T den = g.tt * kt * kt;
    const T num = g.rr * kr * kr + g.phph * kph * kph + g.thth * kth * kth + T(2) * g.tph * kt * kph;
    return fabs(num + den) > eps * fabs(den);
}

// Integrator constants of one photon.
template <class T>
struct StepConst {
    T a, a2, rbh, step_frac, xi_eps, euler_div;
};

// One accepted step of the production scheme (Sec. 2): classical RK4 with h
// from eq. (2); if the proposal violates the null condition, |xi + 1| > eps
// (eq. 4), one forward-Euler step of h / euler_div from the same start
// replaces it; then the remap of eq. (3). Returns bit 0 = Euler fallback,
// bit 1 = remap, or -1 when h is not a positive finite number (state kept).
template <class T>
GRAY_HD int rk4_step(const StepConst<T> &K, State<T> &x)
{
    const T h1 = K.step_frac / (fabs(x.kr) / x.r + fabs(x.kth) + fabs(x.kph));
    const T h2 = (x.kr != T(0)) ? (x.r - K.rbh) / (T(2) * fabs(x.kr)) : T(INFINITY);
    const T h = h2 < h1 ? h2 : h1;
    if (!(h > T(0) && h < T(INFINITY))) return -1;

    State<T> k1, k2, k3, k4;
    deriv(K.a, K.a2, x, k1);
    deriv(K.a, K.a2, axpy(x, T(0.5) * h, k1), k2);
    deriv(K.a, K.a2, axpy(x, T(0.5) * h, k2), k3);
    deriv(K.a, K.a2, axpy(x, h, k3), k4);

    const T h6 = h * T(1.0 / 6.0);
    State<T> xn;
#define GRAY_RK4(c) xn.c = fma(h6, k1.c + T(2) * (k2.c + k3.c) + k4.c, x.c)
    GRAY_RK4(t); GRAY_RK4(r); GRAY_RK4(th); GRAY_RK4(ph);
    GRAY_RK4(kt); GRAY_RK4(kr); GRAY_RK4(kth); GRAY_RK4(kph);
#undef GRAY_RK4

    int flags = 0;
    T s, c;
    sin_cos(xn.th, s, c);
    const Metric<T> g = metric(K.a, K.a2, xn.r, s, c);
    if (xi_violated(g, xn.kt, xn.kr, xn.kth, xn.kph, K.xi_eps)) {
        xn = axpy(x, h / K.euler_div, k1);
        flags |= 1;
    }
    if (xn.th > T(kPi)) {
        xn.th = T(kTwoPi) - xn.th;
        xn.ph = xn.ph + T(kPi);
        xn.kth = -xn.kth;
        flags |= 2;
    } else if (xn.th < T(0)) {
        xn.th = -xn.th;
        xn.ph = xn.ph - T(kPi);
        xn.kth = -xn.kth;
        flags |= 2;
    }
    x = xn;
    return flags;
}

// Initial state of the ray through image-plane point (alpha, beta) of an
// observer at distance D and inclination incl (flat plane-parallel screen,
// ray traced backwards: k = -p, p^t > 0 from the null condition).
GRAY_HD void camera_state(double a, double D, double incl, double alpha, double beta, State<double> &x)
{
    double si, ci;
    sincos(incl, &si, &ci);
    const double X = D * si - beta * ci;
    const double Y = alpha;
    const double Z = fma(beta, si, D * ci);
    const double b2 = fma(alpha, alpha, beta * beta);
    const double r0sq = fma(D, D, b2);
    const double r0 = sqrt(r0sq);
    const double rho2 = fma(X, X, Y * Y);
    const double rho = sqrt(rho2);
    const double th0 = atan2(rho, Z);
    const double ph0 = atan2(Y, X);
    const double pr = D / r0;
    double pth = 0.0, pph = 0.0;
    if (rho > 0.0) {
        pth = (D * beta * si - b2 * ci) / (r0sq * rho);
        pph = -alpha * si / rho2;
    }
    double s0, c0;
    sincos(th0, &s0, &c0);
    const Metric<double> g = metric(a, a * a, r0, s0, c0);
    const double S = g.rr * pr * pr + g.thth * pth * pth + g.phph * pph * pph;
    const double B = g.tph * pph;
    const double pt = (-B - sqrt(B * B - g.tt * S)) / g.tt;
    x.t = 0.0;
    x.r = r0;
    x.th = th0;
    x.ph = ph0;
    x.kt = -pt;
    x.kr = -pr;
    x.kth = -pth;
    x.kph = -pph;
}

// E = -p_t, L = p_phi, Q = p_th^2 + cos^2 (L^2 / sin^2 - a^2 E^2) of p = -k.
GRAY_HD void conserved(double a, const State<double> &x, double &E, double &L, double &Q)
{
    double s, c;
    sincos(x.th, &s, &c);
    const Metric<double> g = metric(a, a * a, x.r, s, c);
    E = g.tt * x.kt + g.tph * x.kph;
    L = -(g.tph * x.kt + g.phph * x.kph);
    const double pth = -g.thth * x.kth;
    Q = pth * pth + c * c * (L * L / (s * s) - a * a * E * E);
}

// Redshift of light from a prograde Keplerian emitter at radius rc in the
// equatorial plane, seen by a static observer at infinity.
GRAY_HD double disk_redshift(double a, double rc, double E, double L)
{
    const Metric<double> g = metric(a, a * a, rc, 1.0, 0.0);
    const double om = 1.0 / (rc * sqrt(rc) + a);
    const double ut = 1.0 / sqrt(-(g.tt + 2.0 * om * g.tph + om * om * g.phph));
    return 1.0 / (ut * (1.0 - om * L / E));
}

GRAY_HD double horizon_radius(double a) { return 1.0 + sqrt(1.0 - a * a); }

// Prograde ISCO radius (Bardeen, Press & Teukolsky 1972).
inline double isco_radius(double a)
{
    const double z1 = 1.0 + cbrt(1.0 - a * a) * (cbrt(1.0 + a) + cbrt(1.0 - a));
    const double z2 = sqrt(3.0 * a * a + z1 * z1);
    return 3.0 + z2 - sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

} // namespace gray
