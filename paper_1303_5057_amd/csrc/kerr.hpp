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
#include <type_traits>

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

// True when p holds on some lane of the wave (on the host: p). Branching on
// it costs a wave one scalar branch; a per-lane branch also saves, masks
// and restores the execution mask, and a wave alone on its SIMD waits tens
// of cycles for each, so rare cases are tested with any_lane first.
GRAY_HD bool any_lane(bool p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_ballot_w64(p) != 0ull;
#else
    return p;
#endif
}

// ------------------------------------------------------------ FP64 primitives
// Reciprocal: the hardware estimate (relative error below 2^-24, measured)
// refined by one third-order step, y <- y + y (e + e^2) with e = 1 - x y,
// which leaves an error of order e^3 before the final rounding (on 10^6
// random x in 1e-4 .. 1e7 it equalled the correctly rounded 1/x every time,
// as two Newton-Raphson steps do, with one instruction less). No
// denormals; 0 and inf give non-finite results.
GRAY_HD double rcp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, fma(e, e, e), y);
#else
    return 1.0 / x;
#endif
}

GRAY_HD double quot(double a, double b) { return a * rcp(b); }

// Two Horner chains in z evaluated side by side:
//   ps = (..((s[0] z + s[1]) z + s[2]) z ..) + s[NS-1]
//   pc = (..((c[0] z + c[1]) z + c[2]) z ..) + c[NC-1]
// On the device each step is one VOP3 v_fma_f64 whose addend, a coefficient
// held in a scalar register pair, it does not overwrite (the leading
// coefficient sits in vector registers: an instruction reads at most one
// scalar source). (Written as fma(),
// the compiler selects the two-address v_fmac_f64, whose accumulator is the
// addend, and so copies every loop-invariant coefficient into it first: one
// extra move per step; and coefficients kept in vector registers cost 34 of
// them per lane for the whole loop.) One asm statement holds both chains,
// interleaved, so no wait states are inserted between them; the steps are
// dependent plain FP64 FMAs.
#if defined(__HIP_DEVICE_COMPILE__)
#define GRAY_HORNER_STEP(acc, k) "v_fma_f64 %" #acc ", %2, %" #acc ", %" #k "\n\t"
#endif

// The coefficients are asm operands of constraint K: "s" keeps them in
// scalar registers (the FP64 integrator, where 34 vector registers per lane
// decide how many waves fit on a SIMD), "v" in vector registers (kernels
// whose scalar registers are the scarcer resource).
#if defined(__HIP_DEVICE_COMPILE__)
#define GRAY_SINCOS_SMALL_ASM(K)                                                         \
    asm("v_fma_f64 %0, %2, %3, %4\n\t"                                                  \
        "v_fma_f64 %1, %2, %7, %8\n\t"                                                  \
        GRAY_HORNER_STEP(0, 5) GRAY_HORNER_STEP(1, 9) GRAY_HORNER_STEP(0, 6)             \
        GRAY_HORNER_STEP(1, 10)                                                          \
        : "=&v"(ps), "=&v"(pc)                                                           \
        : "v"(z), "v"(S0), K(S1), K(S2), K(S3), "v"(C0), K(C1), K(C2), K(C3))
#define GRAY_SINCOS_FULL_ASM(K)                                                          \
    asm("v_fma_f64 %0, %2, %3, %4\n\t"                                                  \
        "v_fma_f64 %1, %2, %11, %12\n\t"                                                \
        GRAY_HORNER_STEP(0, 5) GRAY_HORNER_STEP(1, 13) GRAY_HORNER_STEP(0, 6)            \
        GRAY_HORNER_STEP(1, 14) GRAY_HORNER_STEP(0, 7) GRAY_HORNER_STEP(1, 15)           \
        GRAY_HORNER_STEP(0, 8) GRAY_HORNER_STEP(1, 16) GRAY_HORNER_STEP(0, 9)            \
        GRAY_HORNER_STEP(1, 17) GRAY_HORNER_STEP(0, 10) GRAY_HORNER_STEP(1, 18)          \
        GRAY_HORNER_STEP(1, 19)                                                          \
        : "=&v"(ps), "=&v"(pc)                                                           \
        : "v"(z), "v"(S0), K(S1), K(S2), K(S3), K(S4), K(S5), K(S6), K(S7), "v"(C0),     \
          K(C1), K(C2), K(C3), K(C4), K(C5), K(C6), K(C7), K(C8))
#endif

// sin and cos of a small angle, |d| <= 1/16, from their Taylor series (sin
// to d^9, cos to d^8: truncation below 3e-19). The stage offsets of a step
// obey |d| <= Delta of eq. (2) to first order, so this covers them.
template <bool SGPR = true>
GRAY_HD void sincos_small(double d, double &sd, double &cd)
{
    const double z = d * d;
    constexpr double S0 = 2.755731922398589e-06, S1 = -1.984126984126984e-04,
                     S2 = 8.333333333333333e-03, S3 = -1.6666666666666666e-01;
    constexpr double C0 = 2.48015873015873e-05, C1 = -1.388888888888889e-03,
                     C2 = 4.1666666666666664e-02, C3 = -0.5;
    double ps, pc;
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (SGPR) GRAY_SINCOS_SMALL_ASM("s");
    else GRAY_SINCOS_SMALL_ASM("v");
#else
    ps = fma(z, fma(z, fma(z, S0, S1), S2), S3);
    pc = fma(z, fma(z, fma(z, C0, C1), C2), C3);
#endif
    sd = fma(d * z, ps, d);
    cd = fma(z, pc, 1.0);
}

// sin and cos of a moderate angle (|x| << 2^20): Cody-Waite reduction by
// pi/2 with a two-term split of pi/2 (FMA keeps the first subtraction exact),
// then Taylor series on |r| <= pi/4 (sin to r^17, cos to r^18, truncation
// below 1e-19), then the quadrant.
template <bool SGPR = true>
GRAY_HD void sincos_full(double x, double &s, double &c)
{
    const double k = rint(x * 0.6366197723675814);
    double r = fma(-k, 1.5707963267948966, x);
    r = fma(-k, 6.123233995736766e-17, r);
    const double z = r * r;
    constexpr double S0 = 2.8114572543455206e-15, S1 = -7.647163731819816e-13,
                     S2 = 1.6059043836821613e-10, S3 = -2.505210838544172e-08,
                     S4 = 2.755731922398589e-06, S5 = -1.984126984126984e-04,
                     S6 = 8.333333333333333e-03, S7 = -1.6666666666666666e-01;
    constexpr double C0 = -1.5619206968586225e-16, C1 = 4.779477332387385e-14,
                     C2 = -1.1470745597729725e-11, C3 = 2.08767569878681e-09,
                     C4 = -2.755731922398589e-07, C5 = 2.48015873015873e-05,
                     C6 = -1.388888888888889e-03, C7 = 4.1666666666666664e-02, C8 = -0.5;
    double ps, pc;
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (SGPR) GRAY_SINCOS_FULL_ASM("s");
    else GRAY_SINCOS_FULL_ASM("v");
#else
    ps = S0;
    for (double sk : {S1, S2, S3, S4, S5, S6, S7}) ps = fma(z, ps, sk);
    pc = C0;
    for (double ck : {C1, C2, C3, C4, C5, C6, C7, C8}) pc = fma(z, pc, ck);
#endif
    const double sr = fma(r * z, ps, r);
    const double cr = fma(z, pc, 1.0);
    const int q = (int)k & 3;
    const double a = (q & 1) ? cr : sr;
    const double b = (q & 1) ? sr : cr;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

template <bool SGPR = true>
GRAY_HD void sin_cos(double x, double &s, double &c) { sincos_full<SGPR>(x, s, c); }

// sin and cos of th = th0 + d from those of th0 (angle addition with the
// small-angle series); the full evaluation where |d| > 1/16 (rare: the
// stage offsets obey |d| <= Delta to first order).
template <bool SGPR = true>
GRAY_HD void shift_sincos(double s0, double c0, double d, double th, double &s, double &c)
{
    double sd, cd;
    sincos_small<SGPR>(d, sd, cd);
    s = fma(s0, cd, c0 * sd);
    c = fma(c0, cd, -(s0 * sd));
    const bool wide = !(fabs(d) <= 0.0625);
    if (__builtin_expect(any_lane(wide), 0)) {
        double sf, cf;
        sincos_full<SGPR>(th, sf, cf);
        s = wide ? sf : s;
        c = wide ? cf : c;
    }
}

// ------------------------------------------------------------ FP32 primitives
// Reciprocal: the hardware v_rcp_f32 (about one ulp, denormals flushed).
GRAY_HD float rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

GRAY_HD float quot(float a, float b) { return a * rcp(b); }

// sin and cos of |d| <= 1/16 (sin to d^5, cos to d^4: truncation < 1e-10).
GRAY_HD void sincos_small(float d, float &sd, float &cd)
{
    const float z = d * d;
    sd = fma(d * z, fma(z, 0.008333333767950535f, -0.1666666716337204f), d);
    cd = fma(z, fma(z, 0.0416666679084301f, -0.5f), 1.0f);
}

// sin and cos of a moderate float angle x + lo (lo a low word below half an
// ulp of x, or 0): reduction of x by pi/2 with a two-term float split of
// pi/2, the low word added to the reduced argument (so an angle held as
// hi + lo keeps its digits next to pi), then Taylor series on |r| <= pi/4
// (sin to r^9, cos to r^10: truncation below 3e-9).
GRAY_HD void sincos_full_lo(float x, float lo, float &s, float &c)
{
    const float k = rintf(x * 0.6366197466850281f);
    float r = fma(-k, 1.5707963705062866f, x);
    r = fma(-k, -4.371138828673793e-08f, r);
    r = r + lo;
    const float z = r * r;
    float ps = fma(z, 2.7557318844628753e-06f, -0.00019841270113829523f);
    ps = fma(z, ps, 0.008333333767950535f);
    ps = fma(z, ps, -0.1666666716337204f);
    const float sr = fma(r * z, ps, r);
    float pc = fma(z, -2.755731998149713e-07f, 2.4801587642286904e-05f);
    pc = fma(z, pc, -0.0013888889225199819f);
    pc = fma(z, pc, 0.0416666679084301f);
    pc = fma(z, pc, -0.5f);
    const float cr = fma(z, pc, 1.0f);
    const int q = (int)k & 3;
    const float a = (q & 1) ? cr : sr;
    const float b = (q & 1) ? sr : cr;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

GRAY_HD void sincos_full(float x, float &s, float &c) { sincos_full_lo(x, 0.0f, s, c); }

GRAY_HD void sin_cos(float x, float &s, float &c) { sincos_full(x, s, c); }

GRAY_HD void shift_sincos(float s0, float c0, float d, float th, float &s, float &c)
{
    float sd, cd;
    sincos_small(d, sd, cd);
    s = fma(s0, cd, c0 * sd);
    c = fma(c0, cd, -(s0 * sd));
    const bool wide = !(fabsf(d) <= 0.0625f);
    if (__builtin_expect(any_lane(wide), 0)) {
        float sf, cf;
        sincos_full(th, sf, cf);
        s = wide ? sf : s;
        c = wide ? cf : c;
    }
}

// Spin-dependent constants of one photon's spacetime.
template <class T>
struct Spin {
    T a, a2;   // a, a^2
};

template <class T>
GRAY_HD Spin<T> make_spin(T a)
{
    Spin<T> B;
    B.a = a;
    B.a2 = a * a;
    return B;
}

// Geodesic acceleration given sin and cos of theta (see the file comment),
// written out operation by operation: one reciprocal of Sigma Delta sin gives
// 1/Sigma, 1/Delta and cot; every contraction is shaped into fused
// multiply-adds, and products that several terms share (w P, k^r k^th) are
// formed once. With rho^2 = r^2 + a^2 the identity rho^2 - a^2 sin^2 = Sigma
// gives the short forms used below:
//   X = (a k^t - rho^2 k^phi) / Sigma  = a P / Sigma - k^phi,
//   F - 2 q rho^2 = Delta (F = g_phph / sin^2), so that
//   F k^phi - 2 a q W P = Delta k^phi - 2 q rho^2 X   (W = rho^2 / Sigma) and
//   the k^phi^2 coefficient of A_th is -Delta,
//   (Delta / Sigma) (1/2) d_r g_rr = q - (r - 1) / Delta.
// At2 and Aph2 are half of the lowered components A_t and A_phi / sin^2;
// dk^r = -(Delta / Sigma) A_r is formed without A_r.
// Given Delta = r^2 - 2 r + a^2 (the float step passes it in factored form,
// (r - r_+)(r - r_-) with r - r_+ from the compensated state, which keeps its
// digits next to the horizon; Delta enters directly where the earlier forms
// took it as a difference of two larger terms).
template <class T>
GRAY_HD void accel_del(const Spin<T> &B, T r, T del, T s, T c, T kt, T kr, T kth, T kph, T &dkt, T &dkr,
                       T &dkth, T &dkph)
{
    const T a = B.a, a2 = B.a2;
    const T r2 = r * r;
    const T s2 = s * s;
    const T sc = s * c;
    const T sig = fma(a2, c * c, r2);
    const T rho2 = r2 + a2;
    const T sd = sig * del;
    const T i3 = rcp(sd * s);
    const T si3 = s * i3;
    const T isig = del * si3;
    const T idel = sig * si3;
    const T cot = c * (sd * i3);
    const T q = r * isig;                                    // r / Sigma
    const T q2 = q + q;
    const T w = fma(-q2, q, isig);                           // (Sigma - 2 r^2) / Sigma^2
    const T P = fma(-(a * s2), kph, kt);
    const T wP = w * P;
    const T X = fma(a * isig, P, -kph);
    const T kr2 = kr * kr, kth2 = kth * kth, kph2 = kph * kph;
    const T krth = kr * kth;
    const T aq2 = a * q2;                                    // 2 a r / Sigma
    const T r_2 = r + r;

    // A_t / 2
    const T At2 = fma(wP, kr, ((aq2 * sc) * kth) * X);
    // A_phi / (2 sin^2)
    const T t1 = fma(-a, wP, r * kph);
    const T Aph2 = fma(kth * cot, fma(del, kph, -((q2 * rho2) * X)), kr * t1);
    // -A_r Delta / Sigma
    const T Tr = fma(r, fma(s2, kph2, kth2), wP * P);
    T mAr = fma(-fma(T(1) - r, idel, q), kr2, (del * isig) * Tr);
    mAr = fma((a2 * sc) * (isig + isig), krth, mAr);
    // A_theta = sin cos g + 2 r k^r k^theta
    T g = a2 * fma(idel, kr2, -kth2);
    g = fma(-del, kph2, g);
    g = fma(-(r_2 * X), X, g);
    const T Ath = fma(sc, g, r_2 * krth);

    const T F = fma(a2 * s2, q2, rho2);                      // g_phiphi / sin^2
    const T idel2 = idel + idel;
    dkt = fma(aq2 * s2, Aph2, F * At2) * idel2;
    dkr = mAr;
    dkth = -Ath * isig;
    dkph = fma(fma(T(2), q, T(-1)), Aph2, aq2 * At2) * idel2;
}

template <class T>
GRAY_HD void accel(const Spin<T> &B, T r, T s, T c, T kt, T kr, T kth, T kph, T &dkt, T &dkr,
                   T &dkth, T &dkph)
{
    const T del = fma(r, r - T(2), B.a2);
    accel_del<T>(B, r, del, s, c, kt, kr, kth, kph, dkt, dkr, dkth, dkph);
}

// f(y) of the geodesic equation given sin and cos of y.th, in the spacetime
// B describes (Spin<T>: Kerr; DeformedSpin: the deformed metric below).
template <class T, class SP>
GRAY_HD void deriv(const SP &B, const State<T> &y, T s, T c, State<T> &f)
{
    f.t = y.kt;
    f.r = y.kr;
    f.th = y.kth;
    f.ph = y.kph;
    accel(B, y.r, s, c, y.kt, y.kr, y.kth, y.kph, f.kt, f.kr, f.kth, f.kph);
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
    const T i2 = rcp(sig * del);
    const T q = r * (del * i2);
    Metric<T> g;
    g.tt = T(2) * q - T(1);
    g.tph = T(-2) * a * q * s2;
    g.rr = sig * (sig * i2);
    g.thth = sig;
    g.phph = fma(T(2) * a2 * s2, q, r * r + a2) * s2;
    return g;
}

// Null-condition test of eq. (4) at (r, theta) given sin/cos of theta, free
// of divisions: |xi + 1| > eps  <=>  |N + D| > eps |D| with N the numerator
// of xi and D = g_tt kt^2, both multiplied by Sigma Delta (a factor that
// changes neither side). N + D is then Sigma Delta g(k, k); writing the t-phi
// block as -(Delta / Sigma) P^2 + (sin^2 / Sigma) Y^2 with P = kt - a sin^2 kph
// and Y = a kt - rho^2 kph = a P - Sigma kph,
//   Sigma Delta g(k, k) = Sigma^2 kr^2 + Delta (Sigma^2 kth^2 + sin^2 Y^2) - Delta^2 P^2,
//   Sigma Delta g_tt    = (2 r - Sigma) Delta.
template <class T>
GRAY_HD bool xi_violated_del(T a, T a2, T r, T del, T s, T c, T kt, T kr, T kth, T kph, T eps)
{
    const T sig = fma(a2, c * c, r * r);
    const T P = fma(-(a * (s * s)), kph, kt);
    const T sY = s * fma(a, P, -(sig * kph));
    const T skth = sig * kth, skr = sig * kr, dP = del * P;
    const T gkk = fma(del, fma(skth, skth, sY * sY), fma(skr, skr, -(dP * dP)));
    const T den = ((r + r - sig) * del) * (kt * kt);
    return fabs(gkk) > eps * fabs(den);
}

template <class T>
GRAY_HD bool xi_violated_at(T a, T a2, T r, T s, T c, T kt, T kr, T kth, T kph, T eps)
{
    const T del = fma(r, r - T(2), a2);
    return xi_violated_del<T>(a, a2, r, del, s, c, kt, kr, kth, kph, eps);
}

template <class T>
GRAY_HD bool null_violated(const Spin<T> &B, T r, T s, T c, T kt, T kr, T kth, T kph, T eps)
{
    return xi_violated_at(B.a, B.a2, r, s, c, kt, kr, kth, kph, eps);
}

// ------------------------------------------------------- deformed Kerr metric
// A non-Kerr spacetime of the kind Sec. 1 gives as the reason to integrate
// the second-order geodesic equations (no Carter constant): the
// Johannsen-Psaltis deformation of Kerr with deviation function
// h = eps3 r / Sigma^2,
//   g_tt   = -(1 + h)(1 - 2 r / Sigma),   g_tphi = -2 a (r / Sigma) sin^2 (1 + h),
//   g_rr   = Sigma (1 + h) / (Delta + a^2 sin^2 h),   g_thth = Sigma,
//   g_phph = sin^2 (r^2 + a^2 + 2 a^2 (r / Sigma) sin^2) + h a^2 (Sigma + 2 r) sin^4 / Sigma,
// eps3 = 0 being Kerr. Its right-hand side is metric-generic: the metric is
// evaluated once per call on numbers that carry their r and theta
// derivatives (forward mode), and the lowered acceleration
//   A_mu = (k^r d_r + k^th d_th)(g_mu b) k^b - 1/2 d_mu(g_ab) k^a k^b
// (d_t = d_phi = 0) is raised with the inverse of the t-phi block.
struct DeformedSpin {
    double a, a2, eps3;
};

GRAY_HD DeformedSpin make_deformed(double a, double eps3) { return DeformedSpin{a, a * a, eps3}; }

// A value with its derivatives by r and by theta.
struct Dual2 {
    double v, r, t;
};
GRAY_HD Dual2 operator+(Dual2 x, Dual2 y) { return Dual2{x.v + y.v, x.r + y.r, x.t + y.t}; }
GRAY_HD Dual2 operator-(Dual2 x, Dual2 y) { return Dual2{x.v - y.v, x.r - y.r, x.t - y.t}; }
GRAY_HD Dual2 operator+(double k, Dual2 y) { return Dual2{k + y.v, y.r, y.t}; }
GRAY_HD Dual2 operator*(double k, Dual2 y) { return Dual2{k * y.v, k * y.r, k * y.t}; }
GRAY_HD Dual2 operator*(Dual2 x, Dual2 y)
{
    return Dual2{x.v * y.v, fma(x.r, y.v, x.v * y.r), fma(x.t, y.v, x.v * y.t)};
}
GRAY_HD Dual2 rcp(Dual2 x)
{
    const double y = rcp(x.v);
    const double m = -(y * y);
    return Dual2{y, x.r * m, x.t * m};
}

// The five metric components, on plain doubles or on Dual2 (one expression
// for both; only the operations defined for Dual2 are used).
template <class N>
struct MetricN {
    N tt, tph, rr, thth, phph;
};

template <class N>
GRAY_HD MetricN<N> deformed_metric(const DeformedSpin &B, N r, N s, N c)
{
    const N s2 = s * s;
    const N r2 = r * r;
    const N sig = r2 + B.a2 * (c * c);                 // Sigma
    const N isig = rcp(sig);
    const N q = r * isig;                              // r / Sigma
    const N h = B.eps3 * (q * isig);                   // eps3 r / Sigma^2
    const N h1 = 1.0 + h;
    const N del = B.a2 + (r2 - 2.0 * r);               // Delta
    MetricN<N> g;
    g.tt = h1 * (-1.0 + 2.0 * q);
    g.tph = (-2.0 * B.a) * ((q * s2) * h1);
    g.rr = (sig * h1) * rcp(del + B.a2 * (s2 * h));
    g.thth = sig;
    const N F = B.a2 + (r2 + (2.0 * B.a2) * (q * s2)); // r^2 + a^2 + 2 a^2 q sin^2
    g.phph = s2 * F + (B.a2 * h) * ((sig + 2.0 * r) * ((s2 * s2) * isig));
    return g;
}

GRAY_HD void accel(const DeformedSpin &B, double r, double s, double c, double kt, double kr, double kth,
                   double kph, double &dkt, double &dkr, double &dkth, double &dkph)
{
    const MetricN<Dual2> g = deformed_metric<Dual2>(B, Dual2{r, 1.0, 0.0}, Dual2{s, 0.0, c}, Dual2{c, 0.0, -s});
    // derivative along the motion, k^r d_r + k^th d_th
    const double Dtt = fma(kr, g.tt.r, kth * g.tt.t), Dtph = fma(kr, g.tph.r, kth * g.tph.t);
    const double Drr = fma(kr, g.rr.r, kth * g.rr.t), Dthth = fma(kr, g.thth.r, kth * g.thth.t);
    const double Dphph = fma(kr, g.phph.r, kth * g.phph.t);
    const double At = fma(Dtt, kt, Dtph * kph);
    const double Aph = fma(Dtph, kt, Dphph * kph);
    // d_r and d_theta of g_ab k^a k^b
    const double ktph2 = 2.0 * kt * kph, kt2 = kt * kt, kr2 = kr * kr, kth2 = kth * kth, kph2 = kph * kph;
    double Qr = g.tt.r * kt2;
    Qr = fma(g.tph.r, ktph2, Qr);
    Qr = fma(g.rr.r, kr2, Qr);
    Qr = fma(g.thth.r, kth2, Qr);
    Qr = fma(g.phph.r, kph2, Qr);
    double Qt = g.tt.t * kt2;
    Qt = fma(g.tph.t, ktph2, Qt);
    Qt = fma(g.rr.t, kr2, Qt);
    Qt = fma(g.thth.t, kth2, Qt);
    Qt = fma(g.phph.t, kph2, Qt);
    const double Ar = fma(-0.5, Qr, Drr * kr);
    const double Ath = fma(-0.5, Qt, Dthth * kth);
    // inverse of the t-phi block: g^tt = g_phph / D2, g^tph = -g_tph / D2,
    // g^phph = g_tt / D2 with D2 = g_tt g_phph - g_tph^2
    const double iD2 = rcp(fma(g.tt.v, g.phph.v, -(g.tph.v * g.tph.v)));
    dkt = -fma(g.phph.v, At, -(g.tph.v * Aph)) * iD2;
    dkph = -fma(g.tt.v, Aph, -(g.tph.v * At)) * iD2;
    dkr = -Ar * rcp(g.rr.v);
    dkth = -Ath * rcp(g.thth.v);
}

// Null-condition test of eq. (4) in the deformed metric: |xi + 1| > eps with
// xi the ratio of eq. (4), written |N + g_tt kt^2| > eps |g_tt kt^2|.
GRAY_HD bool null_violated(const DeformedSpin &B, double r, double s, double c, double kt, double kr,
                           double kth, double kph, double eps)
{
    const MetricN<double> g = deformed_metric<double>(B, r, s, c);
    const double den = (g.tt * kt) * kt;
    double num = g.rr * (kr * kr);
    num = fma(g.thth, kth * kth, num);
    num = fma(g.phph, kph * kph, num);
    num = fma(2.0 * g.tph, kt * kph, num);
    return fabs(num + den) > eps * fabs(den);
}

// Treatment of the polar axis (values of gray_pole_mode): the production
// null-condition monitor, the earlier Euler step on pole crossings, or none.
constexpr int kPoleMonitor = 0, kPoleEulerCrossing = 1, kPoleNone = 2;

// Integrator constants of one photon; SP describes the spacetime.
template <class T, class SP = Spin<T>>
struct StepConst {
    SP B;
    T rbh, step_frac, xi_eps;
    T euler_inv;   // 1 / (the Euler fallback's step divisor, 9 in Sec. 2)
};

// One accepted step of the production scheme (Sec. 2): classical RK4 with h
// from eq. (2); if the proposal violates the null condition, |xi + 1| > eps
// (eq. 4), one forward-Euler step of h / euler_div from the same start
// replaces it; then the remap of eq. (3). observe(start, end) sees every
// accepted step just before the state is overwritten (so a caller that needs
// the start state keeps no copy of it). PM selects the paper's earlier
// treatments instead: kPoleEulerCrossing replaces a step that ends across a
// pole by one forward-Euler step of the same h; kPoleNone keeps every RK4
// step. (s, c) = sin/cos(x.th) on entry and
// on exit (always recomputed from the final theta, so a step is a function of
// the stored state alone). Returns bit 0 = Euler fallback, bit 1 = remap, or
// -1 when h is not a positive finite number (state kept). With R48 (FP64
// only) the accepted state is rounded to 48-bit significands (round48)
// before its sin/cos and the null test are taken, so that it is exactly the
// float pair the compensated-float path stores.
// sin/cos helpers of the step template: the FP64 versions take the
// coefficient placement SC, other number types use their own overloads.
template <bool SC, class T>
GRAY_HD void step_shift_sincos(T s0, T c0, T d, T th, T &s, T &c)
{
    if constexpr (std::is_same<T, double>::value) shift_sincos<SC>(s0, c0, d, th, s, c);
    else shift_sincos(s0, c0, d, th, s, c);
}

template <bool SC, class T>
GRAY_HD void step_sin_cos(T x, T &s, T &c)
{
    if constexpr (std::is_same<T, double>::value) sin_cos<SC>(x, s, c);
    else sin_cos(x, s, c);
}

// x with the low five bits of its 53-bit significand cleared (rounded toward
// zero to 48 bits). Such a value is exactly hi + lo with hi = x rounded to
// float and lo = x - hi, both floats (for |x| above about 1e-30, where lo is
// not below the float range): the pair the compensated-float state stores.
// One integer AND on the low word.
GRAY_HD double round48(double x)
{
    return __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, x) & ~0x1Full);
}

template <class T>
GRAY_HD void round48_state(State<T> &x)
{
    x.t = round48(x.t); x.r = round48(x.r); x.th = round48(x.th); x.ph = round48(x.ph);
    x.kt = round48(x.kt); x.kr = round48(x.kr); x.kth = round48(x.kth); x.kph = round48(x.kph);
}

// Step observer that does nothing (see rk4_step).
struct NoObserver {
    template <class S>
    GRAY_HD void operator()(const S &, const S &) const {}
};

template <int PM = kPoleMonitor, bool SC = true, bool R48 = false, class T, class SP, class Obs = NoObserver>
GRAY_HD int rk4_step(const StepConst<T, SP> &K, State<T> &x, T &s, T &c, Obs &&observe = Obs())
{
    // eq. (2): h1 = Delta r / D1 with D1 = |k^r| + r (|k^th| + |k^ph|), and
    // h2 = (r - r_bh) / (2 |k^r|); h2 < h1 is decided without dividing.
    const T akr = fabs(x.kr);
    const T D1 = fma(x.r, fabs(x.kth) + fabs(x.kph), akr);
    const T n1 = K.step_frac * x.r;
    const T n2 = x.r - K.rbh;
    const T d2 = akr + akr;
    const bool second = (x.kr != T(0)) && (n2 * D1 < d2 * n1);
    const T h = quot(second ? n2 : n1, second ? d2 : D1);
    const bool hbad = !(h > T(0) && h < T(INFINITY));
    if (__builtin_expect(any_lane(hbad), 0))
        if (hbad) return -1;
    const T hh = T(0.5) * h;

    // The stage derivatives are summed as they come, k1 + 2 k2 + 2 k3 + k4
    // from left to right, so k2 and k3 need no registers once used; k1 stays
    // for the Euler fallback.
    State<T> k1, k, y, acc;
    T sy, cy;
    // (a stage's sin/cos from the angle addition formula with the offset
    // h k^th itself; the stage's theta is needed only where the offset is
    // too large for the series)
    deriv(K.B, x, s, c, k1);
    y = axpy(x, hh, k1);
    step_shift_sincos<SC>(s, c, hh * k1.th, y.th, sy, cy);
    deriv(K.B, y, sy, cy, k);
    acc = axpy(k1, T(2), k);
    y = axpy(x, hh, k);
    step_shift_sincos<SC>(s, c, hh * k.th, y.th, sy, cy);
    deriv(K.B, y, sy, cy, k);
    acc = axpy(acc, T(2), k);
    y = axpy(x, h, k);
    step_shift_sincos<SC>(s, c, h * k.th, y.th, sy, cy);
    deriv(K.B, y, sy, cy, k);

    const T h6 = h * T(1.0 / 6.0);
    State<T> xn;
#define GRAY_RK4(cmp) xn.cmp = fma(h6, acc.cmp + k.cmp, x.cmp)
    GRAY_RK4(t); GRAY_RK4(r); GRAY_RK4(th); GRAY_RK4(ph);
    GRAY_RK4(kt); GRAY_RK4(kr); GRAY_RK4(kth); GRAY_RK4(kph);
#undef GRAY_RK4
    if constexpr (R48) round48_state(xn);

    int flags = 0;
    step_sin_cos<SC>(xn.th, sy, cy);
    bool viol = false;
    if constexpr (PM == kPoleMonitor) {
        viol = null_violated(K.B, xn.r, sy, cy, xn.kt, xn.kr, xn.kth, xn.kph, K.xi_eps);
    } else if constexpr (PM == kPoleEulerCrossing) {
        viol = xn.th > T(kPi) || xn.th < T(0);
    }
    // The fallback and the remap, entered only when some lane needs one
    // (the remap and the new sin/cos by selects: a photon locked into the
    // fallback takes this block on most steps).
    if (__builtin_expect(any_lane(viol || xn.th > T(kPi) || xn.th < T(0)), 0)) {
        if (viol) {
            xn = axpy(x, PM == kPoleMonitor ? h * K.euler_inv : h, k1);
            flags |= 1;
        }
        const bool up = xn.th > T(kPi), down = xn.th < T(0);
        xn.th = up ? T(kTwoPi) - xn.th : (down ? -xn.th : xn.th);
        xn.ph = up ? xn.ph + T(kPi) : (down ? xn.ph - T(kPi) : xn.ph);
        xn.kth = (up || down) ? -xn.kth : xn.kth;
        flags |= (up || down) ? 2 : 0;
        if constexpr (R48) round48_state(xn);
        T sf, cf;
        step_sin_cos<SC>(xn.th, sf, cf);
        sy = flags ? sf : sy;
        cy = flags ? cf : cy;
    }
    observe(x, xn);
    x = xn;
    s = sy;
    c = cy;
    return flags;
}

// Error-free sum of two floats (Knuth's TwoSum): hi + lo == a + b exactly.
GRAY_HD void two_sum(float a, float b, float &hi, float &lo)
{
    const float t = a + b;
    const float z = t - a;
    lo = (a - (t - z)) + (b - z);
    hi = t;
}

// The null monitor of eq. (4) in float with a bound on its own rounding:
// returns 1 when |xi + 1| > eps holds (written |N + D| > eps |D| as in
// xi_violated_del, N the numerator of xi, D = g_tt kt^2, both times
// Sigma Delta), 0 when it fails, and -1 when the float evaluation cannot
// decide: | |N + D| - eps |D| | is within 32 float roundings of the sum of the
// magnitudes of the terms of N and D (they cancel to |xi + 1| |D| on a null
// ray, by orders of magnitude next to the horizon, so a fixed guard band
// would be either too wide far out or too narrow there).
GRAY_HD int xi_violated_guarded(float a, float a2, float r, float del, float s, float c, float kt, float kr,
                                float kth, float kph, float eps)
{
    const float s2 = s * s;
    const float r2 = r * r;
    const float sig = fma(a2, c * c, r2);
    const float sig2 = sig * sig;
    const float ar2 = (a + a) * r;
    const float phph = fma(ar2 * a, s2, (r2 + a2) * sig);
    const float t_th = sig2 * (kth * kth);
    const float t_ph = phph * (s2 * kph) * kph;
    const float t_x = -(ar2 + ar2) * (s2 * kt) * kph;
    const float t_r = sig2 * (kr * kr);
    const float num = fma(del, (t_th + t_ph) + t_x, t_r);
    const float den = ((r + r - sig) * del) * (kt * kt);
    const float mag = fma(fabsf(del), (fabsf(t_th) + fabsf(t_ph)) + fabsf(t_x), fabsf(t_r)) + fabsf(den);
    const float margin = fabsf(num + den) - eps * fabsf(den);
    if (!(fabsf(margin) > 1.9073486e-06f * mag)) return -1;   // 32 * 2^-24
    return margin > 0.0f ? 1 : 0;
}

// Horizon radii of one photon's spacetime for the float step: r_+ as a
// float pair (r_+ = rp_hi + rp_lo to about 1e-15) and r_- in float.
struct FloatHorizon {
    float rp_hi, rp_lo, rm;
};

GRAY_HD FloatHorizon make_float_horizon(double a)
{
    const double rp = 1.0 + sqrt(1.0 - a * a);
    FloatHorizon H;
    H.rp_hi = (float)rp;
    H.rp_lo = (float)(rp - (double)H.rp_hi);
    H.rm = (float)(2.0 - rp);
    return H;
}

// Error-free sum when |a| >= |b| (or a = 0): s + e == a + b exactly.
GRAY_HD void fast_two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    e = b - (s - a);
}

// pi as a float pair
constexpr float kPiHi = 3.14159274101257324f, kPiLo = -8.74227765734758577e-08f;

// One step of the production scheme (Sec. 2) in float arithmetic on the
// compensated state hi + lo, written to keep the digits that plain float
// loses: r - r_bh of eq. (2) and Delta = (r - r_+)(r - r_-) near the horizon
// are formed from hi + lo (and the stage offsets h k^r), sin and cos of the
// state's theta include its low word, and the stage angles are reached from
// them through the offsets h k^theta (never through a rounded float theta),
// which keeps cot and 1/sin^2 accurate next to the poles. The classical RK4
// increment is added with TwoSum; the null monitor of eq. (4) is evaluated in
// float on the proposal and a violation re-integrates with the forward-Euler
// step h / euler_div, also compensated; the remap of eq. (3) is applied to
// the float pair (theta compared with pi as a pair). Decisions are taken in
// float: the monitor's |xi + 1| is reproduced to about 1e-6 relative, so a
// decision can differ from the FP64 step's only for a proposal within that of
// epsilon, and a proposal whose monitor float cannot decide (its rounding
// bound, xi_violated_guarded) or that is not finite returns -2 with the
// state kept, for the caller to take the step in FP64. Returns the flags of
// rk4_step, -1 when h is not a positive finite number, or -2 (state kept in
// both cases). (s, c) = sin/cos(hi.th + lo.th) on entry and exit.
GRAY_HD int rk4_step_f32(const StepConst<float> &K, const FloatHorizon &H, State<float> &hi, State<float> &lo,
                         float &s, float &c)
{
    const float dr = (hi.r - H.rp_hi) + (lo.r - H.rp_lo);   // r - r_bh
    const float akr = fabsf(hi.kr);
    const float D1 = fma(hi.r, fabsf(hi.kth) + fabsf(hi.kph), akr);
    const float n1 = K.step_frac * hi.r;
    const float d2 = akr + akr;
    const bool second = (hi.kr != 0.0f) && (dr * D1 < d2 * n1);
    const float h = second ? quot(dr, d2) : quot(n1, D1);
    const bool hbad = !(h > 0.0f && h < INFINITY);
    if (__builtin_expect(any_lane(hbad), 0))
        if (hbad) return -1;
    const float hh = 0.5f * h;

    // stage derivatives summed as they come; k1 stays for the Euler fallback
    State<float> k1, k, y, acc;
    float sy, cy;
    auto stage = [&](const State<float> &ks, float hs) {
        y = axpy(hi, hs, ks);
        const float ydr = fma(hs, ks.r, dr);
        shift_sincos(s, c, hs * ks.th, y.th, sy, cy);
        k.t = y.kt;
        k.r = y.kr;
        k.th = y.kth;
        k.ph = y.kph;
        accel_del<float>(K.B, y.r, ydr * (y.r - H.rm), sy, cy, y.kt, y.kr, y.kth, y.kph, k.kt, k.kr, k.kth, k.kph);
    };
    k1.t = hi.kt;
    k1.r = hi.kr;
    k1.th = hi.kth;
    k1.ph = hi.kph;
    accel_del<float>(K.B, hi.r, dr * (hi.r - H.rm), s, c, hi.kt, hi.kr, hi.kth, hi.kph, k1.kt, k1.kr, k1.kth, k1.kph);
    stage(k1, hh);
    acc = axpy(k1, 2.0f, k);
    stage(k, hh);
    acc = axpy(acc, 2.0f, k);
    stage(k, h);

    const float h6 = h * (1.0f / 6.0f);
    State<float> nh, nl;
#define GRAY_F32(cmp) two_sum(hi.cmp, fma(h6, acc.cmp + k.cmp, lo.cmp), nh.cmp, nl.cmp)
    GRAY_F32(t); GRAY_F32(r); GRAY_F32(th); GRAY_F32(ph);
    GRAY_F32(kt); GRAY_F32(kr); GRAY_F32(kth); GRAY_F32(kph);
#undef GRAY_F32
    int flags = 0;
    sincos_full_lo(nh.th, nl.th, sy, cy);
    const float ndr = (nh.r - H.rp_hi) + (nl.r - H.rp_lo);
    const int vm = xi_violated_guarded(K.B.a, K.B.a2, nh.r, ndr * (nh.r - H.rm), sy, cy, nh.kt, nh.kr, nh.kth,
                                       nh.kph, K.xi_eps);
    // a decision float cannot take is left to the FP64 step (state kept)
    const bool undecided = vm < 0 || !(__builtin_isfinite(nh.t) && __builtin_isfinite(nh.r) && __builtin_isfinite(nh.th) && __builtin_isfinite(nh.ph) &&
                                       __builtin_isfinite(nh.kt) && __builtin_isfinite(nh.kr) && __builtin_isfinite(nh.kth) && __builtin_isfinite(nh.kph));
    if (__builtin_expect(any_lane(undecided), 0))
        if (undecided) return -2;
    const bool viol = vm > 0;
    // theta - pi of the proposal as one float (exact difference next to pi)
    bool up = (nh.th - kPiHi) + (nl.th - kPiLo) > 0.0f;
    bool down = nh.th < 0.0f || (nh.th == 0.0f && nl.th < 0.0f);
    if (__builtin_expect(any_lane(viol || up || down), 0)) {
        if (viol) {
            const float he = h * K.euler_inv;
#define GRAY_F32E(cmp) two_sum(hi.cmp, fma(he, k1.cmp, lo.cmp), nh.cmp, nl.cmp)
            GRAY_F32E(t); GRAY_F32E(r); GRAY_F32E(th); GRAY_F32E(ph);
            GRAY_F32E(kt); GRAY_F32E(kr); GRAY_F32E(kth); GRAY_F32E(kph);
#undef GRAY_F32E
            flags |= 1;
            up = (nh.th - kPiHi) + (nl.th - kPiLo) > 0.0f;
            down = nh.th < 0.0f || (nh.th == 0.0f && nl.th < 0.0f);
        }
        if (up) {
            // theta -> 2 pi - theta = pi - (theta - pi); phi -> phi + pi
            const float d = (nh.th - kPiHi) + (nl.th - kPiLo);
            two_sum(kPiHi, kPiLo - d, nh.th, nl.th);
        } else if (down) {
            nh.th = -nh.th;
            nl.th = -nl.th;
        }
        if (up || down) {
            const float sg = up ? 1.0f : -1.0f;
            float ps, pe;
            two_sum(nh.ph, sg * kPiHi, ps, pe);
            fast_two_sum(ps, pe + (nl.ph + sg * kPiLo), nh.ph, nl.ph);
            nh.kth = -nh.kth;
            nl.kth = -nl.kth;
            flags |= 2;
        }
        float sf, cf;
        sincos_full_lo(nh.th, nl.th, sf, cf);
        sy = flags ? sf : sy;
        cy = flags ? cf : cy;
    }
    hi = nh;
    lo = nl;
    s = sy;
    c = cy;
    return flags;
}

// Initial state of the ray through image-plane point (alpha, beta) of an
// observer at distance D and inclination incl (flat plane-parallel screen,
// ray traced backwards: k = -p, p^t > 0 from the null condition).
// Metric components at (r, theta) of the camera's spacetime: Kerr, or the
// deformed metric when `deformed` (deviation eps3).
GRAY_HD Metric<double> metric_of(double a, double eps3, bool deformed, double r, double s, double c)
{
    if (!deformed) return metric(a, a * a, r, s, c);
    const MetricN<double> d = deformed_metric<double>(make_deformed(a, eps3), r, s, c);
    Metric<double> g;
    g.tt = d.tt;
    g.tph = d.tph;
    g.rr = d.rr;
    g.thth = d.thth;
    g.phph = d.phph;
    return g;
}

GRAY_HD void camera_state(double a, double D, double incl, double alpha, double beta, State<double> &x,
                          double eps3 = 0.0, bool deformed = false)
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
    const Metric<double> g = metric_of(a, eps3, deformed, r0, s0, c0);
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

// E = -p_t, L = p_phi, Q = p_th^2 + cos^2 (L^2 / sin^2 - a^2 E^2) of p = -k,
// given s, c = sin, cos of x.th.
GRAY_HD void conserved_g(const Metric<double> &g, double a, const State<double> &x, double s, double c, double &E,
                         double &L, double &Q)
{
    E = g.tt * x.kt + g.tph * x.kph;
    L = -(g.tph * x.kt + g.phph * x.kph);
    const double pth = -g.thth * x.kth;
    Q = pth * pth + c * c * (L * L / (s * s) - a * a * E * E);
}

GRAY_HD void conserved_sc(double a, const State<double> &x, double s, double c, double &E, double &L, double &Q)
{
    conserved_g(metric(a, a * a, x.r, s, c), a, x, s, c, E, L, Q);
}

GRAY_HD void conserved(double a, const State<double> &x, double &E, double &L, double &Q)
{
    double s, c;
    sincos(x.th, &s, &c);
    conserved_sc(a, x, s, c, E, L, Q);
}

// E and L_z in the camera's spacetime; Q is the Kerr expression, a constant
// of motion only in Kerr (eps3 = 0 or not deformed).
GRAY_HD void conserved_in(double a, double eps3, bool deformed, const State<double> &x, double &E, double &L,
                          double &Q)
{
    double s, c;
    sincos(x.th, &s, &c);
    conserved_g(metric_of(a, eps3, deformed, x.r, s, c), a, x, s, c, E, L, Q);
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
