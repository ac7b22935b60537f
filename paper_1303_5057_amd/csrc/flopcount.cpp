// flopcount.cpp -- counts the arithmetic of one photon-step of the GPU
// integrator by instantiating the very same templated step (kerr.hpp) with a
// counting number type on the host.
//
// Weights: add, sub, mul = 1 flop; fma = 2; a division or reciprocal = 1;
// sqrt = 1; sin and cos of an angle = 1 each, however they are evaluated (the
// kernel's polynomial and angle-addition evaluations are counted as the two
// functions they stand for). Comparisons, fabs and negation are free. The
// count is for the common path of a step (no Euler fallback, no remap); it is
// the algorithmic work per accepted photon-step used for the roofline.
//
// Build and run (host only):
//   hipcc -x hip --offload-host-only -O1 -I include flopcount.cpp -o flopcount && ./flopcount
#include <cmath>
#include <cstdio>

struct Cnt {
    long add = 0, mul = 0, fma = 0, div = 0, sqrt = 0, trans = 0;
};
static Cnt g;

struct Flop {
    double v;
    Flop() : v(0) {}
    Flop(double x) : v(x) {}
};
inline Flop operator+(Flop a, Flop b) { ++g.add; return Flop(a.v + b.v); }
inline Flop operator-(Flop a, Flop b) { ++g.add; return Flop(a.v - b.v); }
inline Flop operator*(Flop a, Flop b) { ++g.mul; return Flop(a.v * b.v); }
inline Flop operator/(Flop a, Flop b) { ++g.div; return Flop(a.v / b.v); }
inline Flop operator-(Flop a) { return Flop(-a.v); }
inline bool operator<(Flop a, Flop b) { return a.v < b.v; }
inline bool operator>(Flop a, Flop b) { return a.v > b.v; }
inline bool operator!=(Flop a, Flop b) { return a.v != b.v; }
inline Flop fabs(Flop a) { return Flop(std::fabs(a.v)); }
inline Flop fma(Flop a, Flop b, Flop c) { ++g.fma; return Flop(a.v * b.v + c.v); }
inline Flop sqrt(Flop a) { ++g.sqrt; return Flop(std::sqrt(a.v)); }
inline Flop rcp(Flop a) { ++g.div; return Flop(1.0 / a.v); }
inline Flop quot(Flop a, Flop b) { ++g.div; return Flop(a.v / b.v); }
inline void sin_cos(Flop x, Flop &s, Flop &c)
{
    g.trans += 2;
    s = Flop(std::sin(x.v));
    c = Flop(std::cos(x.v));
}
inline void shift_sincos(Flop, Flop, Flop, Flop th, Flop &s, Flop &c) { sin_cos(th, s, c); }

#include "kerr.hpp"

int main()
{
    using namespace gray;
    // A generic null state: a = 0.9 ray launched from a screen at r = 12 with
    // all momentum components nonzero, far from the horizon, poles and the
    // static limit.
    StepConst<Flop> K;
    K.B = make_spin(Flop(0.9)); K.rbh = horizon_radius(0.9);
    K.step_frac = 1.0 / 32; K.xi_eps = 1e-3; K.euler_inv = 1.0 / 9.0;
    State<double> x0;
    camera_state(0.9, 12.0, 1.0, 4.0, 3.0, x0);
    State<Flop> x;
    x.t = x0.t; x.r = x0.r; x.th = x0.th; x.ph = x0.ph;
    x.kt = x0.kt; x.kr = x0.kr; x.kth = x0.kth; x.kph = x0.kph;

    g = Cnt();
    Flop sn(std::sin(x0.th)), cn(std::cos(x0.th));
    const int fl = rk4_step(K, x, sn, cn);
    const long step_flops = g.add + g.mul + 2 * g.fma + g.div + g.sqrt + g.trans;
    Cnt st = g;

    g = Cnt();
    Flop dkt, dkr, dkth, dkph;
    accel<Flop>(K.B, Flop(12.0), Flop(0.8), Flop(0.6), Flop(-1.0), Flop(-0.9), Flop(0.01),
                Flop(0.02), dkt, dkr, dkth, dkph);
    const long rhs_flops = g.add + g.mul + 2 * g.fma + g.div + g.sqrt + g.trans;

    printf("{\"flags\": %d, \"step_flops\": %ld, \"rhs_flops\": %ld, \"add\": %ld, \"mul\": %ld, "
           "\"fma\": %ld, \"div\": %ld, \"sqrt\": %ld, \"trans\": %ld}\n",
           fl, step_flops, rhs_flops, st.add, st.mul, st.fma, st.div, st.sqrt, st.trans);
    return fl == 0 ? 0 : 1;
}
