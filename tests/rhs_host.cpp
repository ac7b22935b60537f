// Host build of the integrator's right-hand side (csrc/kerr.hpp), for the
// CPU test that compares it with the oracle's Christoffel-sum RHS. Reads
// lines "a r theta kt kr kth kph" on stdin, writes "dkt dkr dkth dkph".
#include <cmath>
#include <cstdio>

#include "kerr.hpp"

int main()
{
    double a, r, th, kt, kr, kth, kph;
    while (std::scanf("%lf %lf %lf %lf %lf %lf %lf", &a, &r, &th, &kt, &kr, &kth, &kph) == 7) {
        double o[4];
        gray::accel<double>(gray::make_spin(a), r, std::sin(th), std::cos(th), kt, kr, kth, kph, o[0], o[1], o[2],
                            o[3]);
        std::printf("%.17g %.17g %.17g %.17g\n", o[0], o[1], o[2], o[3]);
    }
    return 0;
}
