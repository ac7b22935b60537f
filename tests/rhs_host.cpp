// Host build of the integrator's right-hand side and null-condition test
// (csrc/kerr.hpp), for the CPU tests that compare them with the oracle.
// Default: reads lines "a r theta kt kr kth kph" on stdin, writes
// "dkt dkr dkth dkph". With the argument "xi": reads lines
// "a r theta kt kr kth kph eps", writes 1 when the test of eq. (4) reports
// |xi + 1| > eps, else 0.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "kerr.hpp"

int main(int argc, char **argv)
{
    double a, r, th, kt, kr, kth, kph, eps;
    if (argc > 1 && std::strcmp(argv[1], "xi") == 0) {
        while (std::scanf("%lf %lf %lf %lf %lf %lf %lf %lf", &a, &r, &th, &kt, &kr, &kth, &kph, &eps) == 8)
            std::printf("%d\n", gray::xi_violated_at(a, a * a, r, std::sin(th), std::cos(th), kt, kr, kth, kph, eps)
                                    ? 1 : 0);
        return 0;
    }
    while (std::scanf("%lf %lf %lf %lf %lf %lf %lf", &a, &r, &th, &kt, &kr, &kth, &kph) == 7) {
        double o[4];
        gray::accel<double>(gray::make_spin(a), r, std::sin(th), std::cos(th), kt, kr, kth, kph, o[0], o[1], o[2],
                            o[3]);
        std::printf("%.17g %.17g %.17g %.17g\n", o[0], o[1], o[2], o[3]);
    }
    return 0;
}
