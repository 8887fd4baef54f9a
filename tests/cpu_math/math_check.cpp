// Prints the device math functions of device_common.hpp on a grid of
// arguments (one line per argument) so a test can compare them with mpmath.
#include <cstdio>
#include <cstdint>
#include <cstdlib>

#include "../../paper_2311_17189_amd/csrc/device_common.hpp"

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const char *what = argv[1];
    double x;
    while (std::scanf("%lf", &x) == 1) {
        if (what[0] == 'r') {
            std::printf("%.17g\n", ami::reduce_2pi(x));
        } else if (what[0] == 'c') {
            std::printf("%.17g\n", ami::cos_red(x));
        } else if (what[0] == 's') {
            double s, c;
            ami::sincos_red(x, s, c);
            std::printf("%.17g %.17g\n", s, c);
        } else if (what[0] == 'e') {
            double t, m;
            ami::exp_split(x, t, m);
            std::printf("%.17g %.17g\n", t, m);
        } else {
            double f, fm;
            const bool bose = what[0] == 'b';
            ami::leaf_pair(bose, x, f, fm);
            std::printf("%.17g %.17g %.17g\n", f, fm, ami::leaf_deriv(bose, x));
        }
    }
    return 0;
}
