// Prints the device math functions of device_common.hpp on a grid of
// arguments (one line per argument) so a test can compare them with mpmath.
#include <cstdio>
#include <cstdint>
#include <cstdlib>

#include "../../paper_2311_17189_amd/csrc/device_common.hpp"

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const char *what = argv[1];
    if (what[0] == 'p') {   // Philox4x32-10: counter[4] key[2] per line -> 4 words, and their momenta
        unsigned long long v[6];
        while (std::scanf("%llu %llu %llu %llu %llu %llu", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 6) {
            uint32_t c[4] = {static_cast<uint32_t>(v[0]), static_cast<uint32_t>(v[1]), static_cast<uint32_t>(v[2]),
                             static_cast<uint32_t>(v[3])};
            ami::philox4x32_10(c, static_cast<uint32_t>(v[4]), static_cast<uint32_t>(v[5]));
            std::printf("%u %u %u %u %.17g %.17g %.17g %.17g\n", c[0], c[1], c[2], c[3], ami::word_to_momentum(c[0]),
                        ami::word_to_momentum(c[1]), ami::word_to_momentum(c[2]), ami::word_to_momentum(c[3]));
        }
        return 0;
    }
    if (what[0] == 'F' || what[0] == 'B') {   // leaf at a complex argument: yr yi per line -> re im
        double yr, yi, fr, fi;
        while (std::scanf("%lf %lf", &yr, &yi) == 2) {
            ami::leaf_complex(what[0] == 'B', yr, yi, fr, fi);
            std::printf("%.17g %.17g\n", fr, fi);
        }
        return 0;
    }
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
        } else if (what[0] == 'u' || what[0] == 'v') {   // leaf_and_slope: Fermi (u) / Bose-type (v)
            double f, dv;
            ami::leaf_and_slope(what[0] == 'v', x, f, dv);
            std::printf("%.17g %.17g\n", f, dv);
        } else {
            double f, fm;
            const bool bose = what[0] == 'b';
            ami::leaf_pair(bose, x, f, fm);
            std::printf("%.17g %.17g %.17g\n", f, fm, ami::leaf_deriv(bose, x));
        }
    }
    return 0;
}
