// Host check of the generated part of the adjoint at complex energies in
// passes: the complex two-pass forward's group_sums_c_store (first pass),
// then per frequency row cadj_freq_row (values, complex group-sum
// cotangents, the denominators' scatter; second pass), then cleaf_pass
// (third pass), compiled with a host compiler and driven one sample at a
// time through the kernels' steps with a one-sample workspace (ld = 1), so a
// test can compare values and gradients with the oracle.  The generated
// source is included through AMI_GENERATED without its two #include lines.
//
// stdin/stdout: as jit_check_cadj.cpp.
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <vector>

#include "../../paper_2311_17189_amd/csrc/device_common.hpp"

#include AMI_GENERATED

using namespace amijit;

constexpr int NXA = NX > 0 ? NX : 1;

int main() {
    int n_s, n_f;
    double beta, e_reg;
    if (std::scanf("%d %d %lf %lf", &n_s, &n_f, &beta, &e_reg) != 4) return 2;
    std::vector<double> wre(static_cast<size_t>(n_f) * NXA, 0.0), wim(static_cast<size_t>(n_f) * NXA, 0.0);
    for (int f = 0; f < n_f; ++f)
        for (int x = 0; x < NX; ++x)
            if (std::scanf("%lf %lf", &wre[f * NXA + x], &wim[f * NXA + x]) != 2) return 2;
    // workspace of one sample: FT (re G, im G), E (re NE, im NE), the
    // denominators' energy cotangents (re NE, im NE), FTB (re G, im G)
    std::vector<double> ws(4 * static_cast<size_t>(G) + 4 * NE, 0.0);
    for (int s = 0; s < n_s; ++s) {
        double Er[NE], Ei[NE];
        for (int i = 0; i < NE; ++i)
            if (std::scanf("%lf %lf", &Er[i], &Ei[i]) != 2) return 2;
        std::vector<double> cre(n_f), cim(n_f);
        for (int f = 0; f < n_f; ++f)
            if (std::scanf("%lf %lf", &cre[f], &cim[f]) != 2) return 2;
        // first pass
        double xr[L], xi[L], Fr[L], Fi[L];
        leaf_args(Er, xr);
        leaf_args(Ei, xi);
        for (int l = 0; l < L; ++l)
            ami::leaf_complex(kBose[l], beta * (kBose[l] ? xr[l] + e_reg : xr[l]), beta * xi[l], Fr[l], Fi[l]);
        group_sums_c_store(Fr, Fi, ws.data(), 1, 0u);
        for (int j = 0; j < NE; ++j) {
            ws[2 * G + j] = Er[j];
            ws[2 * G + NE + j] = Ei[j];
        }
        // frequency pass
        double er[NE], ei[NE], gEr[NE] = {0.0}, gEi[NE] = {0.0};
        for (int j = 0; j < NE; ++j) {
            er[j] = ws[2 * G + j];
            ei[j] = ws[2 * G + NE + j];
        }
        std::vector<double> gw(2 * static_cast<size_t>(n_f) * NXA, 0.0);
        for (int f = 0; f < n_f; ++f) {
            double wr[NXA], wi[NXA], gwr[NXA] = {0.0}, gwi[NXA] = {0.0};
            for (int x = 0; x < NXA; ++x) {
                wr[x] = wre[f * NXA + x];
                wi[x] = wim[f * NXA + x];
            }
            double acc_re = 0.0, acc_im = 0.0;
            if (f == 0)
                cadj_freq_row<true>(er, ei, wr, wi, cre[f], cim[f], ws.data(), 1, 0u, acc_re, acc_im, gEr, gEi, gwr, gwi);
            else
                cadj_freq_row<false>(er, ei, wr, wi, cre[f], cim[f], ws.data(), 1, 0u, acc_re, acc_im, gEr, gEi, gwr,
                                     gwi);
            std::printf("%.17g %.17g ", acc_re, acc_im);
            for (int x = 0; x < NX; ++x) {
                gw[2 * (f * NXA + x)] = gwr[x];
                gw[2 * (f * NXA + x) + 1] = -gwi[x];
            }
        }
        for (int j = 0; j < NE; ++j) {
            ws[2 * G + 2 * NE + j] = gEr[j];
            ws[2 * G + 3 * NE + j] = gEi[j];
        }
        // leaf pass
        double hr[NE], hi[NE], gbeta = 0.0;
        for (int j = 0; j < NE; ++j) {
            hr[j] = ws[2 * G + 2 * NE + j];
            hi[j] = ws[2 * G + 3 * NE + j];
        }
        cleaf_pass(er, ei, beta, e_reg, ws.data(), 1, 0u, hr, hi, gbeta);
        for (int i = 0; i < NE; ++i) std::printf("%.17g %.17g ", hr[i], hi[i]);
        std::printf("%.17g", gbeta);
        for (int f = 0; f < n_f; ++f)
            for (int x = 0; x < NX; ++x) std::printf(" %.17g %.17g", gw[2 * (f * NXA + x)], gw[2 * (f * NXA + x) + 1]);
        std::printf("\n");
    }
    return 0;
}
