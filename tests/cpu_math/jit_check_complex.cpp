// Host check of the generated part of the complex-energy evaluator: the
// diagram's leaf_args, den_args, group_sums_c and group_products compiled with
// a host compiler, with the device leaf at a complex argument, driven one
// sample at a time through the steps of the complex-energy kernel, so a test
// can compare values with the oracle.  The generated source is included
// through AMI_GENERATED without its two #include lines.
//
// stdin: n_s n_f beta e_reg, then the frequencies (n_f * NX pairs re im),
// then per sample its NE energies (pairs re im).
// stdout per sample: n_f values (re im).
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
    for (int s = 0; s < n_s; ++s) {
        double Er[NE], Ei[NE];
        for (int i = 0; i < NE; ++i)
            if (std::scanf("%lf %lf", &Er[i], &Ei[i]) != 2) return 2;
        double xr[L], xi[L], Fr[L], Fi[L], FTr[G], FTi[G];
        leaf_args(Er, xr);
        leaf_args(Ei, xi);
        for (int l = 0; l < L; ++l)
            ami::leaf_complex(kBose[l], beta * (kBose[l] ? xr[l] + e_reg : xr[l]), beta * xi[l], Fr[l], Fi[l]);
        group_sums_c(Fr, Fi, FTr, FTi);
        double zr[NXA] = {0.0}, zi[NXA] = {0.0}, dEi[D], unused[D];
        den_args(Ei, zr, zi, dEi, unused);
        for (int f = 0; f < n_f; ++f) {
            double wr[NXA], wi[NXA], dr[D], di[D], rr[D], ri[D], Rr[G], Ri[G];
            for (int x = 0; x < NXA; ++x) {
                wr[x] = wre[f * NXA + x];
                wi[x] = wim[f * NXA + x];
            }
            den_args(Er, wr, wi, dr, di);
            for (int k = 0; k < D; ++k) {
                const double im = di[k] + dEi[k];
                const double inv = 1.0 / std::fma(dr[k], dr[k], im * im);
                rr[k] = dr[k] * inv;
                ri[k] = -im * inv;
            }
            group_products(rr, ri, Rr, Ri);
            double acc_re = 0.0, acc_im = 0.0;
            for (int g = 0; g < G; ++g) {
                acc_re = std::fma(FTr[g], Rr[g], std::fma(-FTi[g], Ri[g], acc_re));
                acc_im = std::fma(FTr[g], Ri[g], std::fma(FTi[g], Rr[g], acc_im));
            }
            std::printf("%.17g %.17g ", acc_re, acc_im);
        }
        std::printf("\n");
    }
    return 0;
}
