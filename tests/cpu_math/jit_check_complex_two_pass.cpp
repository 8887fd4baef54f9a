// Host check of the generated part of the two-pass forward at complex
// energies: the diagram's leaf_args, group_sums_c_store (first pass) and
// den_args, group_accumulate_c (second pass) compiled with a host compiler,
// with the device leaf at a complex argument, driven one sample at a time
// through the steps of the two kernels with a one-sample workspace (ld = 1),
// so a test can compare values with the oracle.  The generated source is
// included through AMI_GENERATED without its two #include lines.
//
// stdin/stdout: as jit_check_complex.cpp.
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
    std::vector<double> ws(2 * static_cast<size_t>(G) + 2 * NE);
    for (int s = 0; s < n_s; ++s) {
        double Er[NE], Ei[NE];
        for (int i = 0; i < NE; ++i)
            if (std::scanf("%lf %lf", &Er[i], &Ei[i]) != 2) return 2;
        // first pass: the complex group sums and the energies into the workspace
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
        // second pass, frequency by frequency, from the workspace
        double er[NE], ei[NE];
        for (int j = 0; j < NE; ++j) {
            er[j] = ws[2 * G + j];
            ei[j] = ws[2 * G + NE + j];
        }
        double zr[NXA] = {0.0}, zi[NXA] = {0.0}, dEi[D], unused[D];
        den_args(ei, zr, zi, dEi, unused);
        for (int f = 0; f < n_f; ++f) {
            double wr[NXA], wi[NXA], dr[D], di[D], rr[D], ri[D];
            for (int x = 0; x < NXA; ++x) {
                wr[x] = wre[f * NXA + x];
                wi[x] = wim[f * NXA + x];
            }
            den_args(er, wr, wi, dr, di);
            for (int k = 0; k < D; ++k) {
                const double im = di[k] + dEi[k];
                const double inv = 1.0 / std::fma(dr[k], dr[k], im * im);
                rr[k] = dr[k] * inv;
                ri[k] = -im * inv;
            }
            double acc_re = 0.0, acc_im = 0.0;
            group_accumulate_c(rr, ri, ws.data(), 1, 0u, acc_re, acc_im);
            std::printf("%.17g %.17g ", acc_re, acc_im);
        }
        std::printf("\n");
    }
    return 0;
}
