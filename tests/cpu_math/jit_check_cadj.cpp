// Host check of the generated part of the adjoint at complex energies: the
// diagram's leaf_args, den_args, group_sums_c, group_products, den_cotangents,
// den_scatter, leaf_cotangents_c and leaf_scatter compiled with a host
// compiler, with the device leaf pair at a complex argument, driven one sample
// at a time through the steps of the complex-energy adjoint kernel, so a test
// can compare values and gradients with the oracle.  The generated source is
// included through AMI_GENERATED without its two #include lines.
//
// stdin: n_s n_f beta e_reg, then the frequencies (n_f * NX pairs re im), then
// per sample its NE energies (pairs re im) and n_f cotangents (re im).
// stdout per sample: n_f values (re im), NE energy gradients (re im),
// dL/dbeta, then n_f * NX dL/dw (re im).
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
        std::vector<double> cre(n_f), cim(n_f);
        for (int f = 0; f < n_f; ++f)
            if (std::scanf("%lf %lf", &cre[f], &cim[f]) != 2) return 2;
        double xr[L], xi[L], Fr[L], Fi[L], Mr[L], Mi[L], FTr[G], FTi[G];
        leaf_args(Er, xr);
        leaf_args(Ei, xi);
        for (int l = 0; l < L; ++l) {
            if (kBose[l]) xr[l] += e_reg;
            ami::leaf_complex_pair(kBose[l], beta * xr[l], beta * xi[l], Fr[l], Fi[l], Mr[l], Mi[l]);
        }
        group_sums_c(Fr, Fi, FTr, FTi);
        double zr[NXA] = {0.0}, zi[NXA] = {0.0}, dEi[D], unused[D];
        den_args(Ei, zr, zi, dEi, unused);
        double FTBr[G] = {0.0}, FTBi[G] = {0.0}, gEr[NE] = {0.0}, gEi[NE] = {0.0};
        std::vector<double> gw(2 * static_cast<size_t>(n_f) * NXA, 0.0);
        for (int f = 0; f < n_f; ++f) {
            double wr[NXA], wi[NXA], dr[D], di[D], rr[D], ri[D], Rr[G], Ri[G], ur[G], ui[G];
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
            const double cr = cre[f], ci = cim[f];
            double acc_re = 0.0, acc_im = 0.0;
            for (int g = 0; g < G; ++g) {
                acc_re = std::fma(FTr[g], Rr[g], std::fma(-FTi[g], Ri[g], acc_re));
                acc_im = std::fma(FTr[g], Ri[g], std::fma(FTi[g], Rr[g], acc_im));
                FTBr[g] += std::fma(cr, Rr[g], ci * Ri[g]);
                FTBi[g] += std::fma(ci, Rr[g], -cr * Ri[g]);
                const double qr = std::fma(FTr[g], cr, FTi[g] * ci);
                const double qi = std::fma(FTi[g], cr, -FTr[g] * ci);
                ur[g] = -std::fma(qr, Rr[g], -qi * Ri[g]);
                ui[g] = -std::fma(qr, Ri[g], qi * Rr[g]);
            }
            std::printf("%.17g %.17g ", acc_re, acc_im);
            double Ur[D], Ui[D], dR[D], dI[D], ndI[D], gwr[NXA] = {0.0}, gwi[NXA] = {0.0}, jr[NXA], ji[NXA];
            den_cotangents(ur, ui, Ur, Ui);
            for (int k = 0; k < D; ++k) {
                dR[k] = std::fma(Ur[k], rr[k], -Ui[k] * ri[k]);
                dI[k] = std::fma(Ur[k], ri[k], Ui[k] * rr[k]);
                ndI[k] = -dI[k];
            }
            den_scatter(dR, dI, gEr, gwr, gwi);
            den_scatter(ndI, dR, gEi, jr, ji);
            for (int x = 0; x < NX; ++x) {
                gw[2 * (f * NXA + x)] = gwr[x];
                gw[2 * (f * NXA + x) + 1] = -gwi[x];
            }
        }
        double cFi[L], FBr[L] = {0.0}, FBi[L] = {0.0}, vr[L], vi[L], gbeta = 0.0;
        for (int l = 0; l < L; ++l) cFi[l] = -Fi[l];
        leaf_cotangents_c(Fr, cFi, FTBr, FTBi, FBr, FBi);
        for (int l = 0; l < L; ++l) {
            const double dpr = -std::fma(Fr[l], Mr[l], -Fi[l] * Mi[l]);
            const double dpi = -std::fma(Fr[l], Mi[l], Fi[l] * Mr[l]);
            const double Vr = std::fma(FBr[l], dpr, FBi[l] * dpi);
            const double Vi = std::fma(FBi[l], dpr, -FBr[l] * dpi);
            gbeta = std::fma(Vr, xr[l], std::fma(Vi, xi[l], gbeta));
            vr[l] = Vr * beta;
            vi[l] = Vi * beta;
        }
        leaf_scatter(vr, gEr);
        leaf_scatter(vi, gEi);
        for (int i = 0; i < NE; ++i) std::printf("%.17g %.17g ", gEr[i], gEi[i]);
        std::printf("%.17g", gbeta);
        for (int f = 0; f < n_f; ++f)
            for (int x = 0; x < NX; ++x) std::printf(" %.17g %.17g", gw[2 * (f * NXA + x)], gw[2 * (f * NXA + x) + 1]);
        std::printf("\n");
    }
    return 0;
}
