// Host check of the generated part of the specialized evaluator: the
// diagram's straight-line functions (leaf_args, group_sums, den_args,
// group_products, groups_combine, den_cotangents, den_scatter, leaf_cotangents, leaf_scatter,
// line_trig, line_scatter, taylor_leaves, taylor_slopes) compiled with a host compiler and driven one sample at
// a time through the same steps as the device kernels, so a test can compare
// values and gradients with the oracle.  The generated source is included
// through AMI_GENERATED without its two #include lines.
//
// stdin: n_s n_f beta e_reg t mu, then q (2 NX), then the frequencies
// (n_f * NX pairs re im), then per sample its inputs (NE energies, or 2 NI
// momenta with AMI_JIT_HUB) and n_f cotangents (re im).
// stdout per sample: n_f values (re im), then the input gradients (NE or
// 2 NI), then dL/dbeta, dL/dmu, dL/dt, then n_f * NX dL/dw (re im).
#include <cstdio>
#include <cstdint>
#include <vector>

#include "../../paper_2311_17189_amd/csrc/device_common.hpp"

#include AMI_GENERATED

using namespace amijit;

constexpr int NXA = NX > 0 ? NX : 1;
constexpr int NIA = NI > 0 ? NI : 1;
constexpr int NGA = NG > 0 ? NG : 1;

int main() {
    int n_s, n_f;
    double beta, e_reg, t, mu;
    if (std::scanf("%d %d %lf %lf %lf %lf", &n_s, &n_f, &beta, &e_reg, &t, &mu) != 6) return 2;
    double q[2 * NXA] = {0.0};
    for (int x = 0; x < 2 * NX; ++x)
        if (std::scanf("%lf", &q[x]) != 1) return 2;
    std::vector<double> wre(static_cast<size_t>(n_f) * NXA), wim(static_cast<size_t>(n_f) * NXA);
    for (int f = 0; f < n_f; ++f)
        for (int x = 0; x < NX; ++x)
            if (std::scanf("%lf %lf", &wre[f * NXA + x], &wim[f * NXA + x]) != 2) return 2;
    for (int s = 0; s < n_s; ++s) {
        double E[NE], sx[NGA] = {0.0}, sy[NGA] = {0.0}, cs[NGA] = {0.0};
        if (AMI_JIT_HUB) {
            double kx[NIA], ky[NIA], Kx[NGA], Ky[NGA];
            for (int l = 0; l < NI; ++l) {
                double a, b;
                if (std::scanf("%lf %lf", &a, &b) != 2) return 2;
                kx[l] = ami::reduce_2pi(a);
                ky[l] = ami::reduce_2pi(b);
            }
            double qr[2 * NXA], qs[2 * NXA], qc[2 * NXA];
            for (int x = 0; x < 2 * NXA; ++x) {
                qr[x] = ami::reduce_2pi(q[x]);
                qs[x] = std::sin(qr[x]);
                qc[x] = std::cos(qr[x]);
            }
            (void)Kx;
            (void)Ky;
            // as the adjoint kernel: sin/cos of the loop momenta, lines by angle addition
            double lsx[NIA], lcx[NIA], lsy[NIA], lcy[NIA], Cx[NGA], Cy[NGA];
            for (int l = 0; l < NI; ++l) {
                ami::sincos_red(kx[l], lsx[l], lcx[l]);
                ami::sincos_red(ky[l], lsy[l], lcy[l]);
            }
            line_trig(lsx, lcx, lsy, lcy, qs, qc, sx, Cx, sy, Cy);
            for (int j = 0; j < NG; ++j) {
                cs[j] = Cx[j] + Cy[j];
                E[j] = std::fma(2.0 * t, cs[j], mu);
            }
        } else {
            for (int i = 0; i < NE; ++i)
                if (std::scanf("%lf", &E[i]) != 1) return 2;
        }
        std::vector<double> cre(n_f), cim(n_f);
        for (int f = 0; f < n_f; ++f)
            if (std::scanf("%lf %lf", &cre[f], &cim[f]) != 2) return 2;

        double x[L], F[L], FM[L], Dv[L];
        leaf_args(E, x);
        for (int l = 0; l < L; ++l) {
            if (kBose[l]) x[l] += e_reg;
            ami::leaf_pair(kBose[l], beta * x[l], F[l], FM[l]);
            Dv[l] = -(F[l] * FM[l]);
        }
        double DX[L], DB[L];          // Taylor-coefficient leaves: dT/dx, dT/dbeta
        taylor_slopes(F, FM, x, beta, DX, DB);
        taylor_leaves(F, FM, beta);
        double FT[G], FTB[G] = {0.0}, gE[NE] = {0.0};
        group_sums(F, FT);
        std::vector<double> gw(2 * static_cast<size_t>(n_f) * NXA, 0.0);
        for (int f = 0; f < n_f; ++f) {
            double wr[NXA], wi[NXA], dr[D], di[D], xr[D], xi[D], Rr[G], Ri[G];
            for (int xx = 0; xx < NXA; ++xx) {
                wr[xx] = wre[f * NXA + xx];
                wi[xx] = wim[f * NXA + xx];
            }
            den_args(E, wr, wi, dr, di);
            for (int k = 0; k < D; ++k) {
                const double inv = 1.0 / std::fma(dr[k], dr[k], di[k] * di[k]);
                xr[k] = dr[k] * inv;
                xi[k] = -di[k] * inv;
            }
            group_products(xr, xi, Rr, Ri);
            double acc_re, acc_im, ur[G], ui[G];
            groups_combine(xr, xi, FT, acc_re, acc_im);     // the kernels' values
            const double cr = cre[f], ci = cim[f];
            for (int g = 0; g < G; ++g) {
                FTB[g] += std::fma(cr, Rr[g], ci * Ri[g]);
                const double qr = FT[g] * cr, qi = -FT[g] * ci;
                ur[g] = -std::fma(qr, Rr[g], -qi * Ri[g]);
                ui[g] = -std::fma(qr, Ri[g], qi * Rr[g]);
            }
            std::printf("%.17g %.17g ", acc_re, acc_im);
            double Ur[D], Ui[D], dR[D], dI[D], gwr[NXA] = {0.0}, gwi[NXA] = {0.0};
            den_cotangents(ur, ui, Ur, Ui);
            for (int k = 0; k < D; ++k) {
                dR[k] = std::fma(Ur[k], xr[k], -Ui[k] * xi[k]);
                dI[k] = std::fma(Ur[k], xi[k], Ui[k] * xr[k]);
            }
            den_scatter(dR, dI, gE, gwr, gwi);
            for (int xx = 0; xx < NX; ++xx) {
                gw[2 * (f * NXA + xx)] = gwr[xx];
                gw[2 * (f * NXA + xx) + 1] = -gwi[xx];
            }
        }
        double FB[L] = {0.0}, v[L], gbeta = 0.0;
        leaf_cotangents(F, FTB, FB);
        for (int l = 0; l < L; ++l) {
            if (kTaylor) {
                v[l] = FB[l] * DX[l];
                gbeta = std::fma(FB[l], DB[l], gbeta);
            } else {
                const double fb = FB[l] * Dv[l];
                v[l] = fb * beta;
                gbeta = std::fma(fb, x[l], gbeta);
            }
        }
        leaf_scatter(v, gE);
        double gmu = 0.0, gt = 0.0;
        if (AMI_JIT_HUB) {
            double gx[NGA], gy[NGA], gkx[NIA] = {0.0}, gky[NIA] = {0.0};
            for (int j = 0; j < NG; ++j) {
                gmu += gE[j];
                gt = std::fma(gE[j], 2.0 * cs[j], gt);
                gx[j] = -2.0 * t * gE[j] * sx[j];
                gy[j] = -2.0 * t * gE[j] * sy[j];
            }
            line_scatter(gx, gy, gkx, gky);
            for (int l = 0; l < NI; ++l) std::printf("%.17g %.17g ", gkx[l], gky[l]);
        } else {
            for (int i = 0; i < NE; ++i) std::printf("%.17g ", gE[i]);
        }
        std::printf("%.17g %.17g %.17g", gbeta, gmu, gt);
        for (int f = 0; f < n_f; ++f)
            for (int xx = 0; xx < NX; ++xx) std::printf(" %.17g %.17g", gw[2 * (f * NXA + xx)], gw[2 * (f * NXA + xx) + 1]);
        std::printf("\n");
    }
    return 0;
}
