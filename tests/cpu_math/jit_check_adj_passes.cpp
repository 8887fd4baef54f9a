// Host check of the generated part of the adjoint of large solutions in
// passes: the two-pass forward's group_sums_store (first pass), then per
// frequency row adj_freq_row (values, group-sum cotangents, the
// denominators' scatter; second pass), then leaf_pass and the lines' scatter
// (third pass), compiled with a host compiler and
// driven one sample at a time through the kernels' steps with a one-sample
// workspace (ld = 1), so a test can compare values and gradients with the
// oracle.  The generated source is included through AMI_GENERATED without its
// two #include lines.
//
// stdin/stdout: as jit_check.cpp.
#include <cmath>
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
        taylor_leaves(F, FM, beta);   // as the sums pass (Taylor-coefficient leaves)
        // workspace of one sample: FT_g, E_j, the denominators' energy
        // cotangents, FTB_g
        std::vector<double> ws(2 * static_cast<size_t>(G) + 2 * NE, 0.0);
        group_sums_store(F, ws.data(), 1, 0u);
        for (int j = 0; j < NE; ++j) ws[G + j] = E[j];
        double gE[NE] = {0.0};
        std::vector<double> gw(2 * static_cast<size_t>(n_f) * NXA, 0.0);
        for (int f = 0; f < n_f; ++f) {
            double wr[NXA], wi[NXA], gwr[NXA] = {0.0}, gwi[NXA] = {0.0};
            for (int xx = 0; xx < NXA; ++xx) {
                wr[xx] = wre[f * NXA + xx];
                wi[xx] = wim[f * NXA + xx];
            }
            double acc_re = 0.0, acc_im = 0.0;
            if (f == 0) adj_freq_row<true>(E, wr, wi, cre[f], cim[f], ws.data(), 1, 0u, acc_re, acc_im, gE, gwr, gwi);
            else adj_freq_row<false>(E, wr, wi, cre[f], cim[f], ws.data(), 1, 0u, acc_re, acc_im, gE, gwr, gwi);
            std::printf("%.17g %.17g ", acc_re, acc_im);
            for (int xx = 0; xx < NX; ++xx) {
                gw[2 * (f * NXA + xx)] = gwr[xx];
                gw[2 * (f * NXA + xx) + 1] = -gwi[xx];
            }
        }
        for (int j = 0; j < NE; ++j) ws[G + NE + j] = gE[j];
        double gbeta = 0.0;
        for (int j = 0; j < NE; ++j) gE[j] = ws[G + NE + j];
        leaf_pass(E, beta, e_reg, ws.data(), 1, 0u, gE, gbeta);
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
