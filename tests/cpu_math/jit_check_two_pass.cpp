// Host check of the generated part of the two-pass forward: the diagram's
// leaf_args, taylor_leaves, group_sums_store (first pass) and den_args,
// group_accumulate (second pass) compiled with a host compiler, with the
// device leaves and cosines, driven one sample at a time through the steps of
// the two kernels, so a test can compare values with the oracle.  The
// generated source is included through AMI_GENERATED without its two
// #include lines.
//
// stdin: n_s n_f beta e_reg t mu, then q (2 NX), then the frequencies
// (n_f * NX pairs re im), then per sample its inputs (NE energies, or 2 NI
// momenta with AMI_JIT_HUB).
// stdout per sample: n_f values (re im).
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
    std::vector<double> wre(static_cast<size_t>(n_f) * NXA, 0.0), wim(static_cast<size_t>(n_f) * NXA, 0.0);
    for (int f = 0; f < n_f; ++f)
        for (int x = 0; x < NX; ++x)
            if (std::scanf("%lf %lf", &wre[f * NXA + x], &wim[f * NXA + x]) != 2) return 2;
    for (int s = 0; s < n_s; ++s) {
        double E[NE];
        if (AMI_JIT_HUB) {
            double kx[NIA], ky[NIA], Kx[NGA], Ky[NGA], qr[2 * NXA];
            for (int l = 0; l < NI; ++l) {
                double a, b;
                if (std::scanf("%lf %lf", &a, &b) != 2) return 2;
                kx[l] = ami::reduce_2pi(a);
                ky[l] = ami::reduce_2pi(b);
            }
            for (int x = 0; x < 2 * NXA; ++x) qr[x] = ami::reduce_2pi(q[x]);
            lines(kx, ky, qr, Kx, Ky);
            for (int j = 0; j < NG; ++j) E[j] = std::fma(2.0 * t, ami::cos_red(Kx[j]) + ami::cos_red(Ky[j]), mu);
        } else {
            for (int i = 0; i < NE; ++i)
                if (std::scanf("%lf", &E[i]) != 1) return 2;
        }
        // first pass
        double x[L], F[L], FM[L], ft[G];
        leaf_args(E, x);
        for (int l = 0; l < L; ++l) {
            if (kBose[l]) x[l] += e_reg;
            ami::leaf_pair(kBose[l], beta * x[l], F[l], FM[l]);
        }
        taylor_leaves(F, FM, beta);
        group_sums_store(F, ft, 1, 0u);
        // second pass, frequency by frequency
        for (int f = 0; f < n_f; ++f) {
            double wr[NXA], wi[NXA], dr[D], di[D], xr[D], xi[D];
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
            double acc_re = 0.0, acc_im = 0.0;
            group_accumulate(xr, xi, ft, 1, 0u, acc_re, acc_im);
            std::printf("%.17g %.17g ", acc_re, acc_im);
        }
        std::printf("\n");
    }
    return 0;
}
