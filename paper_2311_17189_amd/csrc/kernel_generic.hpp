// Generic evaluator over the double-valued tables: any coefficient values and
// table sizes, used when the packed form does not apply (see kernels_packed.hpp
// for the specialized evaluator).  One lane per sample; leaves, Fermi-tree
// group sums and denominator reciprocals live in LDS columns.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ami_internal.hpp"

namespace ami {

struct FwdParams {
    // tables
    const double *leaf_coef;
    const double *leaf_sigma;
    const double *den_coef;
    const int32_t *group_dens;
    const int32_t *group_start;
    const double *term_sign;
    const int32_t *term_leaf;
    const double *line_alpha;
    int n_eps, n_ext, n_int, n_g, n_freq;
    int L, D, G, dpt;
    int region_a;            // LDS slots (per lane) before the FT region: max(L, 2D)
    // energy input
    const double *energies;
    int64_t stride_s, stride_i;
    // momentum input
    const double *k;
    int64_t stride_k;
    double q[2 * kMaxExt];
    double hop_t, mu;
    // frequencies, parameters, outputs
    const double *ext_freqs;
    int n_f;
    double beta, e_reg;
    int64_t n_e;
    double *out;
    double *partial;          // [gridDim.x][n_f][2] or NULL
};

// f_sigma(y) = 1/(sigma e^y + 1).  The Bose-type form -1/expm1(y) keeps full
// relative precision next to its removable pole at y = 0.
__device__ __forceinline__ double leaf_fn(double sigma, double y) {
    if (sigma > 0.0) return 1.0 / (1.0 + exp(y));
    return -1.0 / expm1(y);
}

template <int MAXE, bool HUB>
__global__ __launch_bounds__(256) void ami_fwd_kernel(FwdParams p) {
    extern __shared__ double sm[];
    const int tid = threadIdx.x;
    const int B = blockDim.x;
    const int64_t s = static_cast<int64_t>(blockIdx.x) * B + tid;
    const bool active = s < p.n_e;
    const int64_t sc = active ? s : (p.n_e - 1);

    double E[MAXE];
#pragma unroll
    for (int i = 0; i < MAXE; ++i) E[i] = 0.0;

    if constexpr (HUB) {
        // momenta of the summed slots in registers; external momenta are kernel arguments
        double kx[kMaxInt], ky[kMaxInt];
        const double *krow = p.k + sc * p.stride_k;
#pragma unroll
        for (int l = 0; l < kMaxInt; ++l) {
            kx[l] = 0.0;
            ky[l] = 0.0;
            if (l < p.n_int) {
                kx[l] = krow[2 * l];
                ky[l] = krow[2 * l + 1];
            }
        }
#pragma unroll
        for (int j = 0; j < MAXE; ++j) {
            if (j < p.n_g) {
                // K_j = sum_l alpha_jl k_l (Sec. 5.2), E_j = -eps(K_j) = 2t(cos Kx + cos Ky) + mu
                const double *a = p.line_alpha + j * p.n_freq;
                double Kx = 0.0, Ky = 0.0;
#pragma unroll
                for (int l = 0; l < kMaxInt; ++l) {
                    if (l < p.n_int) {
                        Kx = fma(a[l], kx[l], Kx);
                        Ky = fma(a[l], ky[l], Ky);
                    }
                }
#pragma unroll
                for (int x = 0; x < kMaxExt; ++x) {
                    if (x < p.n_ext) {
                        Kx = fma(a[p.n_int + x], p.q[2 * x], Kx);
                        Ky = fma(a[p.n_int + x], p.q[2 * x + 1], Ky);
                    }
                }
                E[j] = fma(2.0 * p.hop_t, cos(Kx) + cos(Ky), p.mu);
            }
        }
    } else {
        const double *erow = p.energies + sc * p.stride_s;
#pragma unroll
        for (int i = 0; i < MAXE; ++i)
            if (i < p.n_eps) E[i] = erow[i * p.stride_i];
    }

    // 2. distinct leaves -> LDS
    for (int l = 0; l < p.L; ++l) {
        const double *c = p.leaf_coef + l * p.n_eps;
        double x = 0.0;
#pragma unroll
        for (int i = 0; i < MAXE; ++i)
            if (i < p.n_eps) x = fma(c[i], E[i], x);
        const double sg = p.leaf_sigma[l];
        if (sg < 0.0) x += p.e_reg;
        sm[l * B + tid] = leaf_fn(sg, p.beta * x);
    }

    // 3. Fermi-tree sums per group of equal denominators -> LDS
    double *ftcol = sm + p.region_a * B;
    for (int g = 0; g < p.G; ++g) {
        const int t0 = p.group_start[g], t1 = p.group_start[g + 1];
        double ft = 0.0;
        for (int t = t0; t < t1; ++t) {
            double prod = p.term_sign[t];
            const int32_t *li = p.term_leaf + t * p.n_int;
            for (int j = 0; j < p.n_int; ++j) prod *= sm[li[j] * B + tid];
            ft += prod;
        }
        ftcol[g * B + tid] = ft;
    }

    // 4. per frequency row
    double *red = sm + (p.region_a + p.G) * B;     // 2 doubles per wave
    const int wave = tid >> 6, lane = tid & 63, nwaves = (B + 63) >> 6;
    const int ncoef = p.n_eps + p.n_ext;
    for (int f = 0; f < p.n_f; ++f) {
        double wre[kMaxExt], wim[kMaxExt];
#pragma unroll
        for (int x = 0; x < kMaxExt; ++x) {
            wre[x] = 0.0;
            wim[x] = 0.0;
            if (x < p.n_ext) {
                wre[x] = p.ext_freqs[2 * (f * p.n_ext + x)];
                wim[x] = p.ext_freqs[2 * (f * p.n_ext + x) + 1];
            }
        }
        for (int r = 0; r < p.D; ++r) {
            const double *c = p.den_coef + r * ncoef;
            double dre = 0.0, dim = 0.0;
#pragma unroll
            for (int i = 0; i < MAXE; ++i)
                if (i < p.n_eps) dre = fma(c[i], E[i], dre);
#pragma unroll
            for (int x = 0; x < kMaxExt; ++x) {
                if (x < p.n_ext) {
                    dre = fma(c[p.n_eps + x], wre[x], dre);
                    dim = fma(c[p.n_eps + x], wim[x], dim);
                }
            }
            const double inv = 1.0 / fma(dre, dre, dim * dim);
            sm[(2 * r) * B + tid] = dre * inv;
            sm[(2 * r + 1) * B + tid] = -dim * inv;
        }
        double acc_re = 0.0, acc_im = 0.0;
        for (int g = 0; g < p.G; ++g) {
            double rr = 1.0, ri = 0.0;
            const int32_t *gd = p.group_dens + g * p.dpt;
            for (int k = 0; k < p.dpt; ++k) {
                const int d = gd[k];
                const double xr = sm[(2 * d) * B + tid], xi = sm[(2 * d + 1) * B + tid];
                const double nr = fma(rr, xr, -ri * xi);
                ri = fma(rr, xi, ri * xr);
                rr = nr;
            }
            const double ft = ftcol[g * B + tid];
            acc_re = fma(ft, rr, acc_re);
            acc_im = fma(ft, ri, acc_im);
        }
        if (active && p.out) {
            double2 v;
            v.x = acc_re;
            v.y = acc_im;
            reinterpret_cast<double2 *>(p.out)[static_cast<int64_t>(f) * p.n_e + s] = v;
        }
        if (p.partial) {
            double vr = active ? acc_re : 0.0, vi = active ? acc_im : 0.0;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                vr += __shfl_xor(vr, off, 64);
                vi += __shfl_xor(vi, off, 64);
            }
            if (lane == 0) {
                red[2 * wave] = vr;
                red[2 * wave + 1] = vi;
            }
            __syncthreads();
            if (tid == 0) {
                double sr = 0.0, si = 0.0;
                for (int w = 0; w < nwaves; ++w) {
                    sr += red[2 * w];
                    si += red[2 * w + 1];
                }
                p.partial[(static_cast<int64_t>(blockIdx.x) * p.n_f + f) * 2] = sr;
                p.partial[(static_cast<int64_t>(blockIdx.x) * p.n_f + f) * 2 + 1] = si;
            }
            __syncthreads();
        }
    }
}

}  // namespace ami
