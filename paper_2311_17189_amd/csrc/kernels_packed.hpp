// Packed evaluators: forward and adjoint of the AMI solution (Burke & LeBlanc,
// arXiv 2311.17189, Sec. 2.2-2.3) over the bit-mask tables of PackedTabs.
//
// One lane per energy sample.  Template parameters NE, NI, DPT bound the
// number of energies, leaves per term and denominators per term; with EXACT
// they are the diagram's own values and every loop over them is unrolled with
// no run-time guard (self-energy shapes are instantiated that way).
//
// Per-lane LDS columns (slot s of lane tid at sm[s * B + tid]):
//   forward: leaves [0, L) -- reused for the denominator reciprocals
//            [0, 2D) of the current frequency row --, then the group sums FT_g.
//   adjoint: leaves F [0,L), FT_g [L, L+G), dL/dFT_g [L+G, L+2G), then a
//            region of max(2D, L) slots: reciprocals during the frequency
//            loop, leaf cotangents afterwards.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.hpp"
#include "kargs.hpp"

namespace ami {


// ---- inputs ---------------------------------------------------------------

template <int NE, bool EXACT>
__device__ __forceinline__ void load_energies(const KArgs &a, int64_t sc, double (&E)[NE]) {
    const int ne = EXACT ? NE : a.tb.n_eps;
    const double *row = a.energies + sc * a.stride_s;
#pragma unroll
    for (int i = 0; i < NE; ++i) E[i] = (i < ne) ? row[i * a.stride_i] : 0.0;
}

// E_j = -eps(K_j) = 2t(cos K_jx + cos K_jy) + mu with K_j = sum_l alpha_jl k_l
// (Sec. 5.2); sK/cs keep sin K_j per component and the cosine sum for the
// chain rule of the adjoint.
template <int NE, int NI, bool EXACT, bool KEEP>
__device__ __forceinline__ void hubbard_energies(const KArgs &a, int64_t sc, double (&E)[NE],
                                                 double (&sKx)[NE], double (&sKy)[NE], double (&cs)[NE]) {
    const int ni = EXACT ? NI : a.tb.n_int;
    const int ng = EXACT ? NE : a.tb.n_g;
    const int nx = a.tb.n_ext;
    // momenta reduced into [-pi, pi] (q is reduced on the host): every K_j then
    // stays within the range of the reduced sin/cos
    double kx[NI > 0 ? NI : 1], ky[NI > 0 ? NI : 1];
    const double *row = a.k + sc * a.stride_k;
#pragma unroll
    for (int l = 0; l < NI; ++l) {
        kx[l] = (l < ni) ? reduce_2pi(row[2 * l]) : 0.0;
        ky[l] = (l < ni) ? reduce_2pi(row[2 * l + 1]) : 0.0;
    }
    cu32 line = (cu32)(a.tb.line);
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        E[j] = 0.0;
        if (KEEP) {
            sKx[j] = 0.0;
            sKy[j] = 0.0;
            cs[j] = 0.0;
        }
        if (j < ng) {
            const uint32_t w = line[j];
            const uint32_t pos = w & 0xffffu, neg = w >> 16;
            double Kx = 0.0, Ky = 0.0;
#pragma unroll
            for (int l = 0; l < NI; ++l) {
                if (pos & (1u << l)) {
                    Kx += kx[l];
                    Ky += ky[l];
                } else if (neg & (1u << l)) {
                    Kx -= kx[l];
                    Ky -= ky[l];
                }
            }
            for (int x = 0; x < nx; ++x) {
                if ((pos >> (ni + x)) & 1u) {
                    Kx += a.q[2 * x];
                    Ky += a.q[2 * x + 1];
                } else if ((neg >> (ni + x)) & 1u) {
                    Kx -= a.q[2 * x];
                    Ky -= a.q[2 * x + 1];
                }
            }
            double cx, cy;
            if (KEEP) {            // the adjoint needs sin K as well
                double sx, sy;
                sincos_red(Kx, sx, cx);
                sincos_red(Ky, sy, cy);
                sKx[j] = sx;
                sKy[j] = sy;
                cs[j] = cx + cy;
            } else {
                cx = cos_red(Kx);
                cy = cos_red(Ky);
            }
            E[j] = fma(2.0 * a.hop_t, cx + cy, a.mu);
        }
    }
}

// ---- leaves and Fermi-tree group sums ------------------------------------

template <int NE>
__device__ __forceinline__ void eval_leaves(const KArgs &a, const double (&E)[NE], double *sm, int tid, int B) {
    const PackedTabs &tb = a.tb;
    cu64 leaf = (cu64)(tb.leaf);
    double u[NE];
    bool prod = tb.use_products != 0;
    if (prod) {
        // exp(beta E_i) of the energies used by Fermi leaves; a leaf is then
        // f = 1/(1 + P/N) = N/(N + P) with P (N) the product over its +1 (-1)
        // energies.  Each factor is kept below e^(600/NE) so no product overflows.
        bool big = false;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            u[i] = 1.0;
            if ((tb.fermi_used >> i) & 1u) {
                const double y = a.beta * E[i];
                big |= fabs(y) > 600.0 / NE;
                double m;
                exp_split(fmax(fmin(y, 650.0), -650.0), u[i], m);
            }
        }
        prod = !__any(big);
    }
    for (int l = 0; l < tb.L; ++l) {
        const uint64_t w = leaf[l];
        const uint32_t pos = static_cast<uint32_t>(w) & 0xffffu;
        const uint32_t neg = (static_cast<uint32_t>(w) >> 16) & 0xffffu;
        double v, vm;
        if ((w >> 32) & 1u) {
            leaf_pair(true, a.beta * (combo<NE>(pos, neg, E) + a.e_reg), v, vm);
        } else if (prod) {
            double P = 1.0, N = 1.0;
#pragma unroll
            for (int i = 0; i < NE; ++i) {
                if (pos & (1u << i)) P *= u[i];
                else if (neg & (1u << i)) N *= u[i];
            }
            v = N * rcp_nr(N + P);
        } else {
            leaf_pair(false, a.beta * combo<NE>(pos, neg, E), v, vm);
        }
        sm[l * B + tid] = v;
    }
}

template <int NI, bool EXACT>
__device__ __forceinline__ void eval_group_sums(const KArgs &a, const double *sm, double *ftcol, int tid, int B) {
    const PackedTabs &tb = a.tb;
    const int ni = EXACT ? NI : tb.n_int;
    cu64 term = (cu64)(tb.term);
    cdbl sign = (cdbl)(tb.term_sign);
    ci32 gs = (ci32)(tb.group_start);
    for (int g = 0; g < tb.G; ++g) {
        const int t0 = gs[g], t1 = gs[g + 1];
        double ft = 0.0;
#pragma unroll 2
        for (int t = t0; t < t1; ++t) {
            const uint64_t w = term[t];
            double prod = 1.0;
#pragma unroll
            for (int j = 0; j < NI; ++j)
                if (j < ni) prod *= sm[static_cast<int>((w >> (8 * j)) & 0xffu) * B + tid];
            ft = fma(sign[t], prod, ft);
        }
        ftcol[g * B + tid] = ft;
    }
}

// Complex reciprocals of every distinct denominator at one frequency row.
template <int NE>
__device__ __forceinline__ void eval_dens(const KArgs &a, const double (&E)[NE], const double *wre,
                                          const double *wim, double *rho, int tid, int B) {
    const PackedTabs &tb = a.tb;
    cu64 den = (cu64)(tb.den);
    const int nx = tb.n_ext;
    for (int r = 0; r < tb.D; ++r) {
        const uint64_t w = den[r];
        double re = combo<NE>(static_cast<uint32_t>(w) & 0xffffu, (static_cast<uint32_t>(w) >> 16) & 0xffffu, E);
        double im = 0.0;
        for (int x = 0; x < nx; ++x) {
            const int c = static_cast<int8_t>((w >> (32 + 8 * x)) & 0xffu);
            if (c == 1) {
                re += wre[x];
                im += wim[x];
            } else if (c == -1) {
                re -= wre[x];
                im -= wim[x];
            } else if (c != 0) {
                re = fma(static_cast<double>(c), wre[x], re);
                im = fma(static_cast<double>(c), wim[x], im);
            }
        }
        const double inv = rcp_nr(fma(re, re, im * im));
        rho[(2 * r) * B + tid] = re * inv;
        rho[(2 * r + 1) * B + tid] = -im * inv;
    }
}

__device__ __forceinline__ void load_freq(const KArgs &a, int f, double *wre, double *wim) {
    const int nx = a.tb.n_ext;
    cdbl fr = (cdbl)(a.ext_freqs);
#pragma unroll
    for (int x = 0; x < kMaxExtDev; ++x) {
        wre[x] = (x < nx) ? fr[2 * (f * nx + x)] : 0.0;
        wim[x] = (x < nx) ? fr[2 * (f * nx + x) + 1] : 0.0;
    }
}

// ---- forward ---------------------------------------------------------------

// One tile of B = blockDim.x samples starting at tile * B; `sm` is the
// block's dynamic LDS (a.slots columns plus the reduction area).  Shared by
// the per-diagram kernel and the persistent batch kernel, so both compute
// every output with the same instructions.
template <int NE, int NI, int DPT, bool EXACT, bool HUB>
__device__ __forceinline__ void fwd_tile(const KArgs &a, int64_t tile, double *sm) {
    const int tid = threadIdx.x, B = blockDim.x;
    const int64_t s = tile * B + tid;
    const bool active = s < a.n_e;
    const int64_t sc = active ? s : a.n_e - 1;
    const PackedTabs &tb = a.tb;
    const int dpt = EXACT ? DPT : tb.dpt;

    double E[NE];
    if constexpr (HUB) {
        double d0[NE], d1[NE], d2[NE];
        hubbard_energies<NE, NI, EXACT, false>(a, sc, E, d0, d1, d2);
    } else {
        load_energies<NE, EXACT>(a, sc, E);
    }
    eval_leaves<NE>(a, E, sm, tid, B);
    const int region_a = (tb.L > 2 * tb.D) ? tb.L : 2 * tb.D;
    double *ftcol = sm + region_a * B;
    eval_group_sums<NI, EXACT>(a, sm, ftcol, tid, B);

    double *red = sm + a.slots * B;
    cu64 grp = (cu64)(tb.group);
    for (int f = 0; f < a.n_f; ++f) {
        double wre[kMaxExtDev], wim[kMaxExtDev];
        load_freq(a, f, wre, wim);
        eval_dens<NE>(a, E, wre, wim, sm, tid, B);
        double acc_re = 0.0, acc_im = 0.0;
        for (int g = 0; g < tb.G; ++g) {
            const uint64_t w = grp[g];
            double rr = 1.0, ri = 0.0;
#pragma unroll
            for (int k = 0; k < DPT; ++k) {
                if (k < dpt) {
                    const int d = static_cast<int>((w >> (8 * k)) & 0xffu);
                    const double xr = sm[(2 * d) * B + tid], xi = sm[(2 * d + 1) * B + tid];
                    const double nr = fma(rr, xr, -ri * xi);
                    ri = fma(rr, xi, ri * xr);
                    rr = nr;
                }
            }
            const double ft = ftcol[g * B + tid];
            acc_re = fma(ft, rr, acc_re);
            acc_im = fma(ft, ri, acc_im);
        }
        if (active && a.out) {
            double2 v;
            v.x = acc_re;
            v.y = acc_im;
            reinterpret_cast<double2 *>(a.out)[static_cast<int64_t>(f) * a.n_e + s] = v;
        }
        if (a.partial)
            block_sum2(active ? acc_re : 0.0, active ? acc_im : 0.0, red, tid, B,
                       a.partial + (tile * a.n_f + f) * 2);
    }
}

template <int NE, int NI, int DPT, bool EXACT, bool HUB>
__global__ __launch_bounds__(256) void ami_fwd_packed(KArgs a) {
    extern __shared__ double sm[];
    fwd_tile<NE, NI, DPT, EXACT, HUB>(a, blockIdx.x, sm);
}

// ---- adjoint ---------------------------------------------------------------
// For L = Re sum_{f,s} conj(c[f,s]) I[f,s] with I = sum_g FT_g R_g, R_g = prod_{k in g} rho_k,
// rho = 1/D:
//   dL/dFT_g = Re sum_f conj(c_f) R_g(f)
//   dR_g/dD_k = -rho_k R_g   (one such term per occurrence of k in g), so with
//   u_g = -FT_g conj(c) R_g:  dL/dE_i += e_ki Re(u_g rho_k),  dL/dw += conj(a_k u_g rho_k)
//   dL/df_l  = sum_{t ni l} dL/dFT_g(t) s_t prod_{k in t, k != l} f_k
//   f_sigma'(y) = -f_sigma(y) f_sigma(-y):  dL/dE_i += dL/df_l beta e_li f'(y_l),
//                                           dL/dbeta += dL/df_l x_l f'(y_l)
//   momentum path: dE_j/dK_jc = -2t sin K_jc, dK_j/dk_l = alpha_jl, dE_j/dmu = 1,
//   dE_j/dt = 2(cos K_jx + cos K_jy).
// The leaves of a term are distinct (checked by the host when packing), so the
// cotangent updates of one term are read together and written together.

template <int NE, int NI, int DPT, bool EXACT, bool HUB>
__global__ __launch_bounds__(256) void ami_adj_packed(KArgs a) {
    extern __shared__ double sm[];
    const int tid = threadIdx.x, B = blockDim.x;
    const int64_t s = static_cast<int64_t>(blockIdx.x) * B + tid;
    const bool active = s < a.n_e;
    const int64_t sc = active ? s : a.n_e - 1;
    const PackedTabs &tb = a.tb;
    const int ni = EXACT ? NI : tb.n_int;
    const int dpt = EXACT ? DPT : tb.dpt;
    const int L = tb.L, G = tb.G, nx = tb.n_ext;

    double E[NE], sKx[NE], sKy[NE], cs[NE];
    if constexpr (HUB) {
        hubbard_energies<NE, NI, EXACT, true>(a, sc, E, sKx, sKy, cs);
    } else {
        load_energies<NE, EXACT>(a, sc, E);
    }
    // LDS columns: F leaves, FT group sums, FTB their cotangents, X reciprocals
    // (during the frequency loop) then leaf cotangents
    double *F = sm;
    double *FT = sm + L * B;
    double *FTB = sm + (L + G) * B;
    double *X = sm + (L + 2 * G) * B;
    double *red = sm + a.slots * B;
    eval_leaves<NE>(a, E, F, tid, B);
    eval_group_sums<NI, EXACT>(a, F, FT, tid, B);
    for (int g = 0; g < G; ++g) FTB[g * B + tid] = 0.0;

    double gE[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) gE[i] = 0.0;
    cu64 grp = (cu64)(tb.group);
    cu64 den = (cu64)(tb.den);
    double *gp = a.gpartial + static_cast<int64_t>(blockIdx.x) * (kAdjScalars + 2 * a.n_f * nx);

    for (int f = 0; f < a.n_f; ++f) {
        double cr = 0.0, ci = 0.0;
        if (active) {
            if (a.g_out) {
                cr = a.g_out[2 * (static_cast<int64_t>(f) * a.n_e + s)];
                ci = a.g_out[2 * (static_cast<int64_t>(f) * a.n_e + s) + 1];
            }
            if (a.g_sum) {
                cr += a.g_sum[2 * f];
                ci += a.g_sum[2 * f + 1];
            }
        }
        double wre[kMaxExtDev], wim[kMaxExtDev];
        load_freq(a, f, wre, wim);
        eval_dens<NE>(a, E, wre, wim, X, tid, B);
        double gwr[kMaxExtDev], gwi[kMaxExtDev];
#pragma unroll
        for (int x = 0; x < kMaxExtDev; ++x) {
            gwr[x] = 0.0;
            gwi[x] = 0.0;
        }
        double acc_re = 0.0, acc_im = 0.0;      // forward value, when asked for
        for (int g = 0; g < G; ++g) {
            const uint64_t w = grp[g];
            double xr[DPT > 0 ? DPT : 1], xi[DPT > 0 ? DPT : 1];
            double Rr = 1.0, Ri = 0.0;
#pragma unroll
            for (int k = 0; k < DPT; ++k) {
                xr[k] = 0.0;
                xi[k] = 0.0;
                if (k < dpt) {
                    const int d = static_cast<int>((w >> (8 * k)) & 0xffu);
                    xr[k] = X[(2 * d) * B + tid];
                    xi[k] = X[(2 * d + 1) * B + tid];
                    const double nr = fma(Rr, xr[k], -Ri * xi[k]);
                    Ri = fma(Rr, xi[k], Ri * xr[k]);
                    Rr = nr;
                }
            }
            FTB[g * B + tid] += fma(cr, Rr, ci * Ri);
            // u = -FT conj(c) R
            const double ft = FT[g * B + tid];
            acc_re = fma(ft, Rr, acc_re);
            acc_im = fma(ft, Ri, acc_im);
            const double qr = ft * cr, qi = -ft * ci;
            const double ur = -fma(qr, Rr, -qi * Ri), ui = -fma(qr, Ri, qi * Rr);
#pragma unroll
            for (int k = 0; k < DPT; ++k) {
                if (k < dpt) {
                    const int d = static_cast<int>((w >> (8 * k)) & 0xffu);
                    const double dr = fma(ur, xr[k], -ui * xi[k]);
                    const double di = fma(ur, xi[k], ui * xr[k]);
                    const uint64_t dw = den[d];
                    combo_adj<NE>(static_cast<uint32_t>(dw) & 0xffffu, (static_cast<uint32_t>(dw) >> 16) & 0xffffu,
                                  dr, gE);
                    for (int x = 0; x < nx; ++x) {
                        const int c = static_cast<int8_t>((dw >> (32 + 8 * x)) & 0xffu);
                        if (c == 1) {
                            gwr[x] += dr;
                            gwi[x] += di;
                        } else if (c == -1) {
                            gwr[x] -= dr;
                            gwi[x] -= di;
                        } else if (c != 0) {
                            gwr[x] = fma(static_cast<double>(c), dr, gwr[x]);
                            gwi[x] = fma(static_cast<double>(c), di, gwi[x]);
                        }
                    }
                }
            }
        }
        for (int x = 0; x < nx; ++x)
            block_sum2(active ? gwr[x] : 0.0, active ? -gwi[x] : 0.0, red, tid, B,
                       gp + kAdjScalars + 2 * (f * nx + x));
        if (active && a.out) {
            double2 v;
            v.x = acc_re;
            v.y = acc_im;
            reinterpret_cast<double2 *>(a.out)[static_cast<int64_t>(f) * a.n_e + s] = v;
        }
        if (a.partial)
            block_sum2(active ? acc_re : 0.0, active ? acc_im : 0.0, red, tid, B,
                       a.partial + (static_cast<int64_t>(blockIdx.x) * a.n_f + f) * 2);
    }

    // leaf cotangents (the X region is free now)
    double *FB = X;
    for (int l = 0; l < L; ++l) FB[l * B + tid] = 0.0;
    cu64 term = (cu64)(tb.term);
    cdbl sign = (cdbl)(tb.term_sign);
    ci32 gs = (ci32)(tb.group_start);
    for (int g = 0; g < G; ++g) {
        const double fb = FTB[g * B + tid];
        const int t0 = gs[g], t1 = gs[g + 1];
        for (int t = t0; t < t1; ++t) {
            const uint64_t w = term[t];
            double fv[NI > 0 ? NI : 1], acc[NI > 0 ? NI : 1], pre[NI + 1];
            int li[NI > 0 ? NI : 1];
            pre[0] = fb * sign[t];
#pragma unroll
            for (int j = 0; j < NI; ++j) {
                li[j] = 0;
                fv[j] = 1.0;
                acc[j] = 0.0;
                pre[j + 1] = pre[j];
                if (j < ni) {
                    li[j] = static_cast<int>((w >> (8 * j)) & 0xffu);
                    fv[j] = F[li[j] * B + tid];
                    acc[j] = FB[li[j] * B + tid];
                    pre[j + 1] = pre[j] * fv[j];
                }
            }
            double suf = 1.0;
#pragma unroll
            for (int j = NI - 1; j >= 0; --j) {
                if (j < ni) {
                    acc[j] = fma(pre[j], suf, acc[j]);
                    suf *= fv[j];
                }
            }
#pragma unroll
            for (int j = 0; j < NI; ++j)
                if (j < ni) FB[li[j] * B + tid] = acc[j];
        }
    }
    cu64 leaf = (cu64)(tb.leaf);
    double gbeta = 0.0;
    for (int l = 0; l < L; ++l) {
        const uint64_t w = leaf[l];
        const uint32_t pos = static_cast<uint32_t>(w) & 0xffffu;
        const uint32_t neg = (static_cast<uint32_t>(w) >> 16) & 0xffffu;
        const bool bose = (w >> 32) & 1u;
        double x = combo<NE>(pos, neg, E);
        if (bose) x += a.e_reg;
        const double fb = FB[l * B + tid] * leaf_deriv(bose, a.beta * x);
        combo_adj<NE>(pos, neg, fb * a.beta, gE);
        gbeta = fma(fb, x, gbeta);
    }

    double gmu = 0.0, gt = 0.0;
    if constexpr (HUB) {
        const int ng = EXACT ? NE : tb.n_g;
        double gkx[NI > 0 ? NI : 1], gky[NI > 0 ? NI : 1];
#pragma unroll
        for (int l = 0; l < NI; ++l) {
            gkx[l] = 0.0;
            gky[l] = 0.0;
        }
        cu32 line = (cu32)(tb.line);
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            if (j < ng) {
                gmu += gE[j];
                gt = fma(gE[j], 2.0 * cs[j], gt);
                const double kbx = -2.0 * a.hop_t * gE[j] * sKx[j];
                const double kby = -2.0 * a.hop_t * gE[j] * sKy[j];
                const uint32_t w = line[j];
                const uint32_t pos = w & 0xffffu, neg = w >> 16;
#pragma unroll
                for (int l = 0; l < NI; ++l) {
                    if (pos & (1u << l)) {
                        gkx[l] += kbx;
                        gky[l] += kby;
                    } else if (neg & (1u << l)) {
                        gkx[l] -= kbx;
                        gky[l] -= kby;
                    }
                }
            }
        }
        if (active && a.grad_k) {
            double *row = a.grad_k + s * (2 * ni);
#pragma unroll
            for (int l = 0; l < NI; ++l)
                if (l < ni) {
                    row[2 * l] = gkx[l];
                    row[2 * l + 1] = gky[l];
                }
        }
    }
    if (active && a.grad_e) {
        const int ne = EXACT ? NE : tb.n_eps;
        double *row = a.grad_e + s * ne;
#pragma unroll
        for (int i = 0; i < NE; ++i)
            if (i < ne) row[i] = gE[i];
    }
    block_sum2(active ? gbeta : 0.0, active ? gmu : 0.0, red, tid, B, gp);
    block_sum2(active ? gt : 0.0, 0.0, red, tid, B, gp + 2);
}

}  // namespace ami
