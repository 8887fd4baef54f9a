// Tile functions of the run-time specialized evaluator (compiled with
// hipRTC), in namespace amijit, after the generated functions of one diagram
// (the sizes, tables and straight-line functions its comment lists).  No
// include guard: a module holding several diagrams (the persistent batch)
// includes it once per diagram, with amijit defined to that diagram's own
// namespace and the AMI_JIT_* settings of that diagram.

#include "kargs.hpp"

namespace amijit {

// The argument block's type as the tile functions see it: a kernel argument
// (ami::KArgs), or, in the persistent batch, a block in constant memory
// (AMI_JIT_ARGS: the constant address space, so that the compiler may read
// its fields again wherever it needs them instead of holding them).
#ifdef AMI_JIT_ARGS
using KArgs = AMI_JIT_ARGS;
#else
using ami::KArgs;
#endif

constexpr int NXA = NX > 0 ? NX : 1;
constexpr int NIA = NI > 0 ? NI : 1;
constexpr int NGA = NG > 0 ? NG : 1;
static_assert(!AMI_JIT_HUB || NG == NE, "momentum input: one energy per line");

// Adjoint LDS columns per lane: the chain-rule values of the momentum input
// (3 NG), then, with AMI_JIT_PARK_DV, the leaf derivatives f'(y_l) (L).
constexpr int kParkChain = AMI_JIT_HUB ? 3 * NG : 0;
constexpr bool kParkDv = AMI_JIT_PARK_DV;
static_assert(!(kParkDv && kTaylor), "Taylor-coefficient leaves keep their slopes out of the park area");
constexpr int kParkCols = kParkChain + (kParkDv ? L : 0);

// Gradient rows (W doubles per sample, row-major, the wave's 64 consecutive
// samples contiguous in memory) leave through LDS, so that each store
// instruction writes 64 consecutive doubles instead of one row piece per lane
// at a W-double stride: lane i puts its row at elements i W .. i W + W - 1 of
// the wave's staging area, then takes back elements 64 j + i.  Element e sits
// at stage[e + e / 64] (one pad double per 64, which keeps both passes free of
// bank conflicts).  The staging areas (65 W doubles per wave) reuse the park
// area once every wave of the block has read its parked values.
template <int W>
constexpr bool kStageFits = kParkCols * AMI_JIT_BLOCK >= (AMI_JIT_BLOCK / 64) * 65 * W;

template <int W>
__device__ __forceinline__ void store_rows_staged(double *stage, int lane, const double (&v)[W], double *dst,
                                                  int64_t n_valid) {
    if constexpr (64 % W == 0) {       // a lane's row does not cross a pad
        double *row = stage + lane * W + ((lane * W) >> 6);
#pragma unroll
        for (int c = 0; c < W; ++c) row[c] = v[c];
    } else {
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const int e = lane * W + c;
            stage[e + (e >> 6)] = v[c];
        }
    }
    __builtin_amdgcn_wave_barrier();
    double x[W];
#pragma unroll
    for (int j = 0; j < W; ++j) x[j] = stage[65 * j + lane];
    if (n_valid >= 64 * W) {           // the whole wave (uniform)
#pragma unroll
        for (int j = 0; j < W; ++j) dst[64 * j + lane] = x[j];
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j)
            if (64 * j + lane < n_valid) dst[64 * j + lane] = x[j];
    }
}

// The momenta of Monte-Carlo sample s: the words of Philox4x32-10 blocks
// b = 0, 1, ... with counter (s mod 2^32, s div 2^32, b, 0) and key = the
// 64-bit seed, component c = 2 l + (0: x, 1: y) from word c, each mapped to
// (-pi, pi) (word_to_momentum).
__device__ __forceinline__ void draw_momenta(const KArgs &a, int64_t s, double (&kx)[NIA], double (&ky)[NIA]) {
    const uint32_t k0 = static_cast<uint32_t>(a.seed), k1 = static_cast<uint32_t>(a.seed >> 32);
#pragma unroll
    for (int b = 0; b < (2 * NI + 3) / 4; ++b) {
        uint32_t c[4] = {static_cast<uint32_t>(s), static_cast<uint32_t>(static_cast<uint64_t>(s) >> 32),
                         static_cast<uint32_t>(b), 0u};
        ami::philox4x32_10(c, k0, k1);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int comp = 4 * b + w;
            if (comp < 2 * NI) {
                const double v = ami::word_to_momentum(c[w]);
                if (comp % 2 == 0) kx[comp / 2] = v;
                else ky[comp / 2] = v;
            }
        }
    }
}

// E from the sample's energies or momenta.  With KEEP (adjoint, momentum
// input) sin K_jx, sin K_jy and cos K_jx + cos K_jy, needed only by the final
// chain rule, are parked in LDS columns (park[(c NG + j) B + tid], c = 0, 1, 2)
// rather than held in registers through the frequency loop; they come from
// sin and cos of the loop momenta by angle addition (line_trig), 2 NI
// reduced sin/cos pairs instead of 2 NG.
// E_j = 2t(cos K_jx + cos K_jy) + mu (Sec. 5.2) from momenta in [-pi, pi]
__device__ __forceinline__ void energies_from(const KArgs &a, const double (&kx)[NIA], const double (&ky)[NIA],
                                              double (&E)[NE]) {
    double Kx[NGA], Ky[NGA];
    lines(kx, ky, a.q, Kx, Ky);
#pragma unroll
    for (int j = 0; j < NG; ++j) E[j] = fma(2.0 * a.hop_t, ami::cos_red(Kx[j]) + ami::cos_red(Ky[j]), a.mu);
}

// The sample's raw inputs: its 2 NI momentum components (momentum input) or
// its NE energies.  Loaded apart from their use so that a kernel can issue
// the loads of a later tile before the arithmetic of the current one.
constexpr int NIN = AMI_JIT_HUB ? 2 * NIA : NE;

template <bool HUB>
__device__ __forceinline__ void load_inputs(const KArgs &a, int64_t sc, double (&in)[NIN]) {
    if constexpr (HUB) {
        const double *row = a.k + sc * a.stride_k;
        if (a.vec_io & 1) {              // one 16-byte load per loop
#pragma unroll
            for (int l = 0; l < NI; ++l) {
                const double2 v = reinterpret_cast<const double2 *>(row)[l];
                in[2 * l] = v.x;
                in[2 * l + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int l = 0; l < 2 * NI; ++l) in[l] = row[l];
        }
    } else {
        const double *row = a.energies + sc * a.stride_s;
#pragma unroll
        for (int i = 0; i < NE; ++i) in[i] = row[i * a.stride_i];
    }
}

template <bool HUB, bool KEEP>
__device__ __forceinline__ void energies(const KArgs &a, const double (&in)[NIN], double (&E)[NE], double *park) {
    if constexpr (HUB) {
        // E_j = 2t(cos K_jx + cos K_jy) + mu (Sec. 5.2), momenta reduced into [-pi, pi]
        double kx[NIA], ky[NIA];
#pragma unroll
        for (int l = 0; l < NI; ++l) {
            kx[l] = ami::reduce_2pi(in[2 * l]);
            ky[l] = ami::reduce_2pi(in[2 * l + 1]);
        }
        if constexpr (!KEEP) {
            energies_from(a, kx, ky, E);
            return;
        }
        // sin and cos of the loop momenta, then of the lines by angle addition
        double sx[NIA], cx[NIA], sy[NIA], cy[NIA], Sx[NGA], Cx[NGA], Sy[NGA], Cy[NGA];
#pragma unroll
        for (int l = 0; l < NI; ++l) {
            ami::sincos_red(kx[l], sx[l], cx[l]);
            ami::sincos_red(ky[l], sy[l], cy[l]);
        }
        line_trig(sx, cx, sy, cy, a.qs, a.qc, Sx, Cx, Sy, Cy);
        const int tid = threadIdx.x, B = blockDim.x;
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            const double cs = Cx[j] + Cy[j];
            park[j * B + tid] = Sx[j];
            park[(NG + j) * B + tid] = Sy[j];
            park[(2 * NG + j) * B + tid] = cs;
            E[j] = fma(2.0 * a.hop_t, cs, a.mu);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NE; ++i) E[i] = in[i];
    }
}

template <bool HUB, bool KEEP>
__device__ __forceinline__ void energies(const KArgs &a, int64_t sc, double (&E)[NE], double *park) {
    double in[NIN];
    load_inputs<HUB>(a, sc, in);
    energies<HUB, KEEP>(a, in, E, park);
}

__device__ __forceinline__ void load_freq(const KArgs &a, int f, double (&wr)[NXA], double (&wi)[NXA]) {
    ami::cdbl fr = (ami::cdbl)(a.ext_freqs);      // wave-uniform: scalar loads
#pragma unroll
    for (int x = 0; x < NXA; ++x) {
        wr[x] = (x < NX) ? fr[2 * (f * NX + x)] : 0.0;
        wi[x] = (x < NX) ? fr[2 * (f * NX + x) + 1] : 0.0;
    }
}

// complex reciprocals rho_k = 1/D_k of every distinct denominator
__device__ __forceinline__ void reciprocals(const double (&E)[NE], const double (&wr)[NXA], const double (&wi)[NXA],
                                            double (&xr)[D], double (&xi)[D]) {
    double dr[D], di[D];
    den_args(E, wr, wi, dr, di);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double inv = ami::rcp_nr(fma(dr[k], dr[k], di[k] * di[k]));
        xr[k] = dr[k] * inv;
        xi[k] = -di[k] * inv;
    }
}

#if AMI_JIT_KERNELS & 1
// Partial sums are per wave: row r = tile * (B / 64) + wave of the partial
// arrays (column c at [c * nrows + r]), each total written by the one lane
// of the wave that holds it (wave_store2, wave_store4).
// NF1: one frequency row (n_f = 1 known at compile time, so the tile is
// straight-line code the compiler schedules as a whole).
template <bool HUB, bool NF1>
__device__ __forceinline__ void fwd_tile(const KArgs &a, int64_t tile) {
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t row = tile * (B >> 6) + (tid >> 6);
    const int64_t s = tile * B + tid;
    const bool active = s < a.n_e;
    const int64_t sc = active ? s : a.n_e - 1;

    double E[NE];
    energies<HUB, false>(a, sc, E, nullptr);
    double x[L], F[L], FM[L];
    leaf_args(E, x);
#pragma unroll
    for (int l = 0; l < L; ++l) {
        if (kBose[l]) ami::leaf_pair(true, a.beta * (x[l] + a.e_reg), F[l], FM[l]);
        else ami::leaf_pair(false, a.beta * x[l], F[l], FM[l]);
    }
    taylor_leaves(F, FM, a.beta);
    double FT[G];
    group_sums(F, FT);

    const int nf = NF1 ? 1 : a.n_f;
    for (int f = 0; f < nf; ++f) {
        double wr[NXA], wi[NXA], xr[D], xi[D];
        load_freq(a, f, wr, wi);
        reciprocals(E, wr, wi, xr, xi);
        double acc_re, acc_im;
        groups_combine(xr, xi, FT, acc_re, acc_im);
        if (active && a.out) {
            double2 v;
            v.x = acc_re;
            v.y = acc_im;
            reinterpret_cast<double2 *>(a.out)[static_cast<int64_t>(f) * a.n_e + s] = v;
        }
        if (a.partial)
            ami::wave_store2(active ? acc_re : 0.0, active ? acc_im : 0.0, lane, a.partial + 2 * f * a.nrows + row,
                             a.nrows);
    }
}

#endif

#if AMI_JIT_KERNELS & (2 | 128)
// The gradients of one sample once its energies' cotangent gE and its dL/dbeta
// contribution are complete: on the momentum input the chain rule through
// dE_j/dK_j = -2t sin K_j to the momenta (the trig values parked by
// energies<HUB, true>), the per-sample gradient rows (staged through the park
// area when they fit), and the wave sums of dL/dbeta, dL/dmu, dL/dt at the
// partial-sum row gp.  s_blk: the block's first sample; s_end: one past the
// last sample the launch writes.
template <bool HUB>
__device__ __forceinline__ void adj_grad_end(const KArgs &a, int64_t s_blk, int64_t s_end, bool active, double *gp,
                                             double *park, double (&gE)[NE], double gbeta) {
#pragma clang fp contract(fast)
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t s = s_blk + tid;

    double gmu = 0.0, gt = 0.0;
    if constexpr (HUB) {
        double gx[NGA], gy[NGA], gkx[NIA], gky[NIA];
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            gmu += gE[j];
            gt = fma(gE[j], 2.0 * park[(2 * NG + j) * B + tid], gt);
            gx[j] = -2.0 * a.hop_t * gE[j] * park[j * B + tid];
            gy[j] = -2.0 * a.hop_t * gE[j] * park[(NG + j) * B + tid];
        }
#pragma unroll
        for (int l = 0; l < NIA; ++l) {
            gkx[l] = 0.0;
            gky[l] = 0.0;
        }
        line_scatter(gx, gy, gkx, gky);
        if constexpr (kStageFits<2 * NI>) {
            if (a.grad_k) {
                double g[2 * NI];
#pragma unroll
                for (int l = 0; l < NI; ++l) {
                    g[2 * l] = gkx[l];
                    g[2 * l + 1] = gky[l];
                }
                __syncthreads();                    // every wave has read its parked values
                const int wave = tid >> 6;
                const int64_t s0 = s_blk + (wave << 6);
                store_rows_staged<2 * NI>(park + wave * 65 * (2 * NI), lane, g, a.grad_k + s0 * (2 * NI),
                                          (s_end - s0) * (2 * NI));
            }
        } else if (active && a.grad_k) {
            double *row = a.grad_k + s * (2 * NI);
            if (a.vec_io & 2) {
#pragma unroll
                for (int l = 0; l < NI; ++l) {
                    double2 g2;
                    g2.x = gkx[l];
                    g2.y = gky[l];
                    reinterpret_cast<double2 *>(row)[l] = g2;
                }
            } else {
#pragma unroll
                for (int l = 0; l < NI; ++l) {
                    row[2 * l] = gkx[l];
                    row[2 * l + 1] = gky[l];
                }
            }
        }
    }
    if constexpr (kStageFits<NE>) {
        if (a.grad_e) {
            __syncthreads();                        // every wave is done with the park area
            const int wave = tid >> 6;
            const int64_t s0 = s_blk + (wave << 6);
            store_rows_staged<NE>(park + wave * 65 * NE, lane, gE, a.grad_e + s0 * NE, (s_end - s0) * NE);
        }
    } else if (active && a.grad_e) {
        double *row = a.grad_e + s * NE;
#pragma unroll
        for (int i = 0; i < NE; ++i) row[i] = gE[i];
    }
    ami::wave_store4(active ? gbeta : 0.0, active ? gmu : 0.0, active ? gt : 0.0, 0.0, lane, gp, gp + a.nrows,
                     gp + 2 * a.nrows, nullptr);
}

// The end of the adjoint of one sample once its leaf cotangents FB are known:
// the leaves' derivatives (f'(y) from Dv or the park area) scattered to the
// energies and to beta, then adj_grad_end.  gE holds the energies' cotangent
// so far.  A solution with Taylor-coefficient leaves recomputes the plain
// leaf pairs here and takes dT/dx and dT/dbeta from taylor_slopes.
template <bool HUB>
__device__ __forceinline__ void adj_leaf_end(const KArgs &a, int64_t s_blk, int64_t s_end, bool active, double *gp,
                                             double *park, const double (&E)[NE], const double (&Dv)[kParkDv ? 1 : L],
                                             const double (&FB)[L], double (&gE)[NE]) {
#pragma clang fp contract(fast)
    const int tid = threadIdx.x, B = blockDim.x;
    double gbeta = 0.0, v[L], x[L];
    leaf_args(E, x);
    if constexpr (kTaylor) {
        double F[L], FM[L], DX[L], DB[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (kBose[l]) x[l] += a.e_reg;
            ami::leaf_pair(kBose[l], a.beta * x[l], F[l], FM[l]);
        }
        taylor_slopes(F, FM, x, a.beta, DX, DB);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            v[l] = FB[l] * DX[l];
            gbeta = fma(FB[l], DB[l], gbeta);
        }
        (void)Dv;
        (void)tid;
        (void)B;
    } else {
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (kBose[l]) x[l] += a.e_reg;
            const double fb = FB[l] * (kParkDv ? park[(kParkChain + l) * B + tid] : Dv[kParkDv ? 0 : l]);
            v[l] = fb * a.beta;
            gbeta = fma(fb, x[l], gbeta);
        }
    }
    leaf_scatter(v, gE);
    adj_grad_end<HUB>(a, s_blk, s_end, active, gp, park, gE, gbeta);
}
#endif

#if AMI_JIT_KERNELS & 2
// Adjoint of L = Re sum_{f,s} conj(c[f,s]) I[f,s] (the packed adjoint's
// derivation), with the denominator cotangents collected per distinct
// denominator: dL/dD_k = -rho_k sum_{g contains k} FT_g conj(c) R_g.
// The leaf arguments x_l are recomputed after the frequency loop instead of
// being kept live through it.
template <bool HUB, bool NF1>
__device__ __forceinline__ void adj_tile(const KArgs &a, int64_t blk, double *park, const double (&in)[NIN]) {
    // multiply-add pairs written here fuse with those of the reverse-sweep
    // functions; the values come from functions compiled without contraction
    // and from explicit fma, so they match the forward kernel bit for bit
#pragma clang fp contract(fast)
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t row = blk * (B >> 6) + (tid >> 6);
    const int64_t s = blk * B + tid;
    const bool active = s < a.n_e;

    double E[NE];
    energies<HUB, HUB>(a, in, E, park);
    double F[L], Dv[kParkDv ? 1 : L];
    {
        double x[L];
        leaf_args(E, x);
        if constexpr (kTaylor) {                // the forward's leaves; slopes at the end
            double FM[L];
#pragma unroll
            for (int l = 0; l < L; ++l) {
                if (kBose[l]) x[l] += a.e_reg;
                ami::leaf_pair(kBose[l], a.beta * x[l], F[l], FM[l]);
            }
            taylor_leaves(F, FM, a.beta);
        } else {
#pragma unroll
            for (int l = 0; l < L; ++l) {
                if (kBose[l]) x[l] += a.e_reg;
                double dv;                      // f'(y) = -f(y) f(-y)
                ami::leaf_and_slope(kBose[l], a.beta * x[l], F[l], dv);
                if constexpr (kParkDv) park[(kParkChain + l) * B + tid] = dv;
                else Dv[kParkDv ? 0 : l] = dv;
            }
        }
    }
    double FT[G], FTB[G];
    group_sums(F, FT);
#pragma unroll
    for (int g = 0; g < G; ++g) FTB[g] = 0.0;
    double gE[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) gE[i] = 0.0;
    double *gp = a.gpartial + row;                   // column c at gp[c * nrows]

    const int nf = NF1 ? 1 : a.n_f;       // NF1: straight-line code for one frequency row
    for (int f = 0; f < nf; ++f) {
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
        double wr[NXA], wi[NXA], xr[D], xi[D], Rr[G], Ri[G];
        load_freq(a, f, wr, wi);
        reciprocals(E, wr, wi, xr, xi);
        group_products(xr, xi, Rr, Ri);
        double acc_re = 0.0, acc_im = 0.0, ur[G], ui[G];
        if constexpr (kNestedGroups) groups_combine(xr, xi, FT, acc_re, acc_im);   // the forward's values
#pragma unroll
        for (int g = 0; g < G; ++g) {
            FTB[g] += fma(cr, Rr[g], ci * Ri[g]);
            if constexpr (!kNestedGroups) {
                acc_re = fma(FT[g], Rr[g], acc_re);
                acc_im = fma(FT[g], Ri[g], acc_im);
            }
            const double qr = FT[g] * cr, qi = -FT[g] * ci;       // u = -FT conj(c) R
            ur[g] = -fma(qr, Rr[g], -qi * Ri[g]);
            ui[g] = -fma(qr, Ri[g], qi * Rr[g]);
        }
        double Ur[D], Ui[D], dR[D], dI[D];
        den_cotangents(ur, ui, Ur, Ui);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            dR[k] = fma(Ur[k], xr[k], -Ui[k] * xi[k]);
            dI[k] = fma(Ur[k], xi[k], Ui[k] * xr[k]);
        }
        double gwr[NXA], gwi[NXA];
#pragma unroll
        for (int xx = 0; xx < NXA; ++xx) {
            gwr[xx] = 0.0;
            gwi[xx] = 0.0;
        }
        den_scatter(dR, dI, gE, gwr, gwi);
        if (active && a.out) {
            double2 v;
            v.x = acc_re;
            v.y = acc_im;
            reinterpret_cast<double2 *>(a.out)[static_cast<int64_t>(f) * a.n_e + s] = v;
        }
        // this row's per-wave sums, four values per reduction: the frequency
        // cotangents (columns kAdjScalars + 2 (f NX + x) and the next), then
        // the forward values' row sums (when asked for)
        constexpr int NV = 2 * NX + 2, NV4 = (NV + 3) / 4 * 4;
        double vv[NV4];
        double *pp[NV4];
#pragma unroll
        for (int xx = 0; xx < NX; ++xx) {
            vv[2 * xx] = active ? gwr[xx] : 0.0;
            vv[2 * xx + 1] = active ? -gwi[xx] : 0.0;
            pp[2 * xx] = gp + (ami::kAdjScalars + 2 * (f * NX + xx)) * a.nrows;
            pp[2 * xx + 1] = pp[2 * xx] + a.nrows;
        }
        vv[2 * NX] = active ? acc_re : 0.0;
        vv[2 * NX + 1] = active ? acc_im : 0.0;
        pp[2 * NX] = a.partial ? a.partial + 2 * f * a.nrows + row : nullptr;
        pp[2 * NX + 1] = a.partial ? pp[2 * NX] + a.nrows : nullptr;
#pragma unroll
        for (int c = NV; c < NV4; ++c) {
            vv[c] = 0.0;
            pp[c] = nullptr;
        }
#pragma unroll
        for (int c = 0; c < NV4; c += 4)
            ami::wave_store4(vv[c], vv[c + 1], vv[c + 2], vv[c + 3], lane, pp[c], pp[c + 1], pp[c + 2], pp[c + 3]);
    }

    double FB[L];
#pragma unroll
    for (int l = 0; l < L; ++l) FB[l] = 0.0;
    leaf_cotangents(F, FTB, FB);
    adj_leaf_end<HUB>(a, blk * B, a.n_e, active, gp, park, E, Dv, FB, gE);
}
#endif

#if AMI_JIT_KERNELS & 4
// Monte-Carlo integration over the internal momenta (Sec. 5.2, the row
// average of Sec. 2.3): sample s = blockIdx.x B + tid + i gridDim.x B draws
// its 2 NI components from Philox blocks (counter (s mod 2^32, s div 2^32,
// b, 0), key = the 64-bit seed), evaluates every frequency row, and
// accumulates sum Re I, sum Im I, sum (Re I)^2, sum (Im I)^2 per lane; the
// wave sums go to row block * (B / 64) + wave, columns 4 f .. 4 f + 3, of the
// partial sums.  Nothing per sample touches HBM.
template <bool HUB>
__device__ __forceinline__ void mc_block(const KArgs &a) {
    static_assert(HUB, "Monte-Carlo integration samples momenta");
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t row = static_cast<int64_t>(blockIdx.x) * (B >> 6) + (tid >> 6);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * B;
    double acc[4][ami::kMcMaxFreqs];
#pragma unroll
    for (int f = 0; f < ami::kMcMaxFreqs; ++f) acc[0][f] = acc[1][f] = acc[2][f] = acc[3][f] = 0.0;
    for (int64_t s = static_cast<int64_t>(blockIdx.x) * B + tid; s < a.n_e; s += stride) {
        double kx[NIA], ky[NIA];
        draw_momenta(a, s, kx, ky);
        double E[NE], x[L], F[L], FM[L], FT[G];
        energies_from(a, kx, ky, E);
        leaf_args(E, x);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (kBose[l]) ami::leaf_pair(true, a.beta * (x[l] + a.e_reg), F[l], FM[l]);
            else ami::leaf_pair(false, a.beta * x[l], F[l], FM[l]);
        }
        taylor_leaves(F, FM, a.beta);
        group_sums(F, FT);
#pragma unroll
        for (int f = 0; f < ami::kMcMaxFreqs; ++f) {
            if (f < a.n_f) {
                double wr[NXA], wi[NXA], xr[D], xi[D];
                load_freq(a, f, wr, wi);
                reciprocals(E, wr, wi, xr, xi);
                double re, im;
                groups_combine(xr, xi, FT, re, im);
                acc[0][f] += re;
                acc[1][f] += im;
                acc[2][f] = fma(re, re, acc[2][f]);
                acc[3][f] = fma(im, im, acc[3][f]);
            }
        }
    }
#pragma unroll
    for (int f = 0; f < ami::kMcMaxFreqs; ++f) {
        if (f < a.n_f) {
            double *dst = a.partial + 4 * f * a.nrows + row;
            ami::wave_store4(acc[0][f], acc[1][f], acc[2][f], acc[3][f], lane, dst, dst + a.nrows,
                             dst + 2 * a.nrows, dst + 3 * a.nrows);
        }
    }
}

#endif

#if AMI_JIT_KERNELS & 16
// Two-pass forward, first pass (large solutions: their group sums do not fit
// in registers through a frequency loop): one lane per sample of the chunk,
// energies, leaves and group sums, each group sum stored to the workspace as
// soon as it is formed, the energies beside them.  Lanes past the chunk write
// rows of the workspace that nothing reads (ld is a multiple of the block).
template <bool HUB>
__device__ __forceinline__ void sums_tile(const KArgs &a, int64_t tile) {
    const int tid = threadIdx.x, B = blockDim.x;
    const int64_t i = tile * B + tid;
    const int64_t sc = a.s0 + (i < a.n_chunk ? i : a.n_chunk - 1);
    double E[NE];
    if (HUB && a.mc) {                  // Monte Carlo: the momenta of sample sc drawn here
        double kx[NIA], ky[NIA];
        draw_momenta(a, sc, kx, ky);
        energies_from(a, kx, ky, E);
    } else {
        energies<HUB, false>(a, sc, E, nullptr);
    }
    double x[L], F[L], FM[L];
    leaf_args(E, x);
#pragma unroll
    for (int l = 0; l < L; ++l) {
        if (kBose[l]) ami::leaf_pair(true, a.beta * (x[l] + a.e_reg), F[l], FM[l]);
        else ami::leaf_pair(false, a.beta * x[l], F[l], FM[l]);
    }
    taylor_leaves(F, FM, a.beta);
    const uint32_t off = static_cast<uint32_t>(i) * 8u;   // i < ld <= 2^28 (host bound)
    group_sums_store(F, a.work, a.ld, off);
#pragma unroll
    for (int j = 0; j < NE; ++j) ami::ws_store(a.work, a.ld, G + j, off, E[j]);
}
#endif

#if AMI_JIT_KERNELS & 32
// Two-pass forward, second pass: block (tile, f) evaluates frequency row f
// for the samples of one tile of the chunk: the reciprocals of every distinct
// denominator from the stored energies, then sum_g FT_g R_g nested over the
// reciprocals, each stored FT_g read where the nesting needs it.  Values go to out[f][s0 + i]; the
// wave sums to row (s0 / B + tile) * (B / 64) + wave, columns 2 f, 2 f + 1.
__device__ __forceinline__ void freq_tile(const KArgs &a, int64_t tile, int f) {
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t i = tile * B + tid;
    const bool active = i < a.n_chunk;
    const int64_t row = (a.s0 / B + tile) * (B >> 6) + (tid >> 6);
    double E[NE];
    const uint32_t off = static_cast<uint32_t>(i) * 8u;   // i < ld <= 2^28 (host bound)
#pragma unroll
    for (int j = 0; j < NE; ++j) E[j] = ami::ws_load(a.work, a.ld, G + j, off);
    double wr[NXA], wi[NXA], xr[D], xi[D];
    load_freq(a, f, wr, wi);
    reciprocals(E, wr, wi, xr, xi);
    double acc_re = 0.0, acc_im = 0.0;
    group_accumulate(xr, xi, a.work, a.ld, off, acc_re, acc_im);
    if (a.mc) {                         // Monte Carlo: sums and sums of squares per frequency row
        const double re = active ? acc_re : 0.0, im = active ? acc_im : 0.0;
        double *dst = a.partial + 4 * f * a.nrows + row;
        ami::wave_store4(re, im, re * re, im * im, lane, dst, dst + a.nrows, dst + 2 * a.nrows, dst + 3 * a.nrows);
        return;
    }
    if (active && a.out) {
        double2 v;
        v.x = acc_re;
        v.y = acc_im;
        reinterpret_cast<double2 *>(a.out)[static_cast<int64_t>(f) * a.n_e + a.s0 + i] = v;
    }
    if (a.partial)
        ami::wave_store2(active ? acc_re : 0.0, active ? acc_im : 0.0, lane, a.partial + 2 * f * a.nrows + row,
                         a.nrows);
}
#endif

#if AMI_JIT_KERNELS & 64
// Adjoint of a large solution, frequency pass (after the two-pass forward's
// first pass stored FT_g and E_j): one lane per sample of the chunk, every
// frequency row in turn.  Per row the generated adj_freq_row forms, chunk of
// groups by chunk, the reciprocals, each group's R_g, the value sum_g FT_g R_g,
// FTB_g += Re(conj(c) R_g) (stored in the workspace) and the denominators'
// cotangents scattered to the energies (gE, stored after the last row) and to
// the frequencies.  Values go to out[f][s]; the wave sums of dL/dw and of the
// values to row (s0 / B + tile) * (B / 64) + wave of the partial sums, in the
// columns of the one-pass adjoint.
__device__ __forceinline__ void adjf_tile(const KArgs &a, int64_t tile) {
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t i = tile * B + tid;
    const bool active = i < a.n_chunk;
    const int64_t s = a.s0 + i;
    const int64_t row = (a.s0 / B + tile) * (B >> 6) + (tid >> 6);
    const uint32_t off = static_cast<uint32_t>(i) * 8u;   // i < ld <= 2^28 (host bound)
    double E[NE], gE[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        E[j] = ami::ws_load(a.work, a.ld, G + j, off);
        gE[j] = 0.0;
    }
    double *gp = a.gpartial + row;
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
        double wr[NXA], wi[NXA], gwr[NXA], gwi[NXA];
        load_freq(a, f, wr, wi);
#pragma unroll
        for (int xx = 0; xx < NXA; ++xx) {
            gwr[xx] = 0.0;
            gwi[xx] = 0.0;
        }
        double acc_re = 0.0, acc_im = 0.0;
        // the offset made opaque per row: the workspace addresses of every
        // column are then formed where they are used, not hoisted out of the
        // loop and held (64-bit per lane and column) through it
        uint32_t off_f = off;
        AMI_OPAQUE(off_f);
        if (f == 0) adj_freq_row<true>(E, wr, wi, cr, ci, a.work, a.ld, off_f, acc_re, acc_im, gE, gwr, gwi);
        else adj_freq_row<false>(E, wr, wi, cr, ci, a.work, a.ld, off_f, acc_re, acc_im, gE, gwr, gwi);
        if (active && a.out) {
            double2 v;
            v.x = acc_re;
            v.y = acc_im;
            reinterpret_cast<double2 *>(a.out)[static_cast<int64_t>(f) * a.n_e + s] = v;
        }
        constexpr int NV = 2 * NX + 2, NV4 = (NV + 3) / 4 * 4;
        double vv[NV4];
        double *pp[NV4];
#pragma unroll
        for (int xx = 0; xx < NX; ++xx) {
            vv[2 * xx] = active ? gwr[xx] : 0.0;
            vv[2 * xx + 1] = active ? -gwi[xx] : 0.0;
            pp[2 * xx] = gp + (ami::kAdjScalars + 2 * (f * NX + xx)) * a.nrows;
            pp[2 * xx + 1] = pp[2 * xx] + a.nrows;
        }
        vv[2 * NX] = active ? acc_re : 0.0;
        vv[2 * NX + 1] = active ? acc_im : 0.0;
        pp[2 * NX] = a.partial ? a.partial + 2 * f * a.nrows + row : nullptr;
        pp[2 * NX + 1] = a.partial ? pp[2 * NX] + a.nrows : nullptr;
#pragma unroll
        for (int c = NV; c < NV4; ++c) {
            vv[c] = 0.0;
            pp[c] = nullptr;
        }
#pragma unroll
        for (int c = 0; c < NV4; c += 4)
            ami::wave_store4(vv[c], vv[c + 1], vv[c + 2], vv[c + 3], lane, pp[c], pp[c + 1], pp[c + 2], pp[c + 3]);
    }
#pragma unroll
    for (int j = 0; j < NE; ++j) ami::ws_store(a.work, a.ld, G + NE + j, off, gE[j]);
}
#endif

#if AMI_JIT_KERNELS & 128
// Adjoint of a large solution, leaf pass (after the frequency pass): one lane
// per sample of the chunk.  The energies again from the sample's inputs (on
// the momentum input with the chain rule's trig values parked), then the
// generated leaf_pass (leaves, their cotangents by the reverse sweep of every
// group's nested sum against the stored FTB_g, their scatter to the energies
// and beta) on the stored energy cotangents of the denominators, then the end
// of the one-pass adjoint (adj_grad_end).
template <bool HUB>
__device__ __forceinline__ void adjl_tile(const KArgs &a, int64_t tile, double *park) {
    const int tid = threadIdx.x, B = blockDim.x;
    const int64_t i = tile * B + tid;
    const bool active = i < a.n_chunk;
    const int64_t row = (a.s0 / B + tile) * (B >> 6) + (tid >> 6);
    const uint32_t off = static_cast<uint32_t>(i) * 8u;
    double in[NIN];
    load_inputs<HUB>(a, a.s0 + (active ? i : a.n_chunk - 1), in);
    double E[NE];
    energies<HUB, HUB>(a, in, E, park);
    double gE[NE], gbeta = 0.0;
#pragma unroll
    for (int j = 0; j < NE; ++j) gE[j] = ami::ws_load(a.work, a.ld, G + NE + j, off);
    leaf_pass(E, a.beta, a.e_reg, a.work, a.ld, off, gE, gbeta);
    adj_grad_end<HUB>(a, a.s0 + tile * B, a.s0 + a.n_chunk, active, a.gpartial + row, park, gE, gbeta);
}
#endif

#if AMI_JIT_KERNELS & 8
// Forward at complex energies (energy input; interleaved complex128 rows,
// strides in complex elements).  The leaf arguments and the energy part of
// the denominators are linear in E, so leaf_args and den_args serve the real
// and the imaginary parts alike; the leaves are complex (leaf_complex) and so
// are the group sums FT_g, each multiplied by R_g in complex arithmetic.
__device__ __forceinline__ void cfwd_tile(const KArgs &a, int64_t tile) {
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t row = tile * (B >> 6) + (tid >> 6);
    const int64_t s = tile * B + tid;
    const bool active = s < a.n_e;
    const int64_t sc = active ? s : a.n_e - 1;

    double Er[NE], Ei[NE];
    const double *erow = a.energies + 2 * sc * a.stride_s;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        Er[i] = erow[2 * i * a.stride_i];
        Ei[i] = erow[2 * i * a.stride_i + 1];
    }
    double FTr[G], FTi[G], dEi[D];
    {
        double xr[L], xi[L], Fr[L], Fi[L];
        leaf_args(Er, xr);
        leaf_args(Ei, xi);
#pragma unroll
        for (int l = 0; l < L; ++l)
            ami::leaf_complex(kBose[l], a.beta * (kBose[l] ? xr[l] + a.e_reg : xr[l]), a.beta * xi[l], Fr[l], Fi[l]);
        group_sums_c(Fr, Fi, FTr, FTi);
        double zr[NXA], zi[NXA], unused[D];
#pragma unroll
        for (int x = 0; x < NXA; ++x) zr[x] = zi[x] = 0.0;
        den_args(Ei, zr, zi, dEi, unused);          // e_k . Im E
    }

    for (int f = 0; f < a.n_f; ++f) {
        double wr[NXA], wi[NXA], dr[D], di[D], xr[D], xi[D], Rr[G], Ri[G];
        load_freq(a, f, wr, wi);
        den_args(Er, wr, wi, dr, di);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double im = di[k] + dEi[k];
            const double inv = ami::rcp_nr(fma(dr[k], dr[k], im * im));
            xr[k] = dr[k] * inv;
            xi[k] = -im * inv;
        }
        group_products(xr, xi, Rr, Ri);
        double acc_re = 0.0, acc_im = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            acc_re = fma(FTr[g], Rr[g], fma(-FTi[g], Ri[g], acc_re));
            acc_im = fma(FTr[g], Ri[g], fma(FTi[g], Rr[g], acc_im));
        }
        if (active && a.out) {
            double2 v;
            v.x = acc_re;
            v.y = acc_im;
            reinterpret_cast<double2 *>(a.out)[static_cast<int64_t>(f) * a.n_e + s] = v;
        }
        if (a.partial)
            ami::wave_store2(active ? acc_re : 0.0, active ? acc_im : 0.0, lane, a.partial + 2 * f * a.nrows + row,
                             a.nrows);
    }
}
#endif

#if AMI_JIT_KERNELS & 512
// Two-pass forward at complex energies, first pass (solutions too large for
// cfwd_tile): one lane per sample of the chunk, complex leaves and group sums,
// each group sum stored as soon as it is formed (real part in column g,
// imaginary part in column G + g), the energies beside them (real parts in
// columns 2 G + j, imaginary parts in 2 G + NE + j).  Lanes past the chunk
// write rows that nothing reads (ld is a multiple of the block).
__device__ __forceinline__ void csums_tile(const KArgs &a, int64_t tile) {
    const int tid = threadIdx.x, B = blockDim.x;
    const int64_t i = tile * B + tid;
    const int64_t sc = a.s0 + (i < a.n_chunk ? i : a.n_chunk - 1);
    double Er[NE], Ei[NE];
    const double *erow = a.energies + 2 * sc * a.stride_s;
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        Er[j] = erow[2 * j * a.stride_i];
        Ei[j] = erow[2 * j * a.stride_i + 1];
    }
    double xr[L], xi[L], Fr[L], Fi[L];
    leaf_args(Er, xr);
    leaf_args(Ei, xi);
#pragma unroll
    for (int l = 0; l < L; ++l)
        ami::leaf_complex(kBose[l], a.beta * (kBose[l] ? xr[l] + a.e_reg : xr[l]), a.beta * xi[l], Fr[l], Fi[l]);
    const uint32_t off = static_cast<uint32_t>(i) * 8u;   // i < ld <= 2^28 (host bound)
    group_sums_c_store(Fr, Fi, a.work, a.ld, off);
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        ami::ws_store(a.work, a.ld, 2 * G + j, off, Er[j]);
        ami::ws_store(a.work, a.ld, 2 * G + NE + j, off, Ei[j]);
    }
}
#endif

#if AMI_JIT_KERNELS & 1024
// Two-pass forward at complex energies, second pass: block (tile, f) as
// freq_tile, from the stored complex energies (the imaginary parts enter the
// denominators' imaginary parts) and the stored complex group sums.
__device__ __forceinline__ void cfreq_tile(const KArgs &a, int64_t tile, int f) {
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t i = tile * B + tid;
    const bool active = i < a.n_chunk;
    const int64_t row = (a.s0 / B + tile) * (B >> 6) + (tid >> 6);
    const uint32_t off = static_cast<uint32_t>(i) * 8u;   // i < ld <= 2^28 (host bound)
    double Er[NE], Ei[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        Er[j] = ami::ws_load(a.work, a.ld, 2 * G + j, off);
        Ei[j] = ami::ws_load(a.work, a.ld, 2 * G + NE + j, off);
    }
    double wr[NXA], wi[NXA], dr[D], di[D], xr[D], xi[D];
    {
        double zr[NXA], zi[NXA], unused[D];
#pragma unroll
        for (int x = 0; x < NXA; ++x) zr[x] = zi[x] = 0.0;
        den_args(Ei, zr, zi, xi, unused);              // e_k . Im E (in xi for now)
    }
    load_freq(a, f, wr, wi);
    den_args(Er, wr, wi, dr, di);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double im = di[k] + xi[k];
        const double inv = ami::rcp_nr(fma(dr[k], dr[k], im * im));
        xr[k] = dr[k] * inv;
        xi[k] = -im * inv;
    }
    double acc_re = 0.0, acc_im = 0.0;
    group_accumulate_c(xr, xi, a.work, a.ld, off, acc_re, acc_im);
    if (active && a.out) {
        double2 v;
        v.x = acc_re;
        v.y = acc_im;
        reinterpret_cast<double2 *>(a.out)[static_cast<int64_t>(f) * a.n_e + a.s0 + i] = v;
    }
    if (a.partial)
        ami::wave_store2(active ? acc_re : 0.0, active ? acc_im : 0.0, lane, a.partial + 2 * f * a.nrows + row,
                         a.nrows);
}
#endif

#if AMI_JIT_KERNELS & 2048
// Adjoint at complex energies in passes, frequency pass (after the complex
// two-pass forward's first pass stored FT_g and E_j): as adjf_tile, with the
// generated cadj_freq_row; the energies' complex cotangents from the
// denominators go to columns 2 G + 2 NE + j (real) and 2 G + 3 NE + j.
__device__ __forceinline__ void cadjf_tile(const KArgs &a, int64_t tile) {
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t i = tile * B + tid;
    const bool active = i < a.n_chunk;
    const int64_t s = a.s0 + i;
    const int64_t row = (a.s0 / B + tile) * (B >> 6) + (tid >> 6);
    const uint32_t off = static_cast<uint32_t>(i) * 8u;   // i < ld <= 2^28 (host bound)
    double Er[NE], Ei[NE], gEr[NE], gEi[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        Er[j] = ami::ws_load(a.work, a.ld, 2 * G + j, off);
        Ei[j] = ami::ws_load(a.work, a.ld, 2 * G + NE + j, off);
        gEr[j] = gEi[j] = 0.0;
    }
    double *gp = a.gpartial + row;
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
        double wr[NXA], wi[NXA], gwr[NXA], gwi[NXA];
        load_freq(a, f, wr, wi);
#pragma unroll
        for (int xx = 0; xx < NXA; ++xx) {
            gwr[xx] = 0.0;
            gwi[xx] = 0.0;
        }
        double acc_re = 0.0, acc_im = 0.0;
        uint32_t off_f = off;                // opaque per row, as in adjf_tile
        AMI_OPAQUE(off_f);
        if (f == 0)
            cadj_freq_row<true>(Er, Ei, wr, wi, cr, ci, a.work, a.ld, off_f, acc_re, acc_im, gEr, gEi, gwr, gwi);
        else
            cadj_freq_row<false>(Er, Ei, wr, wi, cr, ci, a.work, a.ld, off_f, acc_re, acc_im, gEr, gEi, gwr, gwi);
        if (active && a.out) {
            double2 v;
            v.x = acc_re;
            v.y = acc_im;
            reinterpret_cast<double2 *>(a.out)[static_cast<int64_t>(f) * a.n_e + s] = v;
        }
        constexpr int NV = 2 * NX + 2, NV4 = (NV + 3) / 4 * 4;
        double vv[NV4];
        double *pp[NV4];
#pragma unroll
        for (int xx = 0; xx < NX; ++xx) {
            vv[2 * xx] = active ? gwr[xx] : 0.0;
            vv[2 * xx + 1] = active ? -gwi[xx] : 0.0;
            pp[2 * xx] = gp + (ami::kAdjScalars + 2 * (f * NX + xx)) * a.nrows;
            pp[2 * xx + 1] = pp[2 * xx] + a.nrows;
        }
        vv[2 * NX] = active ? acc_re : 0.0;
        vv[2 * NX + 1] = active ? acc_im : 0.0;
        pp[2 * NX] = a.partial ? a.partial + 2 * f * a.nrows + row : nullptr;
        pp[2 * NX + 1] = a.partial ? pp[2 * NX] + a.nrows : nullptr;
#pragma unroll
        for (int c = NV; c < NV4; ++c) {
            vv[c] = 0.0;
            pp[c] = nullptr;
        }
#pragma unroll
        for (int c = 0; c < NV4; c += 4)
            ami::wave_store4(vv[c], vv[c + 1], vv[c + 2], vv[c + 3], lane, pp[c], pp[c + 1], pp[c + 2], pp[c + 3]);
    }
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        ami::ws_store(a.work, a.ld, 2 * G + 2 * NE + j, off, gEr[j]);
        ami::ws_store(a.work, a.ld, 2 * G + 3 * NE + j, off, gEi[j]);
    }
}
#endif

#if AMI_JIT_KERNELS & 4096
// Adjoint at complex energies in passes, leaf pass: one lane per sample of
// the chunk; the energies from the workspace, the generated cleaf_pass on the
// stored energy cotangents of the denominators, then the complex gradient row
// (interleaved) and the per-wave sum of dL/dbeta.
__device__ __forceinline__ void cadjl_tile(const KArgs &a, int64_t tile) {
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t i = tile * B + tid;
    const bool active = i < a.n_chunk;
    const int64_t s = a.s0 + i;
    const int64_t row = (a.s0 / B + tile) * (B >> 6) + (tid >> 6);
    const uint32_t off = static_cast<uint32_t>(i) * 8u;
    double Er[NE], Ei[NE], gEr[NE], gEi[NE], gbeta = 0.0;
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        Er[j] = ami::ws_load(a.work, a.ld, 2 * G + j, off);
        Ei[j] = ami::ws_load(a.work, a.ld, 2 * G + NE + j, off);
        gEr[j] = ami::ws_load(a.work, a.ld, 2 * G + 2 * NE + j, off);
        gEi[j] = ami::ws_load(a.work, a.ld, 2 * G + 3 * NE + j, off);
    }
    cleaf_pass(Er, Ei, a.beta, a.e_reg, a.work, a.ld, off, gEr, gEi, gbeta);
    if (active && a.grad_e) {
        double *grow = a.grad_e + 2 * s * NE;
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            grow[2 * j] = gEr[j];
            grow[2 * j + 1] = gEi[j];
        }
    }
    double *gp = a.gpartial + row;
    ami::wave_store4(active ? gbeta : 0.0, 0.0, 0.0, 0.0, lane, gp, gp + a.nrows, gp + 2 * a.nrows, nullptr);
}
#endif

#if AMI_JIT_KERNELS & 256
// The complex adjoint's leaf slopes S_l (2 L doubles per lane) wait in LDS
// through the reverse sweep where they fit in 80 KB per block (two blocks of
// 256 lanes per CU) and the real adjoint parks its slopes too.
constexpr bool kParkS = kParkDv && 2 * L * AMI_JIT_BLOCK * 8 <= 80 * 1024;

// Adjoint at complex energies (energy input; interleaved complex128 rows,
// strides in complex elements; grad_e complex [n_e][NE]).  Every quantity is
// analytic in E, so the cotangents are complex, in the convention
// Xbar = dL/dRe X + i dL/dIm X of the real objective L = Re sum conj(c) I;
// through z = h(x), xbar += zbar conj(h'(x)).  Per frequency row:
// FTbar_g += c conj(R_g) and, for the denominators, U_k rho_k = conj(Dbar_k)
// with u_g = -FT_g conj(c) R_g as in the real adjoint (its real part scatters
// to Re Ebar and w, minus its imaginary part to Im Ebar).  After the rows the
// leaves are formed again (with f(-y)): Fbar from leaf_cotangents_c at
// conj(F), V_l = Fbar_l conj(f'(y_l)) with f' = -f(y) f(-y) (conj(f') waiting
// in the park area where kParkS), so that
// xbar_l = beta V_l and dL/dbeta = sum_l Re(conj(V_l) x_l).  The values are
// formed as in cfwd_tile.
__device__ __forceinline__ void cadj_tile(const KArgs &a, int64_t blk, double *park) {
#pragma clang fp contract(fast)
    const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63;
    const int64_t row = blk * (B >> 6) + (tid >> 6);
    const int64_t s = blk * B + tid;
    const bool active = s < a.n_e;
    const int64_t sc = active ? s : a.n_e - 1;

    double Er[NE], Ei[NE];
    const double *erow = a.energies + 2 * sc * a.stride_s;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        Er[i] = erow[2 * i * a.stride_i];
        Ei[i] = erow[2 * i * a.stride_i + 1];
    }
    double FTr[G], FTi[G], dEi[D];
    {
        double xr[L], xi[L], Fr[L], Fi[L];
        leaf_args(Er, xr);
        leaf_args(Ei, xi);
#pragma unroll
        for (int l = 0; l < L; ++l)
            ami::leaf_complex(kBose[l], a.beta * (kBose[l] ? xr[l] + a.e_reg : xr[l]), a.beta * xi[l], Fr[l], Fi[l]);
        group_sums_c(Fr, Fi, FTr, FTi);
        double zr[NXA], zi[NXA], unused[D];
#pragma unroll
        for (int x = 0; x < NXA; ++x) zr[x] = zi[x] = 0.0;
        den_args(Ei, zr, zi, dEi, unused);          // e_k . Im E
    }
    double FTBr[G], FTBi[G], gEr[NE], gEi[NE];
#pragma unroll
    for (int g = 0; g < G; ++g) FTBr[g] = FTBi[g] = 0.0;
#pragma unroll
    for (int i = 0; i < NE; ++i) gEr[i] = gEi[i] = 0.0;
    double *gp = a.gpartial + row;                   // column c at gp[c * nrows]

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
        double wr[NXA], wi[NXA], dr[D], di[D], xr[D], xi[D], Rr[G], Ri[G];
        load_freq(a, f, wr, wi);
        den_args(Er, wr, wi, dr, di);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double im = di[k] + dEi[k];
            const double inv = ami::rcp_nr(fma(dr[k], dr[k], im * im));
            xr[k] = dr[k] * inv;
            xi[k] = -im * inv;
        }
        group_products(xr, xi, Rr, Ri);
        double acc_re = 0.0, acc_im = 0.0, ur[G], ui[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            acc_re = fma(FTr[g], Rr[g], fma(-FTi[g], Ri[g], acc_re));
            acc_im = fma(FTr[g], Ri[g], fma(FTi[g], Rr[g], acc_im));
            FTBr[g] += fma(cr, Rr[g], ci * Ri[g]);                  // c conj(R)
            FTBi[g] += fma(ci, Rr[g], -cr * Ri[g]);
            const double qr = fma(FTr[g], cr, FTi[g] * ci);         // q = FT conj(c)
            const double qi = fma(FTi[g], cr, -FTr[g] * ci);
            ur[g] = -fma(qr, Rr[g], -qi * Ri[g]);                   // u = -q R
            ui[g] = -fma(qr, Ri[g], qi * Rr[g]);
        }
        double Ur[D], Ui[D], dR[D], dI[D], ndI[D];
        den_cotangents(ur, ui, Ur, Ui);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            dR[k] = fma(Ur[k], xr[k], -Ui[k] * xi[k]);
            dI[k] = fma(Ur[k], xi[k], Ui[k] * xr[k]);
            ndI[k] = -dI[k];
        }
        double gwr[NXA], gwi[NXA], jr[NXA], ji[NXA];
#pragma unroll
        for (int xx = 0; xx < NXA; ++xx) gwr[xx] = gwi[xx] = jr[xx] = ji[xx] = 0.0;
        den_scatter(dR, dI, gEr, gwr, gwi);
        den_scatter(ndI, dR, gEi, jr, ji);          // its frequency part is not used
        if (active && a.out) {
            double2 v;
            v.x = acc_re;
            v.y = acc_im;
            reinterpret_cast<double2 *>(a.out)[static_cast<int64_t>(f) * a.n_e + s] = v;
        }
        // this row's per-wave sums, as adj_tile: dL/dw, then the values' row sums
        constexpr int NV = 2 * NX + 2, NV4 = (NV + 3) / 4 * 4;
        double vv[NV4];
        double *pp[NV4];
#pragma unroll
        for (int xx = 0; xx < NX; ++xx) {
            vv[2 * xx] = active ? gwr[xx] : 0.0;
            vv[2 * xx + 1] = active ? -gwi[xx] : 0.0;
            pp[2 * xx] = gp + (ami::kAdjScalars + 2 * (f * NX + xx)) * a.nrows;
            pp[2 * xx + 1] = pp[2 * xx] + a.nrows;
        }
        vv[2 * NX] = active ? acc_re : 0.0;
        vv[2 * NX + 1] = active ? acc_im : 0.0;
        pp[2 * NX] = a.partial ? a.partial + 2 * f * a.nrows + row : nullptr;
        pp[2 * NX + 1] = a.partial ? pp[2 * NX] + a.nrows : nullptr;
#pragma unroll
        for (int c = NV; c < NV4; ++c) {
            vv[c] = 0.0;
            pp[c] = nullptr;
        }
#pragma unroll
        for (int c = 0; c < NV4; c += 4)
            ami::wave_store4(vv[c], vv[c + 1], vv[c + 2], vv[c + 3], lane, pp[c], pp[c + 1], pp[c + 2], pp[c + 3]);
    }

    // the leaves again: conj(F) for the reverse sweep and S = conj(f'(y)),
    // formed leaf by leaf so that only these three pairs stay live through it
    double gbeta = 0.0;
    {
        // opaque copies of the energies: the compiler cannot match these
        // evaluations with those before the rows and keep their intermediates
        // live through them
        double er[NE], ei[NE];
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            er[j] = Er[j];
            ei[j] = Ei[j];
            AMI_OPAQUE(er[j]);
            AMI_OPAQUE(ei[j]);
        }
        double Fr[L], cFi[L], Sr[kParkS ? 1 : L], Si[kParkS ? 1 : L], FBr[L], FBi[L];
        {
            double xr[L], xi[L];
            leaf_args(er, xr);
            leaf_args(ei, xi);
#pragma unroll
            for (int l = 0; l < L; ++l) {
                double fi, mr, mi;
                ami::leaf_complex_pair(kBose[l], a.beta * (kBose[l] ? xr[l] + a.e_reg : xr[l]), a.beta * xi[l],
                                       Fr[l], fi, mr, mi);
                cFi[l] = -fi;
                const double sr = -fma(Fr[l], mr, -fi * mi);   // conj(f') = -conj(f) conj(f(-y))
                const double si = fma(Fr[l], mi, fi * mr);
                if constexpr (kParkS) {
                    park[(2 * l) * B + tid] = sr;
                    park[(2 * l + 1) * B + tid] = si;
                } else {
                    Sr[kParkS ? 0 : l] = sr;
                    Si[kParkS ? 0 : l] = si;
                }
                FBr[l] = FBi[l] = 0.0;
            }
        }
        leaf_cotangents_c(Fr, cFi, FTBr, FTBi, FBr, FBi);
        double xr[L], xi[L], vr[L], vi[L];
        leaf_args(er, xr);
        leaf_args(ei, xi);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (kBose[l]) xr[l] += a.e_reg;
            const double sr = kParkS ? park[(2 * l) * B + tid] : Sr[kParkS ? 0 : l];
            const double si = kParkS ? park[(2 * l + 1) * B + tid] : Si[kParkS ? 0 : l];
            const double Vr = fma(FBr[l], sr, -FBi[l] * si);         // V = Fbar conj(f')
            const double Vi = fma(FBr[l], si, FBi[l] * sr);
            gbeta = fma(Vr, xr[l], fma(Vi, xi[l], gbeta));
            vr[l] = Vr * a.beta;
            vi[l] = Vi * a.beta;
        }
        leaf_scatter(vr, gEr);
        leaf_scatter(vi, gEi);
    }
    if (active && a.grad_e) {
        double *grow = a.grad_e + 2 * s * NE;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            grow[2 * i] = gEr[i];
            grow[2 * i + 1] = gEi[i];
        }
    }
    ami::wave_store4(active ? gbeta : 0.0, 0.0, 0.0, 0.0, lane, gp, gp + a.nrows, gp + 2 * a.nrows, nullptr);
}
#endif

}  // namespace amijit
