// Device-side building blocks shared by the forward and adjoint evaluators.
//
// Tables are read through the constant address space so that wave-uniform
// reads become scalar loads, and the +-1 coefficient masks are tested with
// scalar bit tests: only the non-zero coefficients cost vector instructions.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <cstdint>
#else
// compiled at run time (hipRTC): no standard headers
typedef __hip_internal::uint64_t uint64_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::uint8_t uint8_t;
typedef __hip_internal::int8_t int8_t;
#endif

// A value made opaque to the optimizer (an empty asm that may change it; no
// instruction): generated code copies a group's operands through it so that
// equal products of different groups are not merged into long-lived values.
#ifndef AMI_OPAQUE
#define AMI_OPAQUE(x) asm volatile("" : "+v"(x))
#endif

// A scheduling fence: the compiler moves no instruction across it.  Generated
// code puts one between chunks of independent work, so that the loads and
// values of a later chunk do not stay live through an earlier one.
#ifndef AMI_SCHED_FENCE
#define AMI_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)
#endif

namespace ami {

typedef const __attribute__((address_space(4))) uint64_t *cu64;
typedef const __attribute__((address_space(4))) uint32_t *cu32;
typedef const __attribute__((address_space(4))) double *cdbl;
typedef const __attribute__((address_space(4))) int32_t *ci32;

constexpr int kMaxExtDev = 4;

// Packed evaluation tables (built by the host, see construct.cpp):
//   leaf[l]  bits 0-15 energies with coefficient +1, bits 16-31 with -1,
//            bit 32 set for a Bose-type leaf (sigma = -1)
//   den[r]   bits 0-15 / 16-31 energy masks as above, bits 32-63 the external
//            frequency coefficients as four int8
//   line[j]  bits 0-15 / 16-31 frequency/momentum slots with coefficient +1/-1
//   term[t]  leaf indices of term t, one byte each; term_sign[t] its prefactor
//   group[g] denominator indices of group g, one byte each;
//            terms of group g are group_start[g] .. group_start[g+1]-1
struct PackedTabs {
    const uint64_t *leaf;
    const uint64_t *den;
    const uint32_t *line;
    const uint64_t *term;
    const double *term_sign;
    const int32_t *group_start;
    const uint64_t *group;
    int L, D, G, T;
    int n_eps, n_int, n_ext, n_freq, n_g, dpt;
    uint32_t fermi_used;    // energies that appear in Fermi-type leaves
    int use_products;       // Fermi leaves from products of exp(beta E_i)
};

// ---- elementary functions -------------------------------------------------

// Reciprocal: hardware estimate refined by two Newton steps (finite, non-zero,
// normal-range arguments).
__device__ __forceinline__ double rcp_nr(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// sin and cos: x = k pi/2 + r with pi/2 split into three parts (33, 33 and 53
// significant bits, so k * part is exact for |k| < 2^20), |r| <= pi/4, and the
// Taylor series of sin (to r^17) and cos (to r^18), whose truncation errors at
// pi/4 are below 1e-19.  Valid for |x| < 1e5; callers route larger arguments
// to the device library.
__device__ __forceinline__ void sincos_red(double x, double &s, double &c) {
    constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
    constexpr double kPio2Hi = 0x1.921fb54400000p+0;
    constexpr double kPio2Mid = 0x1.0b4611a600000p-34;
    constexpr double kPio2Lo = 0x1.3198a2e037073p-69;
    const double kf = __builtin_rint(x * kTwoOverPi);
    double r = fma(-kf, kPio2Hi, x);
    r = fma(-kf, kPio2Mid, r);
    r = fma(-kf, kPio2Lo, r);
    const double z = r * r;
    double ps = 1.0 / 355687428096000.0;          // 1/17!
    ps = fma(ps, z, -1.0 / 1307674368000.0);      // 1/15!
    ps = fma(ps, z, 1.0 / 6227020800.0);          // 1/13!
    ps = fma(ps, z, -1.0 / 39916800.0);           // 1/11!
    ps = fma(ps, z, 1.0 / 362880.0);              // 1/9!
    ps = fma(ps, z, -1.0 / 5040.0);               // 1/7!
    ps = fma(ps, z, 1.0 / 120.0);                 // 1/5!
    ps = fma(ps, z, -1.0 / 6.0);                  // 1/3!
    const double sr = fma(r * z, ps, r);
    double pc = -1.0 / 6402373705728000.0;        // 1/18!
    pc = fma(pc, z, 1.0 / 20922789888000.0);      // 1/16!
    pc = fma(pc, z, -1.0 / 87178291200.0);        // 1/14!
    pc = fma(pc, z, 1.0 / 479001600.0);           // 1/12!
    pc = fma(pc, z, -1.0 / 3628800.0);            // 1/10!
    pc = fma(pc, z, 1.0 / 40320.0);               // 1/8!
    pc = fma(pc, z, -1.0 / 720.0);                // 1/6!
    pc = fma(pc, z, 1.0 / 24.0);                  // 1/4!
    pc = fma(pc, z, -0.5);                        // 1/2!
    const double cr = fma(z, pc, 1.0);
    const int q = static_cast<int>(kf) & 3;
    const double ss = (q & 1) ? cr : sr;
    const double cc = (q & 1) ? sr : cr;
    s = (q & 2) ? -ss : ss;
    c = ((q + 1) & 2) ? -cc : cc;
}

// x - 2 pi n with n = rint(x / 2pi): the same three-part split scaled by 4
// (exact), so the reduction is exact up to the last part for |x| < 6e6.  The
// energies depend on momenta only through cos/sin of integer combinations, so
// reducing every momentum component first keeps every later argument small.
__device__ __forceinline__ double reduce_2pi(double x) {
    constexpr double kOneOver2Pi = 0x1.45f306dc9c883p-3;
    constexpr double k2PiHi = 0x1.921fb54400000p+2;
    constexpr double k2PiMid = 0x1.0b4611a600000p-32;
    constexpr double k2PiLo = 0x1.3198a2e037073p-67;
    const double n = __builtin_rint(x * kOneOver2Pi);
    double r = fma(-n, k2PiHi, x);
    r = fma(-n, k2PiMid, r);
    return fma(-n, k2PiLo, r);
}

// cos alone: x = k pi + r with the same three-part split (doubled: exact),
// |r| <= pi/2, cos x = (-1)^k cos r with the Taylor series of cos to r^20
// (truncation at pi/2 below 2e-17).  Valid for |x| < 1e5.
__device__ __forceinline__ double cos_red(double x) {
    constexpr double kOneOverPi = 0x1.45f306dc9c883p-2;
    constexpr double kPiHi = 0x1.921fb54400000p+1;
    constexpr double kPiMid = 0x1.0b4611a600000p-33;
    constexpr double kPiLo = 0x1.3198a2e037073p-68;
    const double kf = __builtin_rint(x * kOneOverPi);
    double r = fma(-kf, kPiHi, x);
    r = fma(-kf, kPiMid, r);
    r = fma(-kf, kPiLo, r);
    const double z = r * r;
    double p = 1.0 / 2432902008176640000.0;      // 1/20!
    p = fma(p, z, -1.0 / 6402373705728000.0);    // 1/18!
    p = fma(p, z, 1.0 / 20922789888000.0);       // 1/16!
    p = fma(p, z, -1.0 / 87178291200.0);         // 1/14!
    p = fma(p, z, 1.0 / 479001600.0);            // 1/12!
    p = fma(p, z, -1.0 / 3628800.0);             // 1/10!
    p = fma(p, z, 1.0 / 40320.0);                // 1/8!
    p = fma(p, z, -1.0 / 720.0);                 // 1/6!
    p = fma(p, z, 1.0 / 24.0);                   // 1/4!
    p = fma(p, z, -0.5);                         // 1/2!
    const double c = fma(z, p, 1.0);
    return (static_cast<int>(kf) & 1) ? -c : c;
}

// e^z and e^z - 1 from one reduction: z = k ln2 + r with ln2 split in two
// (42 + 53 significant bits, so k * hi is exact for |k| < 2^11), |r| <= ln2/2,
// and p = e^r - 1 by its Taylor series to r^13 (truncation below 2e-17 relative).
// Then t = 2^k (1 + p) and m = 2^k p + (2^k - 1); the last form has no
// cancellation for any k (2^k - 1 is exact), so m keeps full relative precision
// near z = 0 and t near its underflow.  For |z| < 708.
__device__ __forceinline__ void exp_split(double z, double &t, double &m) {
    constexpr double kLog2e = 0x1.71547652b82fep+0;
    constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;
    constexpr double kLn2Lo = 0x1.ef35793c76730p-45;
    const double kf = __builtin_rint(z * kLog2e);
    double r = fma(-kf, kLn2Hi, z);
    r = fma(-kf, kLn2Lo, r);
    double q = 1.0 / 6227020800.0;               // 1/13!
    q = fma(q, r, 1.0 / 479001600.0);            // 1/12!
    q = fma(q, r, 1.0 / 39916800.0);             // 1/11!
    q = fma(q, r, 1.0 / 3628800.0);              // 1/10!
    q = fma(q, r, 1.0 / 362880.0);               // 1/9!
    q = fma(q, r, 1.0 / 40320.0);                // 1/8!
    q = fma(q, r, 1.0 / 5040.0);                 // 1/7!
    q = fma(q, r, 1.0 / 720.0);                  // 1/6!
    q = fma(q, r, 1.0 / 120.0);                  // 1/5!
    q = fma(q, r, 1.0 / 24.0);                   // 1/4!
    q = fma(q, r, 1.0 / 6.0);                    // 1/3!
    q = fma(q, r, 0.5);                          // 1/2!
    const double p = fma(r * r, q, r);
    const double s = __builtin_ldexp(1.0, static_cast<int>(kf));
    t = fma(s, p, s);
    m = fma(s, p, s - 1.0);
}

// A leaf f_sigma(y) = 1/(sigma e^y + 1) and its mirror f_sigma(-y) = 1 - f_sigma(y),
// without overflow and with full relative precision everywhere: with
// t = e^-|y| and m = e^-|y| - 1 (exp_split),
//   Fermi  (sigma = +1): the two values are t/(1+t) and 1/(1+t)
//   Bose-type (-1):      the two values are t/m and -1/m
// (the first of each pair is f at y > 0).  Arguments are clamped at 700 (the
// leaves there are below 1e-304).
__device__ __forceinline__ void leaf_pair(bool bose, double y, double &f, double &fm) {
    double t, m;
    exp_split(-fmin(fabs(y), 700.0), t, m);
    const double r = rcp_nr(bose ? m : 1.0 + t);
    const double small = t * r;            // value on the decaying side
    const double large = bose ? -r : r;    // value on the other side
    f = y > 0.0 ? small : large;
    fm = y > 0.0 ? large : small;
}

// f_sigma(y) and f_sigma'(y) = -f_sigma(y) f_sigma(-y) together: the product of
// the pair is the same whichever value is f, so it needs no select (the same
// bits as -(f * fm) from leaf_pair).
__device__ __forceinline__ void leaf_and_slope(bool bose, double y, double &f, double &dv) {
    double t, m;
    exp_split(-fmin(fabs(y), 700.0), t, m);
    const double r = rcp_nr(bose ? m : 1.0 + t);
    const double small = t * r;
    const double large = bose ? -r : r;
    f = y > 0.0 ? small : large;
    dv = -(small * large);
}

// f_sigma'(y) = -f_sigma(y) f_sigma(-y) in closed form: -t/(1+t)^2 (Fermi) and
// t/m^2 (Bose-type).
__device__ __forceinline__ double leaf_deriv(bool bose, double y) {
    double t, m;
    exp_split(-fmin(fabs(y), 700.0), t, m);
    const double r = rcp_nr(bose ? m : 1.0 + t);
    return bose ? t * r * r : -t * r * r;
}

// A leaf at a complex argument y = yr + i yi (complex energies): with
// z = -y where yr > 0 and z = y elsewhere (so Re z = -|yr| <= 0),
// w = e^z = t (cos zi + i sin zi), t = e^-|yr|, and Q = sigma + w, the leaf is
// w/Q where yr > 0 and sigma/Q elsewhere (the complex form of leaf_pair).  For
// the Bose-type Q = w - 1, its real part is written m cos zi + (cos zi - 1)
// with m = t - 1 (exp_split) and cos zi - 1 = -sin^2 zi/(1 + cos zi) where
// cos zi > 0, so Q keeps full relative precision near y = 0.  The imaginary
// part is reduced modulo 2 pi first (reduce_2pi, exact for |yi| < 6e6).
// leaf_complex_pair also gives f(-y): for -y the same z, w and Q arise (where
// yr = 0, w/Q equals f(-y) at z = y), with the two quotients exchanged:
// f(y) = w/Q and f(-y) = sigma/Q where yr > 0, the other way round elsewhere.
// The adjoint's slope is f'(y) = -f(y) f(-y).
__device__ __forceinline__ void leaf_complex_pair(bool bose, double yr, double yi, double &fr, double &fi,
                                                  double &mr, double &mi) {
    const bool pos = yr > 0.0;
    double t, m, s, c;
    exp_split(-fmin(fabs(yr), 700.0), t, m);
    sincos_red(reduce_2pi(pos ? -yi : yi), s, c);
    const double wr = t * c, wi = t * s;
    double qr;
    if (bose) {
        const double cm1 = c > 0.0 ? -(s * s) / (1.0 + c) : c - 1.0;
        qr = fma(m, c, cm1);
    } else {
        qr = 1.0 + wr;
    }
    const double qi = wi;
    const double r = rcp_nr(fma(qr, qr, qi * qi));
    const double ir = qr * r, ii = -qi * r;                 // 1/Q
    const double ar = fma(wr, ir, -wi * ii), ai = fma(wr, ii, wi * ir);   // w/Q
    const double br = bose ? -ir : ir, bi = bose ? -ii : ii;             // sigma/Q
    fr = pos ? ar : br;
    fi = pos ? ai : bi;
    mr = pos ? br : ar;
    mi = pos ? bi : ai;
}

__device__ __forceinline__ void leaf_complex(bool bose, double yr, double yi, double &fr, double &fi) {
    double mr, mi;
    leaf_complex_pair(bose, yr, yi, fr, fi, mr, mi);
    (void)mr;
    (void)mi;
}

// ---- counter-based random numbers -----------------------------------------

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw, SC'11): each round
// multiplies words 0 and 2 by the two round constants (64-bit products) and
// forms (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key grows by the Weyl
// increments after every round.
__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = static_cast<uint32_t>(p1);
        c[2] = n2;
        c[3] = static_cast<uint32_t>(p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// A uniform momentum component in (-pi, pi) from one 32-bit word:
// (u - 1/2) * 2 pi with u = (word + 1/2) / 2^32 (exact up to the last product).
__device__ __forceinline__ double word_to_momentum(uint32_t w) {
    const double u = (static_cast<double>(w) + 0.5) * 0x1p-32;
    return (u - 0.5) * 0x1.921fb54442d18p+2;
}

// sum_i (+-1) E_i over the bits of two 16-bit masks (scalar bit tests).
template <int NE>
__device__ __forceinline__ double combo(uint32_t pos, uint32_t neg, const double (&E)[NE]) {
    double x = 0.0;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        if (pos & (1u << i)) x += E[i];
        else if (neg & (1u << i)) x -= E[i];
    }
    return x;
}

// Scatter a value into per-energy accumulators with the mask signs.
template <int NE>
__device__ __forceinline__ void combo_adj(uint32_t pos, uint32_t neg, double v, double (&g)[NE]) {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        if (pos & (1u << i)) g[i] += v;
        else if (neg & (1u << i)) g[i] -= v;
    }
}

// A double moved across lanes by one DPP control (all rows and banks, bound
// control on: a lane whose source lane falls outside the wave or the row
// receives 0), as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(static_cast<unsigned>(u)), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(static_cast<unsigned>(u >> 32)), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                          static_cast<unsigned>(lo));
}

// Sum over the 64 lanes of a wave (every lane active), left in lane 63:
// inclusive prefix sums within each row of 16 lanes (row_shr 1, 2, 4, 8), so
// lane 15 of row r holds the row's sum S_r; row_bcast:15 then adds lane 15 of
// the previous row (lane 63: S_3 + S_2), and row_bcast:31 adds lane 31 (by then
// S_1 + S_0) into rows 2-3.  Register moves only: no LDS round trips, no waits.
__device__ __forceinline__ double wave_sum_lane63(double v) {
    v += dpp_move<0x111>(v);   // row_shr:1
    v += dpp_move<0x112>(v);   // row_shr:2
    v += dpp_move<0x114>(v);   // row_shr:4
    v += dpp_move<0x118>(v);   // row_shr:8
    v += dpp_move<0x142>(v);   // row_bcast:15
    v += dpp_move<0x143>(v);   // row_bcast:31
    return v;
}

// The same sum broadcast to every lane (readlane of lane 63).
__device__ __forceinline__ double wave_sum(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, wave_sum_lane63(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(u)), 63));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(u >> 32)), 63));
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

// Element (column c, sample at byte offset off) of a [column][sample]
// workspace with leading dimension ld: the column's base is wave-uniform and
// the offset a 32-bit lane value, which the compiler turns into a load or store
// with a scalar base and no vector address arithmetic.
__device__ __forceinline__ uint64_t ws_column(const double *ws, int64_t ld, int c) {
    const uint64_t p = reinterpret_cast<uint64_t>(ws + c * ld);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(p));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(p >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ double ws_load(const double *ws, int64_t ld, int c, uint32_t off) {
    return *reinterpret_cast<const double *>(ws_column(ws, ld, c) + off);
}

__device__ __forceinline__ void ws_store(double *ws, int64_t ld, int c, uint32_t off, double v) {
    *reinterpret_cast<double *>(ws_column(ws, ld, c) + off) = v;
}

// gfx950 lane exchanges of a double, as two 32-bit halves: swap32 exchanges
// lanes 32-63 of x with lanes 0-31 of y (afterwards x holds the lower halves
// of both, y the upper halves); swap16 exchanges rows 1 and 3 of x with rows 0
// and 2 of y (x then holds the even rows of both, y the odd ones).  Every lane
// of the wave takes part.
__device__ __forceinline__ void swap32(double &x, double &y) {
    const unsigned long long ux = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long uy = __builtin_bit_cast(unsigned long long, y);
    const auto lo = __builtin_amdgcn_permlane32_swap(static_cast<unsigned>(ux), static_cast<unsigned>(uy), false,
                                                     false);
    const auto hi = __builtin_amdgcn_permlane32_swap(static_cast<unsigned>(ux >> 32), static_cast<unsigned>(uy >> 32),
                                                     false, false);
    x = __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<unsigned>(hi[0])) << 32) |
                                       static_cast<unsigned>(lo[0]));
    y = __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<unsigned>(hi[1])) << 32) |
                                       static_cast<unsigned>(lo[1]));
}

__device__ __forceinline__ void swap16(double &x, double &y) {
    const unsigned long long ux = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long uy = __builtin_bit_cast(unsigned long long, y);
    const auto lo = __builtin_amdgcn_permlane16_swap(static_cast<unsigned>(ux), static_cast<unsigned>(uy), false,
                                                     false);
    const auto hi = __builtin_amdgcn_permlane16_swap(static_cast<unsigned>(ux >> 32), static_cast<unsigned>(uy >> 32),
                                                     false, false);
    x = __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<unsigned>(hi[0])) << 32) |
                                       static_cast<unsigned>(lo[0]));
    y = __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<unsigned>(hi[1])) << 32) |
                                       static_cast<unsigned>(lo[1]));
}

// Inclusive prefix sums within each row of 16 lanes: lane 15 of a row holds
// the row's sum.
__device__ __forceinline__ double row_sums(double v) {
    v += dpp_move<0x111>(v);   // row_shr:1
    v += dpp_move<0x112>(v);   // row_shr:2
    v += dpp_move<0x114>(v);   // row_shr:4
    v += dpp_move<0x118>(v);   // row_shr:8
    return v;
}

// The wave's totals of (vr, vi), stored at dst[0] and dst[stride]: one swap32
// folds the two halves of the wave, leaving vr's 32 partial sums in rows 0-1
// and vi's in rows 2-3; after the row sums, row_bcast:15 adds row 0 into lane
// 31 (vr's total) and row 2 into lane 63 (vi's total).  Register moves only:
// no LDS, no barrier.
__device__ __forceinline__ void wave_store2(double vr, double vi, int lane, double *dst, int64_t stride) {
    swap32(vr, vi);
    double v = row_sums(vr + vi);
    v += dpp_move<0x142>(v);   // row_bcast:15
    if (lane == 31) dst[0] = v;
    if (lane == 63) dst[stride] = v;
}

// The wave's totals of four values, v_k stored at *p_k (a null p_k: not
// stored).  swap32 on the pairs (v0, v1) and (v2, v3) folds the halves of the
// wave; swap16 on the two results folds row pairs, leaving one value per row
// (rows 0-3: v0, v2, v1, v3), whose row sums end in lanes 15, 31, 47 and 63.
__device__ __forceinline__ void wave_store4(double v0, double v1, double v2, double v3, int lane, double *p0,
                                            double *p1, double *p2, double *p3) {
    swap32(v0, v1);
    swap32(v2, v3);
    double x = v0 + v1, y = v2 + v3;
    swap16(x, y);
    const double v = row_sums(x + y);
    double *const p = lane == 15 ? p0 : lane == 31 ? p2 : lane == 47 ? p1 : lane == 63 ? p3 : nullptr;
    if (p) *p = v;
}

__device__ __forceinline__ void block_sum2(double vr, double vi, double *red, int tid, int B, double *dst) {
    vr = wave_sum(vr);
    vi = wave_sum(vi);
    const int wave = tid >> 6, nwaves = B >> 6;
    if ((tid & 63) == 0) {
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
        dst[0] = sr;
        dst[1] = si;
    }
    __syncthreads();
}

}  // namespace ami
