// Argument block of the evaluator kernels (packed, batch and run-time
// specialized): one struct passed by value, with the same layout on the host
// and in code compiled at run time.
#pragma once

#include "device_common.hpp"

namespace ami {

struct KArgs {
    PackedTabs tb;
    int slots;                  // LDS slots per lane (before the reduction area)
    // inputs
    const double *energies;
    int64_t stride_s, stride_i;
    const double *k;
    int64_t stride_k;
    double q[2 * kMaxExtDev];
    double qs[2 * kMaxExtDev], qc[2 * kMaxExtDev];   // sin q, cos q (set on the host)
    int q_big;                  // unused (q is reduced modulo 2 pi on the host)
    double hop_t, mu;
    const double *ext_freqs;
    int n_f;
    double beta, e_reg;
    int64_t n_e;
    // forward outputs
    double *out;
    double *partial;            // [grid][n_f][2]
    // adjoint inputs/outputs
    const double *g_out;        // complex [n_f][n_e] or NULL
    const double *g_sum;        // complex [n_f] or NULL
    double *grad_e;             // [n_e][n_eps] or NULL
    double *grad_k;             // [n_e][2 n_int] or NULL
    double *gpartial;           // [grid][kAdjScalars + 2 n_f n_ext]
    // Monte-Carlo integration (momenta drawn in the kernel; n_e samples)
    uint64_t seed;
    // 16-byte accesses allowed: bit 0 the momentum rows (k 16-byte aligned,
    // stride_k even), bit 1 the rows of grad_k
    int vec_io;
    // rows of the specialized kernels' partial sums (one per wave), stored
    // column by column: element (row r, column c) at [c * nrows + r]
    int64_t nrows;
    // two-pass forward: a chunk of n_chunk samples starting at sample s0;
    // work holds its group sums FT_g at [g * ld + i] and energies E_j at
    // [(G + j) * ld + i] (ld a multiple of the block)
    double *work;
    int64_t ld, s0, n_chunk;
    // two-pass Monte-Carlo sums: the first pass draws sample s's momenta from
    // the counter-based generator (seed), the second accumulates per frequency
    // row sum Re I, sum Im I, sum (Re I)^2, sum (Im I)^2 (columns 4 f .. 4 f + 3)
    int mc;
};

// Frequency rows one Monte-Carlo launch accumulates (the caller splits longer lists).
constexpr int kMcMaxFreqs = 8;

// Per-block adjoint partial sums: dL/dbeta, dL/dmu, dL/dt, (unused), then
// dL/dw as complex [n_f][n_ext].
constexpr int kAdjScalars = 4;

}  // namespace ami
