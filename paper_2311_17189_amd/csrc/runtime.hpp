// Runtime helpers shared by the evaluate and batch entry points (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ami_internal.hpp"
#include "device_common.hpp"
#include "kargs.hpp"

namespace ami {

// Column sums of the partial-sum arrays: element (row r, column c) at
// partial[r * rs + c * cs] (rs = ncols, cs = 1 for the per-block sums of the
// table-driven kernels; rs = 1, cs = rows for the per-wave sums of the
// specialized ones, so that a column is one contiguous read).  One block of
// kRedThreads per column; thread t adds rows t, t + kRedThreads, ... in
// order, loading 16 of them before adding (16 loads in flight per thread),
// then the block adds the threads in a fixed order (wave sums, then the waves
// in order): a fixed summation order for a given row count.
constexpr int kRedThreads = 1024;

__device__ __forceinline__ double column_sum(const double *col, int64_t n, int64_t rs, double *sh) {
    const int tid = threadIdx.x;
    constexpr int kLoads = 16;                 // rows in flight per thread
    double acc = 0.0;
    for (int64_t b0 = tid; b0 < n; b0 += kLoads * kRedThreads) {
        double v[kLoads];
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            const int64_t b = b0 + static_cast<int64_t>(u) * kRedThreads;
            v[u] = b < n ? col[b * rs] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kLoads; ++u) acc += v[u];
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) sh[tid >> 6] = acc;
    __syncthreads();
    double r = 0.0;
    if (tid == 0)
        for (int w = 0; w < kRedThreads / 64; ++w) r += sh[w];
    return r;   // in thread 0
}

struct LaunchShape {
    int block = 256;     // lanes per block (one sample per lane)
    size_t lds = 0;      // dynamic LDS bytes per block
    int slots = 0;       // LDS slots per lane
};

AmiStatus hip_fail(hipError_t e, const char *what);
AmiStatus fill(double *p, int64_t n, hipStream_t stream);
AmiStatus upload(AmiTerms *t, DeviceTables **out);
AmiStatus pick_shape(int slots, LaunchShape &ls);
PackedTabs packed_tabs(const AmiTerms *t, const DeviceTables *dt);
int fwd_slots(const Tables &tb);

// The forward of one handle as an evaluate call with the given variant
// (AMI_VARIANT_*) would launch it on `stream`, row sums included.
AmiStatus launch_forward_as(AmiTerms *t, bool hub, KArgs &a, double *out_sum, hipStream_t stream, int variant);
// Whether AUTO would run the specialized (one- or two-pass) forward of t for
// n_f frequency rows; compiles and loads its kernels on the current device.
bool specialized_forward_ready(AmiTerms *t, bool hub, int n_f);
// The argument block of an evaluate call: momenta (k non-NULL; q reduced
// modulo 2 pi, its sin and cos) or energies, frequencies, beta, regulator.
void set_inputs(KArgs &a, const AmiTerms *t, const double *k, int64_t stride_k, const double *q, double hop_t,
                double mu, const double *energies, int64_t stride_s, int64_t stride_i, const double *ext_freqs,
                int64_t n_f, double beta, double e_reg, int64_t n_e);

}  // namespace ami
