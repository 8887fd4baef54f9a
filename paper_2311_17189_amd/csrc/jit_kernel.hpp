// Kernels of the run-time specialized evaluator (compiled with hipRTC).
//
// The skeleton is the one of the packed evaluators (kernels_packed.hpp), one
// lane per energy sample, but every table walk is replaced by the diagram's own
// straight-line code: the generated part that precedes this file defines, in
// namespace amijit, the sizes NE (energies), NI (loops), NG (lines), NX
// (external slots), L (distinct leaves), D (distinct denominators), G (groups),
// the leaf kinds kBose[L], and the functions
//   lines            K_j = sum_l alpha_jl k_l (+ external q), per component
//   line_trig        sin K_j, cos K_j from those of the k_l and q by angle addition
//   leaf_args        x_l = sum_i c_li E_i                        (Sec. 2.2)
//   taylor_leaves    f_l -> its Taylor coefficient T_j (poles of higher order, Eq. (5))
//   group_sums_c     the group sums at complex leaves (complex energies)
//   group_sums       FT_g = sum_{t in g} s_t prod_{l in t} f_l     (Sec. 2.3)
//   den_args         D_k = e_k . E + a_k . w                        (Sec. 2.2)
//   group_products   R_g = prod_{k in g} 1/D_k
//   den_cotangents   U_k = sum_{g contains k} u_g
//   den_scatter      dL/dE_i += e_ki Re(U_k rho_k), dL/dw_x += a_kx U_k rho_k
//   leaf_cotangents  dL/df_l = sum_{t contains l} dL/dFT_g(t) s_t prod_{l' != l} f_l'
//   leaf_scatter     dL/dE_i += sum_l c_li v_l
//   line_scatter     dL/dk_l += sum_j alpha_jl dL/dK_j
// With every index a constant, all per-sample state lives in registers: no
// LDS beyond the block reduction, no table reads, no scalar bit tests.
// Partial sums are written per wave (no LDS, no barrier), column by column
// (a.nrows = blocks x waves per block rows), in the column order of the packed
// evaluators, so the same reduction kernels finish them.
#pragma once

#include "jit_tiles.hpp"

// AMI_JIT_BLOCK lanes per block (the host launches with the same value);
// AMI_JIT_KERNELS selects the forward (1), the adjoint (2), the Monte-Carlo
// integrator (4), the forward at complex energies (8), the two passes of the
// two-pass forward (16, 32), the frequency and leaf passes of the adjoint of
// large solutions (64, 128), the adjoint at complex energies (256), the two
// passes of the forward at complex energies (512, 1024), the frequency and
// leaf passes of the adjoint at complex energies (2048, 4096), or a sum of
// them
#if AMI_JIT_KERNELS & 1
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_fwd(ami::KArgs a) {
    if (a.n_f == 1) amijit::fwd_tile<AMI_JIT_HUB, true>(a, blockIdx.x);
    else amijit::fwd_tile<AMI_JIT_HUB, false>(a, blockIdx.x);
}
#endif

#if AMI_JIT_ADJ_WAVES > 0
#define AMI_JIT_ADJ_ATTR __attribute__((amdgpu_waves_per_eu(AMI_JIT_ADJ_WAVES)))
#else
#define AMI_JIT_ADJ_ATTR
#endif

#if AMI_JIT_KERNELS & 2

extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) AMI_JIT_ADJ_ATTR void ami_jit_adj(ami::KArgs a) {
    __shared__ double park[amijit::kParkCols > 0 ? amijit::kParkCols * AMI_JIT_BLOCK : 1];
    const int64_t s = static_cast<int64_t>(blockIdx.x) * AMI_JIT_BLOCK + threadIdx.x;
    double in[amijit::NIN];
    amijit::load_inputs<AMI_JIT_HUB>(a, s < a.n_e ? s : a.n_e - 1, in);
    if (a.n_f == 1) amijit::adj_tile<AMI_JIT_HUB, true>(a, blockIdx.x, park, in);
    else amijit::adj_tile<AMI_JIT_HUB, false>(a, blockIdx.x, park, in);
}
#endif

#if AMI_JIT_KERNELS & 4
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_mc(ami::KArgs a) {
    amijit::mc_block<AMI_JIT_HUB>(a);
}
#endif

#if AMI_JIT_KERNELS & 8
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_cfwd(ami::KArgs a) {
    amijit::cfwd_tile(a, blockIdx.x);
}
#endif

#if AMI_JIT_KERNELS & 256
#if AMI_JIT_CADJ_WAVES > 0
__attribute__((amdgpu_waves_per_eu(AMI_JIT_CADJ_WAVES)))
#endif
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_cadj(ami::KArgs a) {
    __shared__ double park[amijit::kParkS ? 2 * amijit::L * AMI_JIT_BLOCK : 1];
    amijit::cadj_tile(a, blockIdx.x, park);
}
#endif

#if AMI_JIT_KERNELS & 512
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_csums(ami::KArgs a) {
    amijit::csums_tile(a, blockIdx.x);
}
#endif

#if AMI_JIT_KERNELS & 1024
// the grid of ami_jit_freq: (tile, frequency) blocks dealt over the XCDs
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_cfreq(ami::KArgs a) {
    const int64_t b = blockIdx.x, local = b >> 3;
    const int f = static_cast<int>(local % a.n_f);
    const int64_t tile = 8 * (local / a.n_f) + (b & 7);
    if (tile * AMI_JIT_BLOCK >= a.n_chunk) return;
    amijit::cfreq_tile(a, tile, f);
}
#endif

// occupancy floors of the large adjoint's passes (waves per SIMD; 0: none)
#ifndef AMI_JIT_ADJF_WAVES
#define AMI_JIT_ADJF_WAVES 2
#endif
#ifndef AMI_JIT_ADJL_WAVES
#define AMI_JIT_ADJL_WAVES 2
#endif
#if AMI_JIT_KERNELS & 64
#if AMI_JIT_ADJF_WAVES > 0
__attribute__((amdgpu_waves_per_eu(AMI_JIT_ADJF_WAVES)))
#endif
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_adjf(ami::KArgs a) {
    amijit::adjf_tile(a, blockIdx.x);
}
#endif

#if AMI_JIT_KERNELS & 128
#if AMI_JIT_ADJL_WAVES > 0
__attribute__((amdgpu_waves_per_eu(AMI_JIT_ADJL_WAVES)))
#endif
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_adjl(ami::KArgs a) {
    __shared__ double park[amijit::kParkCols > 0 ? amijit::kParkCols * AMI_JIT_BLOCK : 1];
    amijit::adjl_tile<AMI_JIT_HUB>(a, blockIdx.x, park);
}
#endif

#ifndef AMI_JIT_SUMS_WAVES
#define AMI_JIT_SUMS_WAVES 0
#endif
#if AMI_JIT_KERNELS & 16
#if AMI_JIT_SUMS_WAVES > 0
__attribute__((amdgpu_waves_per_eu(AMI_JIT_SUMS_WAVES)))
#endif
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_sums(ami::KArgs a) {
    amijit::sums_tile<AMI_JIT_HUB>(a, blockIdx.x);
}
#endif

#if AMI_JIT_KERNELS & 32
// One block per (tile, frequency row) in a one-dimensional grid: block b runs
// on the XCD b mod 8 (the dispatcher deals blocks round-robin over the eight
// XCDs), and the n_f blocks of a tile are consecutive on that XCD, so a
// tile's stored group sums come from HBM once and from the XCD's L2 for the
// other frequency rows.  Blocks past the last tile (the tile count rounded up
// to a multiple of 8) return at once.
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_freq(ami::KArgs a) {
    const int64_t b = blockIdx.x, local = b >> 3;
    const int f = static_cast<int>(local % a.n_f);
    const int64_t tile = 8 * (local / a.n_f) + (b & 7);
    if (tile * AMI_JIT_BLOCK >= a.n_chunk) return;
    amijit::freq_tile(a, tile, f);
}
#endif

#if AMI_JIT_KERNELS & 2048
#if AMI_JIT_ADJF_WAVES > 0
__attribute__((amdgpu_waves_per_eu(AMI_JIT_ADJF_WAVES)))
#endif
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_cadjf(ami::KArgs a) {
    amijit::cadjf_tile(a, blockIdx.x);
}
#endif

#if AMI_JIT_KERNELS & 4096
#if AMI_JIT_CADJL_WAVES > 0
__attribute__((amdgpu_waves_per_eu(AMI_JIT_CADJL_WAVES)))
#endif
extern "C" __global__ __launch_bounds__(AMI_JIT_BLOCK) void ami_jit_cadjl(ami::KArgs a) {
    amijit::cadjl_tile(a, blockIdx.x);
}
#endif
