// Host stand-in for the HIP runtime header, so that the device math of
// device_common.hpp can be compiled and checked with a host compiler.
#pragma once
#include <cmath>
#define __device__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define AMI_OPAQUE(x) asm volatile("" : "+m"(x))
#define AMI_SCHED_FENCE()
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
using std::expm1;
using std::fabs;
using std::fma;
using std::fmax;
using std::fmin;
inline double __shfl_xor(double v, int, int) { return v; }
// one lane per "wave" on the host: cross-lane moves return the lane's own value
inline int __builtin_amdgcn_mov_dpp(int src, int, int, int, bool) { return src; }
inline int __builtin_amdgcn_readlane(int v, int) { return v; }
inline unsigned __builtin_amdgcn_readfirstlane(unsigned v) { return v; }
struct AmiLanePair {
    unsigned v[2];
    unsigned operator[](int i) const { return v[i]; }
};
inline AmiLanePair __builtin_amdgcn_permlane32_swap(unsigned x, unsigned y, bool, bool) { return {{x, y}}; }
inline AmiLanePair __builtin_amdgcn_permlane16_swap(unsigned x, unsigned y, bool, bool) { return {{x, y}}; }
inline void __syncthreads() {}
