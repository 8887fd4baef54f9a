// FP64 fused multiply-add throughput of the device, measured beside the
// vendor's peak so that the evaluation kernels' rates can be put against both.
// Every lane runs eight independent chains a <- fma(a, m, c), so a wave always
// has a FMA whose operands are ready; with eight waves per SIMD the FP64 pipes
// issue back to back.  With 0 < m < 1 the chains converge to c / (1 - m) = 1
// and never leave the normal range.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ami_internal.hpp"
#include "runtime.hpp"

namespace ami {
namespace {

constexpr int kPeakChains = 8;
constexpr int kPeakBlock = 256;
constexpr int kPeakBlocksPerCu = 8;   // 32 waves per CU: eight per SIMD

__global__ __launch_bounds__(kPeakBlock) void ami_fp64_peak_kernel(double *sink, int64_t iters, double m,
                                                                    double c) {
    double a[kPeakChains];
#pragma unroll
    for (int j = 0; j < kPeakChains; ++j) a[j] = 1.0 + 0.125 * j + 1e-3 * (threadIdx.x & 7);
    for (int64_t t = 0; t < iters; ++t) {
#pragma unroll
        for (int j = 0; j < kPeakChains; ++j) a[j] = fma(a[j], m, c);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kPeakChains; ++j) s += a[j];
    sink[static_cast<int64_t>(blockIdx.x) * kPeakBlock + threadIdx.x] = s;   // keeps the chains live
}

}  // namespace
}  // namespace ami

extern "C" {

AmiStatus amiMeasureFp64Peak(int64_t iters, double *tflops, void *hip_stream) {
    using namespace ami;
    clear_error();
    if (iters < 1 || iters > (int64_t(1) << 24)) return fail(AMI_E_ARG, "iters must be in 1..2^24");
    if (!tflops) return fail(AMI_E_ARG, "tflops is NULL");
    const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    const int blocks = std::max(cus, 1) * kPeakBlocksPerCu;
    double *sink = nullptr;
    e = hipMalloc(&sink, static_cast<size_t>(blocks) * kPeakBlock * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "peak sink allocation");
    hipEvent_t t0 = nullptr, t1 = nullptr;
    e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    float ms = 0.0f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // the second launch is the one timed
        e = hipEventRecord(t0, stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(ami_fp64_peak_kernel, dim3(blocks), dim3(kPeakBlock), 0, stream, sink, iters,
                               0.999999, 1e-6);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(t1, stream);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    const hipError_t ef = hipFree(sink);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return hip_fail(e, "peak kernel");
    if (ms <= 0.0f) return fail(AMI_E_HIP, "peak kernel: no elapsed time");
    const double flops = 2.0 * kPeakChains * static_cast<double>(iters) * blocks * kPeakBlock;
    *tflops = flops / (static_cast<double>(ms) * 1e-3) / 1e12;
    return AMI_OK;
}

}  // extern "C"
