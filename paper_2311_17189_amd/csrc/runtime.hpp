// Runtime helpers shared by the evaluate and batch entry points (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ami_internal.hpp"
#include "device_common.hpp"

namespace ami {

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

}  // namespace ami
