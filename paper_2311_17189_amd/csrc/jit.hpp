// Run-time specialized evaluator: source generation (codegen.cpp) and its
// compilation, caching and loading (jit.cpp).
#pragma once

#include <string>

#include "ami_internal.hpp"

namespace ami {

// Largest solution (flat terms) specialized; larger ones stay on the
// table-driven kernels, whose code size does not grow with the diagram.
constexpr int kJitMaxTerms = 1024;
// AMI_VARIANT_AUTO uses the specialized adjoint up to this many terms: beyond
// it the straight-line reverse sweep outgrows the register file.
constexpr int kJitAutoAdjointTerms = 128;

// Whether the diagram can be specialized for the energy (hub = false) or
// momentum (hub = true) input; *why says why not.
bool jit_supported(const AmiTerms *t, bool hub, std::string *why);

// Lanes per block of the specialized kernels.
int jit_block(const AmiTerms *t, bool hub);

// Device source of the specialized kernels: the forward (kernels & 1), the
// adjoint (kernels & 2), the Monte-Carlo integrator (kernels & 4) and/or the
// forward at complex energies (kernels & 8).
std::string jit_source(const AmiTerms *t, bool hub, int kernels);

// Kernels of the specialized evaluator.
enum JitKind { kJitForward = 0, kJitAdjoint = 1, kJitMonteCarlo = 2, kJitComplex = 3 };
constexpr int kJitKinds = 4;

// The specialized kernel of `kind` for the energy (hub = false) or momentum
// input as a hipFunction_t: compiled (or fetched from the code-object cache)
// and loaded on the current device on first use; thread-safe per handle.
// The Monte-Carlo kernel exists for the momentum input only, the complex one
// for the energy input only.
AmiStatus jit_get(AmiTerms *t, bool hub, int kind, void **fn);

// Only the code object of `kind` (compiled or fetched from the cache): needs
// no device.
AmiStatus jit_compile(AmiTerms *t, bool hub, int kind);

// Unload every module of the handle (amiFree).
void jit_release(AmiTerms *t);

}  // namespace ami
