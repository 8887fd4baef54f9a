// Run-time specialized evaluator: source generation (codegen.cpp) and its
// compilation, caching and loading (jit.cpp).
#pragma once

#include <string>
#include <vector>

#include "ami_internal.hpp"

namespace ami {

// Largest solution (flat terms) specialized; larger ones stay on the
// table-driven kernels, whose code size does not grow with the diagram.
constexpr int kJitMaxTerms = 1024;
// Largest solution evaluated by the two-pass specialized forward (group sums
// stored per sample by a first kernel, read back per frequency by a second):
// its register use does not grow with the number of groups.
constexpr int kJitTwoPassMaxTerms = 4096;
// AMI_VARIANT_AUTO uses the one-pass specialized adjoint up to this many
// terms: beyond it the straight-line reverse sweep outgrows the register file,
// and the adjoint runs in passes over a workspace (up to kJitTwoPassMaxTerms).
constexpr int kJitAutoAdjointTerms = 128;
// The same switch for the adjoint at complex energies, whose passes hold
// complex values per leaf and node (per 10^6-sample step: 264 terms one pass
// 0.91 ms, passes 1.75 ms; 380: 1.30 / 3.18 ms; 560: 2.21 / 1.91 ms).
constexpr int kJitAutoComplexAdjointTerms = 512;

// Whether the adjoint of a solution above kJitAutoAdjointTerms can run in
// passes (the two-pass form, no Taylor-coefficient leaves).
bool jit_adjoint_passes_supported(const AmiTerms *t, bool hub, std::string *why);

// Whether the diagram can be specialized for the energy (hub = false) or
// momentum (hub = true) input; *why says why not.
bool jit_supported(const AmiTerms *t, bool hub, std::string *why, bool two_pass = false);

// Whether AUTO evaluates the forward in two passes: the group sums and the
// reciprocals the one-pass kernel holds in registers across its frequency
// loop would exceed about half of a wave's registers.
bool jit_prefers_two_pass(const AmiTerms *t);

// Lanes per block of the specialized kernels.
int jit_block(const AmiTerms *t, bool hub);

// Device source of the specialized kernels: the forward (kernels & 1), the
// adjoint (kernels & 2), the Monte-Carlo integrator (kernels & 4), the
// forward at complex energies (kernels & 8), the two passes of the
// two-pass forward (kernels & 16: group sums and energies stored per sample;
// kernels & 32: per frequency, reciprocals and group products against them),
// and the passes of the adjoint of large solutions that follow the first of
// those (kernels & 64: per frequency, the group-sum and denominator
// cotangents; kernels & 128: the leaf cotangents and the gradients), the
// adjoint at complex energies (kernels & 256), and the two passes of the
// forward at complex energies (kernels & 512: complex group sums and energies
// stored per sample; kernels & 1024: per frequency, against them), and the
// passes of the adjoint at complex energies that follow the first of those
// (kernels & 2048: per frequency, the complex group-sum and denominator
// cotangents; kernels & 4096: the complex leaf cotangents and the gradients).
// nested_part: terms per part of the one-pass adjoint's leaf cotangents as a
// reverse sweep of the nested group sums (0: per-term prefix/suffix products;
// -1: the AMIGPU_JIT_NESTED_COTANGENTS override, else per-term products).
std::string jit_source(const AmiTerms *t, bool hub, int kernels, int nested_part = -1);

// The part size named by AMIGPU_JIT_NESTED_COTANGENTS, or -1.
int jit_nested_override();

// Terms per part of the nested leaf-cotangent sweep the one-pass adjoint
// tries beside the per-term products (the code object kept is chosen from
// the two compiled ones' registers and spills).
constexpr int kJitNestedPartTerms = 4;

// Unsigned ints between two work-list counters of a persistent batch kernel
// (one 128-byte cache line each).
constexpr int kBatchCounterStride = 32;

// Source of one module of the persistent specialized batch: the generated
// functions of every item (forward in one pass, or the two-pass forward where
// two_pass[j] is set; one_row[j]: the one-pass tile for exactly one frequency
// row) in a namespace of its own with the tile functions, all at `block`
// lanes per block, and the persistent kernels selected by `phases`:
// ami_batch_p1 (phases & 1: one-pass tiles and the two-pass items' first
// pass) and ami_batch_p2 (phases & 2, with any two-pass item: their frequency
// pass, a work item being a tile range at a range of rows).  The kernels take
// eight counters kBatchCounterStride apart, one per work list.
// A work item names its item by labels[j] (by j when labels is empty).
// claim_ahead: a block claims its next work item before it runs the current
// one (the claim's round trip overlaps the work, for a register more);
// waves > 0: the kernels are compiled for at least that many waves per SIMD.
std::string jit_batch_source(const std::vector<const AmiTerms *> &items, const std::vector<int> &two_pass,
                             const std::vector<int> &one_row, bool hub, int block, int phases,
                             const std::vector<int> &labels, bool claim_ahead = true, int waves = 0);

// An unsigned value of the kernel metadata of a code object built here (the
// integer after the key in its one kernel's note), or -1.
int64_t code_meta(const std::vector<char> &code, const char *key);

// Kernels of the specialized evaluator.
// kJitAdjFreq and kJitAdjLeaf are the frequency and leaf passes of the
// adjoint of large solutions (after kJitSumsPass); kJitComplexAdj is the
// adjoint at complex energies (energy input only, as kJitComplex);
// kJitComplexSums and kJitComplexFreq the two passes of the forward at complex
// energies (solutions above kJitMaxTerms terms); kJitComplexAdjFreq and
// kJitComplexAdjLeaf the frequency and leaf passes of the adjoint at complex
// energies (after kJitComplexSums).
enum JitKind {
    kJitForward = 0,
    kJitAdjoint = 1,
    kJitMonteCarlo = 2,
    kJitComplex = 3,
    kJitSumsPass = 4,
    kJitFreqPass = 5,
    kJitAdjFreq = 6,
    kJitAdjLeaf = 7,
    kJitComplexAdj = 8,
    kJitComplexSums = 9,
    kJitComplexFreq = 10,
    kJitComplexAdjFreq = 11,
    kJitComplexAdjLeaf = 12
};
constexpr int kJitKinds = 13;

// Kinds for the energy input only (complex energies).
inline bool jit_kind_complex(int kind) {
    return kind == kJitComplex || kind == kJitComplexAdj || kind == kJitComplexSums || kind == kJitComplexFreq ||
           kind == kJitComplexAdjFreq || kind == kJitComplexAdjLeaf;
}

// The specialized kernel of `kind` for the energy (hub = false) or momentum
// input as a hipFunction_t: compiled (or fetched from the code-object cache)
// and loaded on the current device on first use; thread-safe per handle.
// The Monte-Carlo kernel exists for the momentum input only, the complex one
// for the energy input only.
AmiStatus jit_get(AmiTerms *t, bool hub, int kind, void **fn);

// The kernel of `kind` only if jit_get has already loaded it on the current
// device (loads nothing, allocates nothing): AMI_E_UNSUPPORTED when its
// compilation failed, AMI_E_ARG when it has not been loaded yet.
AmiStatus jit_loaded(AmiTerms *t, bool hub, int kind, void **fn);

// Only the code object of `kind` (compiled or fetched from the cache): needs
// no device.
AmiStatus jit_compile(AmiTerms *t, bool hub, int kind);

// The code object of a generated source: from the disk cache, else compiled
// with hipRTC under the library's flags and stored there.  Needs no device;
// thread-safe.  On failure err says why (the status is AMI_E_HIP).
AmiStatus code_from_source(const std::string &src, std::vector<char> &code, std::string &err);

// Unload every module of the handle (amiFree).
void jit_release(AmiTerms *t);

}  // namespace ami
