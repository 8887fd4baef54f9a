// Internal data structures of libamigpu: the host-side symbolic solution and
// its flattened evaluation tables (shared by the construction and the HIP
// evaluators; not part of the public ABI).
#pragma once

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/amigpu.h"

namespace ami {

// Limits of this build (checked in amiConstruct).
constexpr int kMaxEps = 32;     // energy placeholders
constexpr int kMaxFreq = 16;    // frequency slots
constexpr int kMaxExt = 4;      // external slots evaluated on the device
constexpr int kMaxEpsDev = 16;  // energy placeholders held in registers by the kernels
constexpr int kMaxInt = 12;     // nested sums evaluated on the device

// One term of the flat (FACTORIZE=false) solution: s * prod(leaves) / prod(dens).
// leaves: n_int records (sigma, e[0..n_eps)); dens: records (e[0..n_eps), a[0..n_freq)).
struct FlatTerm {
    int s = 1;
    std::vector<int> leaves;
    std::vector<int> dens;
};

// Node of the factorized Fermi tree (Sec. 2.1, Fig. 1).
struct TreeNode {
    enum Kind : int { ONE = 0, LEAF = 1, MUL = 2, ADD = 3 } kind = ONE;
    int sigma = 0;                 // LEAF
    std::vector<int> e;            // LEAF energy coefficients
    std::vector<int> child;        // MUL / ADD children (node indices)
    std::vector<int> coef;         // ADD integer weights, one per child
};

struct TreeTerm {
    int node = 0;                  // root of its Fermi tree
    std::vector<int> dens;         // sign-normalized, sorted
};

// Device copy of the evaluation tables (one per device the handle is used on).
struct DeviceTables {
    int device = -1;
    void *blob = nullptr;          // one allocation holding every table below
    const double *leaf_coef = nullptr;   // [L][n_eps]
    const double *leaf_sigma = nullptr;  // [L]
    const double *den_coef = nullptr;    // [D][n_eps + n_ext]
    const int32_t *group_dens = nullptr; // [G][dpt]
    const int32_t *group_start = nullptr;// [G+1] term ranges
    const double *term_sign = nullptr;   // [T]
    const int32_t *term_leaf = nullptr;  // [T][n_int]
    const double *line_alpha = nullptr;  // [n_g][n_freq] momentum labels (Hubbard path)
    // packed tables (device_common.hpp, PackedTabs)
    const uint64_t *p_leaf = nullptr;
    const uint64_t *p_den = nullptr;
    const uint32_t *p_line = nullptr;
    const uint64_t *p_term = nullptr;
    const uint64_t *p_group = nullptr;
    // workspaces of the per-block partial sums, one per stream (calls on one
    // stream are ordered on the device, calls on different streams get
    // different buffers); grown on demand, outgrown buffers kept until amiFree
    struct Workspace {
        void *stream = nullptr;
        void *ptr = nullptr;
        size_t bytes = 0;
    };
    std::vector<Workspace> ws;
    std::vector<void *> retired;
};

// Flattened, common-subexpression-eliminated evaluation tables (host).
struct Tables {
    int L = 0, D = 0, G = 0, T = 0;
    int dpt = 0;                          // denominators per term
    std::vector<double> leaf_coef;        // [L][n_eps]
    std::vector<double> leaf_sigma;       // [L]
    std::vector<double> den_coef;         // [D][n_eps + n_ext]
    std::vector<int32_t> group_dens;      // [G][dpt] (uniform solutions only)
    std::vector<int32_t> group_den_start; // [G+1] ranges of group_den_list
    std::vector<int32_t> group_den_list;  // every group's denominator indices (repeats = powers)
    std::vector<int> leaf_order;          // [L] Taylor order j of each leaf (0: the function)
    bool uniform = true;                  // plain leaves, n_g - n_int denominators per term
    std::vector<int32_t> group_start;     // [G+1]
    std::vector<double> term_sign;        // [T]
    std::vector<int32_t> term_leaf;       // [T][n_int]
    std::vector<double> line_alpha;       // [n_g][n_freq]
    // packed form: every energy coefficient +-1, indices below 256, <= 8 leaves
    // and denominators per term, <= 16 energies and frequency slots
    bool packable = false;
    std::vector<uint64_t> p_leaf;         // [L]
    std::vector<uint64_t> p_den;          // [D]
    std::vector<uint32_t> p_line;         // [n_g]
    std::vector<uint64_t> p_term;         // [T]
    std::vector<uint64_t> p_group;        // [G]
    uint32_t fermi_used = 0;
    bool use_products = false;
};

}  // namespace ami

struct AmiTerms {
    int n_g = 0, n_eps = 0, n_freq = 0, n_int = 0, n_ext = 0;
    uint32_t flags = 0;
    int variant = 0;                         // AMI_VARIANT_* (amigpu.h)
    std::vector<int8_t> alpha, eps;
    std::vector<uint8_t> fermionic;
    int64_t raw_terms = 0;
    std::vector<ami::FlatTerm> terms;        // canonical
    std::vector<ami::TreeNode> tree;         // factorized form (AMI_FACTORIZE)
    std::vector<ami::TreeTerm> tree_terms;
    ami::Tables tab;
    std::mutex dev_mu;
    std::vector<ami::DeviceTables> dev;      // uploaded copies
    // run-time specialized kernels: code objects per (input, kernel) -- index
    // 6 * momentum + kernel (0 forward, 1 adjoint, 2 Monte-Carlo, 3 forward at
    // complex energies, 4 and 5 the two passes of the two-pass forward) -- and
    // the modules loaded from them, one per device
    std::mutex jit_mu;
    std::vector<char> jit_code[26];           // [2 inputs][kJitKinds]
    std::string jit_error[26];                // why a compilation failed (not retried)
    struct JitModule {
        int device = -1, kind = 0;
        void *module = nullptr, *fn = nullptr;
    };
    std::vector<JitModule> jit_mods;
};

namespace ami {
// thread-local last-error helpers (abi.cpp)
AmiStatus fail(AmiStatus st, const std::string &msg);
void clear_error();
// construction (construct.cpp)
AmiStatus build_tables(AmiTerms *t);
}  // namespace ami
