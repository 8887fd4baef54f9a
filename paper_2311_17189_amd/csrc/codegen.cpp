// Source generator of the run-time specialized evaluator: writes the
// diagram's evaluation tables (leaves, denominators, groups, terms and
// momentum lines, built by build_tables) out as straight-line device code for
// the kernels of jit_kernel.hpp.  Sums over coefficients keep the order of the
// table-driven evaluators (index order, first term as +v or -v) and products
// their left-to-right association; every fused multiply-add of the values
// is written out (the code is compiled without contraction, which only the
// reverse sweep's functions turn on), so the forward and adjoint kernels of a
// diagram compute the same values bit for bit.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "ami_internal.hpp"
#include "jit.hpp"

namespace ami {

namespace {

// The reverse sweep (cotangents and their scatters) lets the compiler fuse
// its multiply-add pairs; the forward values are computed outside it, with
// every fused multiply-add written out, so they do not change.
const char *const kReverseContract = "#pragma clang fp contract(fast)\n";

std::string num(double v) {
    char b[40];
    std::snprintf(b, sizeof(b), "%.17g", v);
    std::string s(b);
    if (s.find_first_of(".eEn") == std::string::npos) s += ".0";
    return s;
}

// A sum of signed products of leaves, sum_t c_t prod_{l in t} F_l, written as
// nested multiply-adds (a greedy multivariate Horner scheme): the leaf a that
// occurs in the most terms (the lowest index among equals) is factored out,
// F_a * (the terms holding a, one a removed) + (the other terms), and both
// parts are nested the same way.  Each step is one fma (a mul or an add where
// a part is zero or a unit constant); terms with equal leaf multisets merge,
// and a sub-sum met again (or its negative) reuses the node that holds it.
// The nodes are built first (horner_build), then written out (horner_emit:
// const double h<k> of the enclosing block).
struct HornerTerm {
    double c;
    std::vector<int> leaves;   // a multiset (a leaf may repeat)
};

// The terms with their leaf multisets sorted, equal multisets merged and
// zero coefficients dropped.
std::vector<HornerTerm> merged_terms(std::vector<HornerTerm> ts) {
    for (HornerTerm &t : ts) std::sort(t.leaves.begin(), t.leaves.end());
    std::sort(ts.begin(), ts.end(), [](const HornerTerm &x, const HornerTerm &y) { return x.leaves < y.leaves; });
    std::vector<HornerTerm> m;
    for (HornerTerm &t : ts) {
        if (!m.empty() && m.back().leaves == t.leaves) m.back().c += t.c;
        else m.push_back(std::move(t));
    }
    m.erase(std::remove_if(m.begin(), m.end(), [](const HornerTerm &t) { return t.c == 0.0; }), m.end());
    return m;
}

// The merged sum's key up to sign (`flip`: its first coefficient is negative
// and the key is that of the negated sum).
std::string sum_key(const std::vector<HornerTerm> &m, bool &flip) {
    flip = m[0].c < 0.0;
    std::string key;
    for (const HornerTerm &t : m) {
        key += num(flip ? -t.c : t.c) + ":";
        for (int l : t.leaves) key += std::to_string(l) + ",";
        key += ";";
    }
    return key;
}

// One step of the nesting: the leaf in the most terms (the lowest index among
// equals) and the terms split into those holding it (one occurrence removed)
// and the others.
int split_on_shared_leaf(std::vector<HornerTerm> m, std::vector<HornerTerm> &with, std::vector<HornerTerm> &without) {
    std::map<int, int> count;   // terms holding each leaf
    for (const HornerTerm &t : m)
        for (size_t j = 0; j < t.leaves.size(); ++j)
            if (j == 0 || t.leaves[j] != t.leaves[j - 1]) ++count[t.leaves[j]];
    int a = -1, best = 0;
    for (const auto &kv : count)
        if (kv.second > best) {
            a = kv.first;
            best = kv.second;
        }
    for (HornerTerm &t : m) {
        auto it = std::find(t.leaves.begin(), t.leaves.end(), a);
        if (it == t.leaves.end()) {
            without.push_back(std::move(t));
        } else {
            t.leaves.erase(it);
            with.push_back(std::move(t));
        }
    }
    return a;
}

// A value of the nesting: zero, a number, a leaf or a node, with a sign.
struct HRef {
    enum Kind { ZERO, CONST, LEAF, NODE } kind = ZERO;
    double c = 0.0;   // CONST
    int idx = -1;     // LEAF: the leaf; NODE: the node
    bool neg = false;
};

// Node k holds F_a * w + u (w not zero).
struct HNode {
    int a;
    HRef w, u;
};

HRef href_negated(HRef r) {
    if (r.kind == HRef::CONST) r.c = -r.c;
    else if (r.kind != HRef::ZERO) r.neg = !r.neg;
    return r;
}

// Sub-sums already built (up to sign) for the current nesting.
using HMemo = std::map<std::string, HRef>;

HRef horner_nodes(std::vector<HornerTerm> ts, std::vector<HNode> &nodes, HMemo &memo) {
    std::vector<HornerTerm> m = merged_terms(std::move(ts));
    HRef r;
    if (m.empty()) return r;
    if (m.size() == 1 && m[0].leaves.empty()) {
        r.kind = HRef::CONST;
        r.c = m[0].c;
        return r;
    }
    bool flip;
    const std::string key = sum_key(m, flip);
    if (const auto it = memo.find(key); it != memo.end()) return flip ? href_negated(it->second) : it->second;
    std::vector<HornerTerm> with, without;
    const int a = split_on_shared_leaf(std::move(m), with, without);
    const HRef w = horner_nodes(with, nodes, memo);
    const HRef u = horner_nodes(without, nodes, memo);
    if (w.kind == HRef::ZERO) {
        r = u;
    } else if (w.kind == HRef::CONST && (w.c == 1.0 || w.c == -1.0) && u.kind == HRef::ZERO) {
        r.kind = HRef::LEAF;           // +-F_a itself
        r.idx = a;
        r.neg = w.c < 0.0;
    } else {
        nodes.push_back(HNode{a, w, u});
        r.kind = HRef::NODE;
        r.idx = static_cast<int>(nodes.size()) - 1;
    }
    memo[key] = flip ? href_negated(r) : r;
    return r;
}

// The nesting of sum_t c_t prod F over the given terms: its nodes and value.
HRef horner_build(std::vector<HornerTerm> ts, std::vector<HNode> &nodes) {
    HMemo memo;
    return horner_nodes(std::move(ts), nodes, memo);
}

template <typename LeafName>
std::string href_name(const HRef &r, const LeafName &leaf_name) {   // without its sign
    if (r.kind == HRef::LEAF) return leaf_name(r.idx);
    if (r.kind == HRef::NODE) return "h" + std::to_string(r.idx);
    return r.kind == HRef::CONST ? num(r.c) : std::string("0.0");
}

template <typename LeafName>
std::string href_expr(const HRef &r, const LeafName &leaf_name) {
    if (r.kind == HRef::CONST || r.kind == HRef::ZERO) return href_name(r, leaf_name);
    return r.neg ? "(-" + href_name(r, leaf_name) + ")" : href_name(r, leaf_name);
}

// The nodes as "const double h<k> = ...;" (one fma, mul or add each).
template <typename LeafName>
void horner_emit(const std::vector<HNode> &nodes, const LeafName &leaf_name, std::ostream &o) {
    for (size_t k = 0; k < nodes.size(); ++k) {
        const HNode &n = nodes[k];
        const std::string fa = leaf_name(n.a);
        std::string rhs;
        if (n.w.kind == HRef::CONST) {
            if (n.w.c == 1.0 || n.w.c == -1.0) rhs = href_expr(n.u, leaf_name) + (n.w.c < 0 ? " - " : " + ") + fa;
            else if (n.u.kind == HRef::ZERO) rhs = num(n.w.c) + " * " + fa;
            else rhs = "fma(" + num(n.w.c) + ", " + fa + ", " + href_expr(n.u, leaf_name) + ")";
        } else {
            const std::string sfa = n.w.neg ? "-" + fa : fa;
            const std::string wn = href_name(n.w, leaf_name);
            if (n.u.kind == HRef::ZERO) rhs = (n.w.neg ? "(-" + fa + ")" : fa) + " * " + wn;
            else rhs = "fma(" + sfa + ", " + wn + ", " + href_expr(n.u, leaf_name) + ")";
        }
        o << "    const double h" << k << " = " << rhs << ";\n";
    }
}

// The same greedy nesting for a sum of products whose factors may be complex:
// sum_g prod_{k in g} z_k with complex reciprocals z_k and one real factor
// per product (its group sum, read from memory).  Values are zero, a number,
// a real or a complex pair of expressions; each step L * W + U is written out
// with fma and the kinds of its operands (a complex product fused into the
// addend: re = fma(lr, wr, fma(-li, wi, ur))).
struct CVal {
    enum Kind { ZERO, CONST, REAL, CPLX } kind = ZERO;
    double c = 0.0;
    std::string re, im;   // expressions: a name, "(-name)" or a number
};

std::string neg_expr(const std::string &e) {
    if (e.size() > 3 && e.compare(0, 2, "(-") == 0 && e.back() == ')') return e.substr(2, e.size() - 3);
    return "(-" + e + ")";
}

CVal cnegated(CVal v) {
    if (v.kind == CVal::CONST) v.c = -v.c;
    if (v.kind == CVal::REAL || v.kind == CVal::CPLX) v.re = neg_expr(v.re);
    if (v.kind == CVal::CPLX) v.im = neg_expr(v.im);
    return v;
}

// products (sign, x, y) added to an addend: nested fma, or a product alone
std::string fused(const std::vector<std::tuple<bool, std::string, std::string>> &prods, const std::string &addend) {
    std::string acc = addend;
    for (auto it = prods.rbegin(); it != prods.rend(); ++it) {
        const auto &[negp, x, y] = *it;
        const std::string xs = negp ? neg_expr(x) : x;
        acc = acc.empty() ? xs + " * " + y : "fma(" + xs + ", " + y + ", " + acc + ")";
    }
    return acc;
}

using CMemo = std::map<std::string, CVal>;

// leaf(a) gives the value of factor a (a REAL or CPLX CVal of names)
template <typename Leaf>
CVal horner_c(std::vector<HornerTerm> ts, const Leaf &leaf, std::ostream &o, int &temps, CMemo &memo) {
    std::vector<HornerTerm> m = merged_terms(std::move(ts));
    CVal r;
    if (m.empty()) return r;
    if (m.size() == 1 && m[0].leaves.empty()) {
        r.kind = CVal::CONST;
        r.c = m[0].c;
        return r;
    }
    bool flip;
    const std::string key = sum_key(m, flip);
    if (const auto it = memo.find(key); it != memo.end()) return flip ? cnegated(it->second) : it->second;
    std::vector<HornerTerm> with, without;
    const int a = split_on_shared_leaf(std::move(m), with, without);
    const CVal w = horner_c(with, leaf, o, temps, memo);
    const CVal u = horner_c(without, leaf, o, temps, memo);
    const CVal L = leaf(a);
    if (w.kind == CVal::ZERO) {
        r = u;
    } else {
        // the product L * w as real and imaginary lists of (sign, x, y), or a
        // plain (signed) expression where w is a unit
        using Prods = std::vector<std::tuple<bool, std::string, std::string>>;
        Prods pre, pim;
        std::string plain_re, plain_im;
        const bool lc = L.kind == CVal::CPLX;
        bool cplx = lc;
        if (w.kind == CVal::CONST) {
            if (w.c == 1.0 || w.c == -1.0) {
                plain_re = w.c < 0 ? neg_expr(L.re) : L.re;
                if (lc) plain_im = w.c < 0 ? neg_expr(L.im) : L.im;
            } else {
                pre.emplace_back(false, num(w.c), L.re);
                if (lc) pim.emplace_back(false, num(w.c), L.im);
            }
        } else if (w.kind == CVal::REAL) {
            pre.emplace_back(false, L.re, w.re);
            if (lc) pim.emplace_back(false, L.im, w.re);
        } else {
            cplx = true;
            if (lc) {
                pre.emplace_back(false, L.re, w.re);
                pre.emplace_back(true, L.im, w.im);
                pim.emplace_back(false, L.re, w.im);
                pim.emplace_back(false, L.im, w.re);
            } else {
                pre.emplace_back(false, L.re, w.re);
                pim.emplace_back(false, L.re, w.im);
            }
        }
        cplx = cplx || u.kind == CVal::CPLX;
        std::string ure, uim;
        if (u.kind == CVal::CONST) ure = num(u.c);
        if (u.kind == CVal::REAL || u.kind == CVal::CPLX) ure = u.re;
        if (u.kind == CVal::CPLX) uim = u.im;
        auto part = [&](const Prods &pr, const std::string &plain, const std::string &add) -> std::string {
            if (!pr.empty()) return fused(pr, add);
            if (plain.empty()) return add;                    // nothing of L * w here
            if (add.empty()) return plain;
            return add + " + " + plain;
        };
        const std::string ere = part(pre, plain_re, ure);
        const std::string eim = cplx ? part(pim, plain_im, uim) : std::string();
        auto temp = [&](const std::string &e) {
            if (e.empty()) return std::string("0.0");
            const bool simple = e.find_first_of(" (") == std::string::npos || (e.compare(0, 2, "(-") == 0 &&
                                                                               e.find(' ') == std::string::npos);
            if (simple) return e;                              // a name or a negated name
            const std::string n = "c" + std::to_string(temps++);
            o << "    const double " << n << " = " << e << ";\n";
            return n;
        };
        r.kind = cplx ? CVal::CPLX : CVal::REAL;
        r.re = temp(ere);
        if (cplx) r.im = temp(eim);
    }
    memo[key] = flip ? cnegated(r) : r;
    return r;
}

// sum_i c_i v[i] over the non-zero coefficients, in index order: "+-v" for
// unit coefficients, fma for others; "0.0" when every coefficient is zero.
struct Lin {
    std::string expr;
    void add(double c, const std::string &v) {
        if (c == 0.0) return;
        if (expr.empty()) {
            if (c == 1.0) expr = v;
            else if (c == -1.0) expr = "(-" + v + ")";
            else expr = "(" + num(c) + " * " + v + ")";
        } else {
            if (c == 1.0) expr = "(" + expr + " + " + v + ")";
            else if (c == -1.0) expr = "(" + expr + " - " + v + ")";
            else expr = "fma(" + num(c) + ", " + v + ", " + expr + ")";
        }
    }
    std::string str() const { return expr.empty() ? "0.0" : expr; }
};

std::string idx(const char *a, int i) { return std::string(a) + "[" + std::to_string(i) + "]"; }

// Groups per chunk of the adjoint's frequency pass for large solutions (the
// cotangents of a chunk's denominators are gathered in registers).
constexpr int kAdjChunkGroups = 2;
// Whether each chunk forms the reciprocals of its own denominators (else all
// of them are formed once per frequency row and held through the chunks).
constexpr bool kAdjChunkOwnDens = true;
// Terms per nested part of a group in the adjoint's leaf pass, and parts
// between scheduling fences.
constexpr int kAdjLeafPartTerms = 32;
constexpr int kAdjLeafFenceParts = 1;

}  // namespace

bool jit_prefers_two_pass(const AmiTerms *t) {
    const Tables &tb = t->tab;
    return tb.T > kJitMaxTerms || 2 * tb.G + 4 * tb.D > 128;
}

bool jit_supported(const AmiTerms *t, bool hub, std::string *why, bool two_pass) {
    const Tables &tb = t->tab;
    auto no = [&](const std::string &m) {
        if (why) *why = m;
        return false;
    };
    if (tb.L < 1 || tb.G < 1) return no("solution without leaves");
    if (t->n_eps > kMaxEpsDev) return no("more than 16 energies");
    if (t->n_ext > kMaxExt) return no("more than 4 external slots");
    if (hub && t->n_g != t->n_eps) return no("momentum input needs one energy per line");
    const int max_terms = two_pass ? kJitTwoPassMaxTerms : kJitMaxTerms;
    if (tb.T > max_terms) return no("more than " + std::to_string(max_terms) + " terms");
    return true;
}

bool jit_adjoint_passes_supported(const AmiTerms *t, bool hub, std::string *why) {
    return jit_supported(t, hub, why, true);
}

namespace {

// Adjoint values parked in LDS instead of registers: the momentum chain
// rule's 3 per line, and the leaf derivatives while both fit in 40 doubles
// per lane (two resident blocks of 256 lanes per CU).
constexpr int kParkBudget = 40;
int park_chain(const AmiTerms *t, bool hub) { return hub ? 3 * t->n_g : 0; }
bool park_dv(const AmiTerms *t, bool hub) {
    if (const char *e = std::getenv("AMIGPU_JIT_PARK_DV")) return std::atoi(e) != 0;   // tuning override
    for (int o : t->tab.leaf_order)
        if (o > 0) return false;              // Taylor-coefficient leaves: their slopes stay in registers
    return park_chain(t, hub) + t->tab.L <= kParkBudget;
}
int park_cols(const AmiTerms *t, bool hub) { return park_chain(t, hub) + (park_dv(t, hub) ? t->tab.L : 0); }

// occupancy floor of the one-pass adjoint (waves per SIMD; 0: none),
// AMIGPU_JIT_ADJ_WAVES overriding the default of two: an adjoint that would
// take more than 256 VGPRs runs at two waves with a few spills rather than at
// one (order-4 topologies of 40-52 terms: 0.099-0.105 -> 0.081-0.086 ms per
// 10^6-sample step)
// Terms per nested part in the complex adjoint's leaf pass (each node holds
// a complex value and a complex cotangent); AMIGPU_JIT_CADJ_PART overrides.
int cadj_part_terms() {
    const char *e = std::getenv("AMIGPU_JIT_CADJ_PART");
    const int v = e ? std::atoi(e) : 0;
    return v >= 1 && v <= 64 ? v : 64;
}

// occupancy floor of the complex adjoint's leaf pass (one wave: its spills
// at two cost more than the occupancy, 196 terms 1.73 -> 1.25 ms, 560 terms
// 2.63 -> 1.90 ms per 10^6-sample step); AMIGPU_JIT_CADJL_WAVES overrides
int cadjl_waves() {
    const char *e = std::getenv("AMIGPU_JIT_CADJL_WAVES");
    const int v = e ? std::atoi(e) : -1;
    return v >= 0 && v <= 8 ? v : 1;
}

}  // namespace

// Terms per part of the one-pass adjoint's nested leaf-cotangent sweep when
// AMIGPU_JIT_NESTED_COTANGENTS names it (0: per-term products), else -1.
int jit_nested_override() {
    const char *e = std::getenv("AMIGPU_JIT_NESTED_COTANGENTS");
    if (!e) return -1;
    const int v = std::atoi(e);
    return v >= 0 && v <= 64 ? v : 0;
}

namespace {

int adj_waves() {
    const char *e = std::getenv("AMIGPU_JIT_ADJ_WAVES");
    if (!e) return 2;
    const int v = std::atoi(e);
    return (v >= 0 && v <= 8) ? v : 2;
}

}  // namespace

// 256 lanes while the adjoint's parked columns fit in 80 KB per block (two
// blocks per CU), else 128
int jit_block(const AmiTerms *t, bool hub) { return park_cols(t, hub) * 256 * 8 <= 80 * 1024 ? 256 : 128; }

std::string jit_source(const AmiTerms *t, bool hub, int kernels, int nested_part) {
    if (nested_part < 0) nested_part = std::max(0, jit_nested_override());
    const Tables &tb = t->tab;
    const int ne = t->n_eps, ni = t->n_int, ng = t->n_g, nx = t->n_ext, nf = t->n_freq;
    // a solution whose terms hold no denominators gets one phantom
    // denominator equal to 1 (no group uses it), so no array is empty
    const int L = tb.L, D = std::max(tb.D, 1), G = tb.G;
    auto gbegin = [&](int g) { return tb.group_den_start[g]; };
    auto gend = [&](int g) { return tb.group_den_start[g + 1]; };
    const int nc = ne + nx;
    std::ostringstream o;
    o << "// generated: specialized AMI evaluator, " << tb.T << " terms, " << L << " leaves, " << D
      << " denominators, " << G << " groups\n";
    o << "#define AMI_JIT_HUB " << (hub ? "true" : "false") << "\n";
    o << "#define AMI_JIT_KERNELS " << kernels << "\n";
    o << "#define AMI_JIT_BLOCK " << jit_block(t, hub) << "\n";
    o << "#define AMI_JIT_PARK_DV " << (park_dv(t, hub) ? "true" : "false") << "\n";
    o << "#define AMI_JIT_ADJ_WAVES " << adj_waves() << "\n";
    // the complex adjoint (one pass at every size): the same floor up to the
    // one-pass adjoint's automatic size; above it the spills of a two-wave
    // floor cost more than the lost occupancy (196 terms: 1.11 -> 0.86 ms,
    // 560 terms: 6.8 -> 5.7 ms per 10^6-sample step at one wave)
    o << "#define AMI_JIT_CADJ_WAVES " << (tb.T <= kJitAutoAdjointTerms ? adj_waves() : 1) << "\n";
    // the leaf pass of the complex adjoint in passes (its values per leaf and
    // node are complex, twice the real pass's)
    o << "#define AMI_JIT_CADJL_WAVES " << cadjl_waves() << "\n";
    o << "#include \"kargs.hpp\"\n";
    o << "namespace amijit {\n";
    o << "constexpr int NE = " << ne << ", NI = " << ni << ", NG = " << ng << ", NX = " << nx << ";\n";
    o << "constexpr int L = " << L << ", D = " << D << ", G = " << G << ";\n";
    // the forward values from sum_g FT_g R_g nested over the reciprocals
    // (groups_combine) above the adjoint's automatic size, group by group below
    const bool nested_groups = tb.T > kJitAutoAdjointTerms;
    o << "constexpr bool kNestedGroups = " << (nested_groups ? "true" : "false") << ";\n";
    o << "constexpr bool kBose[L] = {";
    for (int l = 0; l < L; ++l) o << (l ? ", " : "") << (tb.leaf_sigma[l] < 0 ? "true" : "false");
    o << "};\n";
    const std::string NXA = "(NX > 0 ? NX : 1)", NIA = "(NI > 0 ? NI : 1)", NGA = "(NG > 0 ? NG : 1)";

    // momentum lines: K_j = sum_l alpha_jl k_l over the loops, then + q of the external slots
    o << "__device__ __forceinline__ void lines(const double (&kx)[" << NIA << "], const double (&ky)[" << NIA
      << "], const double *q, double (&Kx)[" << NGA << "], double (&Ky)[" << NGA << "]) {\n";
    if (hub) {
        for (int j = 0; j < ng; ++j) {
            Lin ax, ay;
            for (int l = 0; l < ni; ++l) {
                const double a = tb.line_alpha[static_cast<size_t>(j) * nf + l];
                ax.add(a, idx("kx", l));
                ay.add(a, idx("ky", l));
            }
            for (int x = 0; x < nx; ++x) {
                const double a = tb.line_alpha[static_cast<size_t>(j) * nf + ni + x];
                ax.add(a, idx("q", 2 * x));
                ay.add(a, idx("q", 2 * x + 1));
            }
            o << "  Kx[" << j << "] = " << ax.str() << ";\n  Ky[" << j << "] = " << ay.str() << ";\n";
        }
    }
    o << "}\n";

    // sin and cos of the line momenta from those of the loop momenta and of
    // q (adjoint): K_j = sum of +-k_l (+-q), folded term by term with
    // sin(A +- b) = sin A cos b +- cos A sin b, cos(A +- b) = cos A cos b -+ sin A sin b
    o << "__device__ __forceinline__ void line_trig(const double (&sx)[" << NIA << "], const double (&cx)[" << NIA
      << "], const double (&sy)[" << NIA << "], const double (&cy)[" << NIA
      << "], const double *qs, const double *qc, double (&Sx)[" << NGA << "], double (&Cx)[" << NGA
      << "], double (&Sy)[" << NGA << "], double (&Cy)[" << NGA << "]) {\n";
    if (hub) {
        o << "  double nS;\n";
        for (int j = 0; j < ng; ++j)
            for (int comp = 0; comp < 2; ++comp) {
                std::vector<std::pair<int, std::pair<std::string, std::string>>> terms;
                for (int l = 0; l < ni; ++l) {
                    const int a = static_cast<int>(tb.line_alpha[static_cast<size_t>(j) * nf + l]);
                    if (a) terms.push_back({a, {idx(comp ? "sy" : "sx", l), idx(comp ? "cy" : "cx", l)}});
                }
                for (int x = 0; x < nx; ++x) {
                    const int a = static_cast<int>(tb.line_alpha[static_cast<size_t>(j) * nf + ni + x]);
                    if (a) terms.push_back({a, {idx("qs", 2 * x + comp), idx("qc", 2 * x + comp)}});
                }
                const std::string S = idx(comp ? "Sy" : "Sx", j), C = idx(comp ? "Cy" : "Cx", j);
                if (terms.empty()) {
                    o << "  " << S << " = 0.0; " << C << " = 1.0;\n";
                    continue;
                }
                for (size_t k = 0; k < terms.size(); ++k) {
                    const int sg = terms[k].first;
                    const std::string &sb = terms[k].second.first, &cb = terms[k].second.second;
                    if (k == 0) {
                        o << "  " << S << " = " << (sg > 0 ? "" : "-") << sb << "; " << C << " = " << cb << ";\n";
                    } else if (sg > 0) {
                        o << "  nS = fma(" << S << ", " << cb << ", " << C << " * " << sb << "); " << C << " = fma("
                          << C << ", " << cb << ", -(" << S << " * " << sb << ")); " << S << " = nS;\n";
                    } else {
                        o << "  nS = fma(" << S << ", " << cb << ", -(" << C << " * " << sb << ")); " << C
                          << " = fma(" << C << ", " << cb << ", " << S << " * " << sb << "); " << S << " = nS;\n";
                    }
                }
            }
        o << "  (void)nS;\n";
    }
    o << "  (void)sx; (void)cx; (void)sy; (void)cy; (void)qs; (void)qc; (void)Sx; (void)Cx; (void)Sy; (void)Cy;\n}\n";

    // leaf arguments x_l = sum_i c_li E_i
    o << "__device__ __forceinline__ void leaf_args(const double (&E)[NE], double (&x)[L]) {\n";
    for (int l = 0; l < L; ++l) {
        Lin s;
        for (int i = 0; i < ne; ++i) s.add(tb.leaf_coef[static_cast<size_t>(l) * ne + i], idx("E", i));
        o << "  x[" << l << "] = " << s.str() << ";\n";
    }
    o << "}\n";

    // group sums FT_g = sum_t s_t prod f, each group in the nested form of
    // horner()
    // leaf names: F[l], or a group's own copy f<l> (opaque copies)
    std::string leaf_prefix = "F[", leaf_suffix = "]";
    auto leaf_name = [&](int l) { return leaf_prefix + std::to_string(l) + leaf_suffix; };
    // the one-pass kernels' functions (and the adjoint's) are emitted when one
    // of those kernels is asked for, or for any solution small enough for them
    // (the host checks compile them); a two-pass source of a large solution
    // holds only what its two kernels use
    const bool small = tb.T <= kJitMaxTerms;
    const bool one_pass = (kernels & (15 | 256)) != 0;
    const bool adj_fns = (kernels & (2 | 256)) || ((kernels & 1) && small);
    // With `opaque`, every group first takes copies of the leaves it reads
    // through an empty asm (no instruction): the compiler then cannot merge
    // equal products of different groups, which for large solutions would
    // keep hundreds of shared products live across the whole function; equal
    // products within a group are still merged.
    auto group_sums_body = [&](const std::string &sink_prefix, const std::string &sink_suffix, bool opaque) {
    for (int g = 0; g < G; ++g) {
        o << "  { double ft;\n";
        leaf_prefix = opaque ? "f" : "F[";
        leaf_suffix = opaque ? "" : "]";
        if (opaque) {
            std::vector<int> used;
            for (int ti = tb.group_start[g]; ti < tb.group_start[g + 1]; ++ti)
                for (int j = 0; j < ni; ++j) used.push_back(tb.term_leaf[static_cast<size_t>(ti) * ni + j]);
            std::sort(used.begin(), used.end());
            used.erase(std::unique(used.begin(), used.end()), used.end());
            for (int l : used)
                o << "    double f" << l << " = F[" << l << "]; AMI_OPAQUE(f" << l << ");\n";
        }
        std::vector<HornerTerm> ts;
        for (int ti = tb.group_start[g]; ti < tb.group_start[g + 1]; ++ti) {
            HornerTerm h{tb.term_sign[ti], {}};
            for (int j = 0; j < ni; ++j) h.leaves.push_back(tb.term_leaf[static_cast<size_t>(ti) * ni + j]);
            ts.push_back(std::move(h));
        }
        std::vector<HNode> nodes;
        const HRef v = horner_build(std::move(ts), nodes);
        horner_emit(nodes, leaf_name, o);
        o << "    ft = " << href_expr(v, leaf_name) << ";\n";
        if (sink_suffix.find("ft)") != std::string::npos) o << "    " << sink_prefix << g << sink_suffix << "; }\n";
        else o << "    " << sink_prefix << g << sink_suffix << " = ft; }\n";
    }
    };
    if (one_pass) {
        o << "__device__ __forceinline__ void group_sums(const double (&F)[L], double (&FT)[G]) {\n";
        group_sums_body("FT[", "]", false);
        o << "}\n";
    }
    // two-pass forward, first pass: each group sum stored as soon as it is formed
    if (kernels & 16) {
        o << "__device__ __forceinline__ void group_sums_store(const double (&F)[L], double *ws, int64_t ld, "
             "uint32_t off) {\n";
        group_sums_body("ami::ws_store(ws, ld, ", ", off, ft)", true);
        o << "}\n";
    }

    // complex group sums (complex energies): each group's sum nested as the
    // real group sums, in complex arithmetic; `store`: each stored to the
    // workspace as soon as it is formed (real part in column g, imaginary part
    // in column G + g; the two-pass complex forward's first pass), the leaves
    // a group reads taken through opaque copies as in group_sums_store
    auto group_sums_c_body = [&](bool store) {
        for (int g = 0; g < G; ++g) {
            o << "  {\n";
            std::vector<HornerTerm> ts;
            for (int ti = tb.group_start[g]; ti < tb.group_start[g + 1]; ++ti) {
                HornerTerm h{tb.term_sign[ti], {}};
                for (int j = 0; j < ni; ++j) h.leaves.push_back(tb.term_leaf[static_cast<size_t>(ti) * ni + j]);
                ts.push_back(std::move(h));
            }
            if (store) {
                std::vector<int> used;
                for (const HornerTerm &h : ts) used.insert(used.end(), h.leaves.begin(), h.leaves.end());
                std::sort(used.begin(), used.end());
                used.erase(std::unique(used.begin(), used.end()), used.end());
                for (int l : used)
                    o << "    double fr" << l << " = Fr[" << l << "], fi" << l << " = Fi[" << l << "]; AMI_OPAQUE(fr" << l
                      << "); AMI_OPAQUE(fi" << l << ");\n";
            }
            auto leaf = [&](int l) {
                CVal v;
                v.kind = CVal::CPLX;
                v.re = store ? "fr" + std::to_string(l) : "Fr[" + std::to_string(l) + "]";
                v.im = store ? "fi" + std::to_string(l) : "Fi[" + std::to_string(l) + "]";
                return v;
            };
            int temps = 0;
            CMemo memo;
            const CVal v = horner_c(ts, leaf, o, temps, memo);
            const std::string re = v.kind == CVal::ZERO ? "0.0" : v.kind == CVal::CONST ? num(v.c) : v.re;
            const std::string im = v.kind == CVal::CPLX ? v.im : "0.0";
            if (store)
                o << "    ami::ws_store(ws, ld, " << g << ", off, " << re << "); ami::ws_store(ws, ld, " << G + g
                  << ", off, " << im << "); }\n";
            else
                o << "    FTr[" << g << "] = " << re << "; FTi[" << g << "] = " << im << "; }\n";
        }
    };
    if (kernels & (8 | 256)) {
        o << "__device__ __forceinline__ void group_sums_c(const double (&Fr)[L], const double (&Fi)[L], double "
             "(&FTr)[G], double (&FTi)[G]) {\n";
        group_sums_c_body(false);
        o << "}\n";
    }
    if (kernels & 512) {
        o << "__device__ __forceinline__ void group_sums_c_store(const double (&Fr)[L], const double (&Fi)[L], "
             "double *ws, int64_t ld, uint32_t off) {\n";
        group_sums_c_body(true);
        o << "}\n";
    }

    // Taylor-coefficient leaves (poles of higher order): T_j = beta^j f^(j) / j!,
    // f^(j) as a polynomial in f and fm = f(-y) (f' = -f fm, fm' = f fm);
    // taylor_expr writes statements that leave T_j of the values named f and m
    // in `dst` (j = 0: f itself)
    auto taylor_expr = [&](int jo, const std::string &dst, const std::string &pad) {
        if (jo == 0) return pad + dst + " = f;\n";
        std::map<std::pair<int, int>, long long> poly{{{1, 0}, 1}};
        for (int step = 0; step < jo; ++step) {
            std::map<std::pair<int, int>, long long> nxt;
            for (const auto &kv : poly) {
                const int a = kv.first.first, b = kv.first.second;
                if (a) nxt[{a, b + 1}] -= a * kv.second;
                if (b) nxt[{a + 1, b}] += b * kv.second;
            }
            poly.clear();
            for (const auto &kv : nxt)
                if (kv.second) poly.insert(kv);
        }
        double fact = 1.0;
        for (int i = 2; i <= jo; ++i) fact *= i;
        std::string scale = "beta";
        for (int i = 1; i < jo; ++i) scale += " * beta";
        std::string out = pad + "{ double acc = 0.0;\n";
        for (const auto &kv : poly) {
            std::string mono;
            for (int i = 0; i < kv.first.first; ++i) mono += (mono.empty() ? "f" : " * f");
            for (int i = 0; i < kv.first.second; ++i) mono += (mono.empty() ? "m" : " * m");
            out += pad + "  acc = fma(" + num(static_cast<double>(kv.second)) + ", " + mono + ", acc);\n";
        }
        out += pad + "  " + dst + " = acc * (" + scale + ") * " + num(1.0 / fact) + "; }\n";
        return out;
    };
    bool taylor = false;
    for (int l = 0; l < L; ++l) taylor = taylor || tb.leaf_order[l] > 0;
    o << "constexpr bool kTaylor = " << (taylor ? "true" : "false") << ";\n";
    o << "__device__ __forceinline__ void taylor_leaves(double (&F)[L], const double (&FM)[L], double beta) {\n";
    for (int l = 0; l < L; ++l) {
        const int jo = tb.leaf_order[l];
        if (jo == 0) continue;
        o << "  { const double f = F[" << l << "], m = FM[" << l << "];\n";
        o << taylor_expr(jo, "F[" + std::to_string(l) + "]", "    ");
        o << "  }\n";
    }
    o << "  (void)FM; (void)beta;\n}\n";
    // the adjoint's derivatives of the leaves of a solution with Taylor
    // coefficients: DX = dT_j/dx = (j + 1) T_(j+1), DB = dT_j/dbeta =
    // (j T_j + x DX) / beta, from the plain leaf pair (f, fm) at x
    o << "__device__ __forceinline__ void taylor_slopes(const double (&F)[L], const double (&FM)[L], const double "
         "(&X)[L], double beta, double (&DX)[L], double (&DB)[L]) {\n";
    if (taylor)
        for (int l = 0; l < L; ++l) {
            const int jo = tb.leaf_order[l];
            o << "  { const double f = F[" << l << "], m = FM[" << l << "]; double tj = 0.0, tn = 0.0;\n";
            o << taylor_expr(jo, "tj", "    ") << taylor_expr(jo + 1, "tn", "    ");
            o << "    DX[" << l << "] = " << num(static_cast<double>(jo + 1)) << " * tn;\n";
            o << "    DB[" << l << "] = fma(" << num(static_cast<double>(jo)) << ", tj, X[" << l << "] * DX[" << l
              << "]) / beta; }\n";
        }
    o << "  (void)F; (void)FM; (void)X; (void)beta; (void)DX; (void)DB;\n}\n";

    // denominators D_k = e_k . E + a_k . w
    o << "__device__ __forceinline__ void den_args(const double (&E)[NE], const double (&wr)[" << NXA
      << "], const double (&wi)[" << NXA << "], double (&dr)[D], double (&di)[D]) {\n";
    if (tb.D == 0) o << "  (void)E; (void)wr; (void)wi;\n  dr[0] = 1.0;\n  di[0] = 0.0;\n";
    for (int k = 0; k < tb.D; ++k) {
        Lin re, im;
        for (int i = 0; i < ne; ++i) re.add(tb.den_coef[static_cast<size_t>(k) * nc + i], idx("E", i));
        for (int x = 0; x < nx; ++x) {
            const double a = tb.den_coef[static_cast<size_t>(k) * nc + ne + x];
            re.add(a, idx("wr", x));
            im.add(a, idx("wi", x));
        }
        o << "  dr[" << k << "] = " << re.str() << ";\n  di[" << k << "] = " << im.str() << ";\n";
    }
    o << "}\n";

    // group products R_g = prod rho_k (complex), left to right
    auto group_product = [&](int g) {
        o << "  { double rr = 1.0, ri = 0.0, nr = 0.0;\n";
        for (int j = 0; j < gend(g) - gbegin(g); ++j) {
            const std::string k = std::to_string(tb.group_den_list[gbegin(g) + j]);
            if (j == 0) {
                o << "    rr = xr[" << k << "]; ri = xi[" << k << "];\n";
            } else {
                o << "    nr = fma(rr, xr[" << k << "], -ri * xi[" << k << "]); ri = fma(rr, xi[" << k
                  << "], ri * xr[" << k << "]); rr = nr;\n";
            }
        }
    };
    if (one_pass) {
        o << "__device__ __forceinline__ void group_products(const double (&xr)[D], const double (&xi)[D], "
             "double (&Rr)[G], double (&Ri)[G]) {\n";
        for (int g = 0; g < G; ++g) {
            group_product(g);
            o << "    (void)nr; Rr[" << g << "] = rr; Ri[" << g << "] = ri; }\n";
        }
        o << "}\n";
    }
    // the one-pass kernels' values sum_g FT_g R_g: nested over the reciprocals
    // (as the two-pass frequency pass) for solutions above the adjoint's
    // automatic size, else group by group from the products R_g (the
    // adjoint's own accumulation, so both kernels give the same bits)
    if (one_pass) {
        o << "__device__ __forceinline__ void groups_combine(const double (&xr)[D], const double (&xi)[D], "
             "const double (&FT)[G], double &acc_re, double &acc_im) {\n";
        if (nested_groups) {
            std::vector<HornerTerm> ts;
            for (int g = 0; g < G; ++g) {
                HornerTerm h{1.0, {}};
                for (int j = gbegin(g); j < gend(g); ++j) h.leaves.push_back(tb.group_den_list[j]);
                h.leaves.push_back(D + g);
                ts.push_back(std::move(h));
            }
            auto leaf = [&](int k) {
                CVal v;
                if (k < D) {
                    v.kind = CVal::CPLX;
                    v.re = "xr[" + std::to_string(k) + "]";
                    v.im = "xi[" + std::to_string(k) + "]";
                } else {
                    v.kind = CVal::REAL;
                    v.re = "FT[" + std::to_string(k - D) + "]";
                }
                return v;
            };
            int temps = 0;
            CMemo memo;
            const CVal v = horner_c(ts, leaf, o, temps, memo);
            const bool z = v.kind == CVal::ZERO;
            o << "    acc_re = " << (z ? "0.0" : v.kind == CVal::CONST ? num(v.c) : v.re) << ";\n";
            o << "    acc_im = " << (v.kind == CVal::CPLX ? v.im : "0.0") << ";\n";
        } else {
            o << "  double Rr[G], Ri[G];\n  group_products(xr, xi, Rr, Ri);\n  acc_re = 0.0;\n  acc_im = 0.0;\n";
            for (int g = 0; g < G; ++g)
                o << "  acc_re = fma(FT[" << g << "], Rr[" << g << "], acc_re);\n  acc_im = fma(FT[" << g << "], Ri[" << g
                  << "], acc_im);\n";
        }
        o << "}\n";
    }
    // two-pass forward, second pass: sum_g FT_g R_g nested over the
    // reciprocals, each stored group sum read where the nesting needs it
    if (kernels & 32) {
        o << "__device__ __forceinline__ void group_accumulate(const double (&xr)[D], const double (&xi)[D], "
             "const double *ws, int64_t ld, uint32_t off, double &acc_re, double &acc_im) {\n";
        // sum_g FT_g R_g nested over the reciprocals (factor k < D: z_k; factor
        // D + g: the stored FT_g, read where the nesting first needs it)
        std::vector<HornerTerm> ts;
        for (int g = 0; g < G; ++g) {
            HornerTerm h{1.0, {}};
            for (int j = gbegin(g); j < gend(g); ++j) h.leaves.push_back(tb.group_den_list[j]);
            h.leaves.push_back(D + g);
            ts.push_back(std::move(h));
        }
        std::vector<bool> loaded(static_cast<size_t>(G), false);
        auto leaf = [&](int k) {
            CVal v;
            if (k < D) {
                v.kind = CVal::CPLX;
                v.re = "xr[" + std::to_string(k) + "]";
                v.im = "xi[" + std::to_string(k) + "]";
            } else {
                const int g = k - D;
                if (!loaded[static_cast<size_t>(g)]) {
                    o << "    const double ft" << g << " = ami::ws_load(ws, ld, " << g << ", off);\n";
                    loaded[static_cast<size_t>(g)] = true;
                }
                v.kind = CVal::REAL;
                v.re = "ft" + std::to_string(g);
            }
            return v;
        };
        int temps = 0;
        CMemo memo;
        const CVal v = horner_c(ts, leaf, o, temps, memo);
        auto comp = [&](bool imag) {
            if (v.kind == CVal::ZERO) return std::string("0.0");
            if (v.kind == CVal::CONST) return imag ? std::string("0.0") : num(v.c);
            if (v.kind == CVal::REAL) return imag ? std::string("0.0") : v.re;
            return imag ? v.im : v.re;
        };
        o << "    acc_re += " << comp(false) << ";\n    acc_im += " << comp(true) << ";\n";
        o << "}\n";
    }

    // the second pass of the two-pass complex forward: as group_accumulate,
    // with each stored FT_g complex (columns g and G + g)
    if (kernels & 1024) {
        o << "__device__ __forceinline__ void group_accumulate_c(const double (&xr)[D], const double (&xi)[D], "
             "const double *ws, int64_t ld, uint32_t off, double &acc_re, double &acc_im) {\n";
        std::vector<HornerTerm> ts;
        for (int g = 0; g < G; ++g) {
            HornerTerm h{1.0, {}};
            for (int j = gbegin(g); j < gend(g); ++j) h.leaves.push_back(tb.group_den_list[j]);
            h.leaves.push_back(D + g);
            ts.push_back(std::move(h));
        }
        std::vector<bool> loaded(static_cast<size_t>(G), false);
        auto leaf = [&](int k) {
            CVal v;
            v.kind = CVal::CPLX;
            if (k < D) {
                v.re = "xr[" + std::to_string(k) + "]";
                v.im = "xi[" + std::to_string(k) + "]";
            } else {
                const int g = k - D;
                if (!loaded[static_cast<size_t>(g)]) {
                    o << "    const double ftr" << g << " = ami::ws_load(ws, ld, " << g << ", off), fti" << g
                      << " = ami::ws_load(ws, ld, " << G + g << ", off);\n";
                    loaded[static_cast<size_t>(g)] = true;
                }
                v.re = "ftr" + std::to_string(g);
                v.im = "fti" + std::to_string(g);
            }
            return v;
        };
        int temps = 0;
        CMemo memo;
        const CVal v = horner_c(ts, leaf, o, temps, memo);
        auto comp = [&](bool imag) {
            if (v.kind == CVal::ZERO) return std::string("0.0");
            if (v.kind == CVal::CONST) return imag ? std::string("0.0") : num(v.c);
            if (v.kind == CVal::REAL) return imag ? std::string("0.0") : v.re;
            return imag ? v.im : v.re;
        };
        o << "    acc_re += " << comp(false) << ";\n    acc_im += " << comp(true) << ";\n";
        o << "}\n";
    }

    // The adjoint of large solutions in passes (after the two-pass forward's
    // first pass has stored every FT_g and E_j in the workspace [column][sample]:
    // columns 0..G-1 FT_g, G..G+NE-1 E_j, then NE columns of the energy
    // cotangents gathered from the denominators, then G columns of the group-sum
    // cotangents FTB_g).
    const std::string ftb0 = "(G + 2 * NE)";
    if (kernels & 64) {
        // frequency pass, one frequency row: every reciprocal, then per chunk
        // of groups (scheduled apart, so that only one chunk's values are live
        // at a time) each group's R_g, the value FT_g R_g, FTB_g +=
        // Re(conj(c) R_g) (stored; added to the stored value after the first
        // row) and u_g = -FT_g conj(c) R_g summed per denominator of the
        // chunk, then per such denominator the scatter of U_k rho_k
        // FIRST: the first frequency row (FTB_g stored, not added to the stored value)
        o << "template <bool FIRST>\n__device__ __forceinline__ void adj_freq_row(const double (&E)[NE], const double (&wr)["
          << NXA << "], const double (&wi)[" << NXA << "], double cr, double ci, double *ws, int64_t ld, uint32_t off, "
             "double &acc_re, double &acc_im, double (&gE)[NE], double (&gwr)["
          << NXA << "], double (&gwi)[" << NXA << "]) {\n";
        const bool own = kAdjChunkOwnDens;
        if (!own)
            o << "  double xr[D], xi[D];\n  { double dr[D], di[D];\n    den_args(E, wr, wi, dr, di);\n"
                 "#pragma unroll\n    for (int k = 0; k < D; ++k) {\n"
                 "      const double inv = ami::rcp_nr(fma(dr[k], dr[k], di[k] * di[k]));\n"
                 "      xr[k] = dr[k] * inv;\n      xi[k] = -di[k] * inv;\n    } }\n";
        for (int g0 = 0; g0 < G; g0 += kAdjChunkGroups) {
            const int g1 = std::min(G, g0 + kAdjChunkGroups);
            std::vector<int> ks;
            for (int g = g0; g < g1; ++g)
                for (int j = gbegin(g); j < gend(g); ++j) ks.push_back(tb.group_den_list[j]);
            std::sort(ks.begin(), ks.end());
            ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
            o << "  {\n";
            if (own) {
                // the chunk's own reciprocals
                o << "    double xr[D], xi[D];\n";
                for (int k : ks) {
                    Lin re, im;
                    for (int i = 0; i < ne; ++i) re.add(tb.den_coef[static_cast<size_t>(k) * nc + i], idx("E", i));
                    for (int x = 0; x < nx; ++x) {
                        const double a = tb.den_coef[static_cast<size_t>(k) * nc + ne + x];
                        re.add(a, idx("wr", x));
                        im.add(a, idx("wi", x));
                    }
                    o << "    { const double dr = " << re.str() << ", di = " << im.str()
                      << ";\n      const double inv = ami::rcp_nr(fma(dr, dr, di * di));\n      xr[" << k
                      << "] = dr * inv;\n      xi[" << k << "] = -di * inv; }\n";
                }
            }
            for (int k : ks) o << "    double Ur" << k << " = 0.0, Ui" << k << " = 0.0;\n";
            for (int g = g0; g < g1; ++g) {
                o << "    { const double ft = ami::ws_load(ws, ld, " << g << ", off);\n";
                o << "      double rr = 1.0, ri = 0.0, nr = 0.0;\n";
                for (int j = gbegin(g); j < gend(g); ++j) {
                    const std::string k = std::to_string(tb.group_den_list[j]);
                    if (j == gbegin(g)) o << "      rr = xr[" << k << "]; ri = xi[" << k << "];\n";
                    else
                        o << "      nr = fma(rr, xr[" << k << "], -ri * xi[" << k << "]); ri = fma(rr, xi[" << k
                          << "], ri * xr[" << k << "]); rr = nr;\n";
                }
                o << "      (void)nr;\n";
                o << "      acc_re = fma(ft, rr, acc_re);\n      acc_im = fma(ft, ri, acc_im);\n";
                o << "      const double tb = fma(cr, rr, ci * ri);\n";
                o << "      if constexpr (FIRST) ami::ws_store(ws, ld, " << ftb0 << " + " << g << ", off, tb);\n"
                  << "      else ami::ws_store(ws, ld, " << ftb0 << " + " << g << ", off, ami::ws_load(ws, ld, " << ftb0
                  << " + " << g << ", off) + tb);\n";
                o << "      const double qr = ft * cr, qi = -ft * ci;\n";
                o << "      const double ur = -fma(qr, rr, -qi * ri), ui = -fma(qr, ri, qi * rr);\n";
                for (int j = gbegin(g); j < gend(g); ++j) {
                    const std::string k = std::to_string(tb.group_den_list[j]);
                    o << "      Ur" << k << " += ur; Ui" << k << " += ui;\n";
                }
                o << "    }\n";
            }
            for (int k : ks) {
                o << "    { const double dR = fma(Ur" << k << ", xr[" << k << "], -Ui" << k << " * xi[" << k
                  << "]), dI = fma(Ur" << k << ", xi[" << k << "], Ui" << k << " * xr[" << k << "]);\n";
                for (int i = 0; i < ne; ++i) {
                    const double c = tb.den_coef[static_cast<size_t>(k) * nc + i];
                    if (c == 1.0) o << "      gE[" << i << "] += dR;\n";
                    else if (c == -1.0) o << "      gE[" << i << "] -= dR;\n";
                    else if (c != 0.0) o << "      gE[" << i << "] = fma(" << num(c) << ", dR, gE[" << i << "]);\n";
                }
                for (int x = 0; x < nx; ++x) {
                    const double a = tb.den_coef[static_cast<size_t>(k) * nc + ne + x];
                    if (a == 0.0) continue;
                    o << "      gwr[" << x << "] = fma(" << num(a) << ", dR, gwr[" << x << "]);\n";
                    o << "      gwi[" << x << "] = fma(" << num(a) << ", dI, gwi[" << x << "]);\n";
                }
                o << "    }\n";
            }
            o << "  }\n";
            if (g1 < G) o << "  AMI_SCHED_FENCE();\n";
        }
        o << "}\n";
    }
    // The leaf passes' parts: each group's terms nested in parts of at most
    // kAdjLeafPartTerms (consecutive in canonical order), with the leaves
    // each part reads and the first and last part that reads each leaf.
    struct Part {
        int g;
        std::vector<HNode> nodes;
        HRef root;
        std::vector<int> leaves;
    };
    auto build_parts = [&](std::vector<Part> &parts, std::vector<int> &first_use, std::vector<int> &last_use,
                           int part_terms) {
        for (int g = 0; g < G; ++g) {
            for (int t0 = tb.group_start[g]; t0 < tb.group_start[g + 1]; t0 += part_terms) {
                const int t1 = std::min(tb.group_start[g + 1], t0 + part_terms);
                std::vector<HornerTerm> ts;
                for (int ti = t0; ti < t1; ++ti) {
                    HornerTerm h{tb.term_sign[ti], {}};
                    for (int j = 0; j < ni; ++j) h.leaves.push_back(tb.term_leaf[static_cast<size_t>(ti) * ni + j]);
                    ts.push_back(std::move(h));
                }
                Part pt;
                pt.g = g;
                pt.root = horner_build(std::move(ts), pt.nodes);
                std::vector<int> used;
                auto note = [&](const HRef &r) {
                    if (r.kind == HRef::LEAF) used.push_back(r.idx);
                };
                note(pt.root);
                for (const HNode &n : pt.nodes) {
                    used.push_back(n.a);
                    note(n.w);
                    note(n.u);
                }
                std::sort(used.begin(), used.end());
                used.erase(std::unique(used.begin(), used.end()), used.end());
                pt.leaves = used;
                parts.push_back(std::move(pt));
            }
        }
        first_use.assign(static_cast<size_t>(L), -1);
        last_use.assign(static_cast<size_t>(L), -1);
        for (size_t p = 0; p < parts.size(); ++p)
            for (int l : parts[p].leaves) {
                if (first_use[l] < 0) first_use[l] = static_cast<int>(p);
                last_use[l] = static_cast<int>(p);
            }
    };
    if (kernels & 128) {
        // leaf pass: FB_l = sum_g FTB_g dFT_g/dF_l by a reverse sweep of each
        // group's nested sum (the nodes recomputed, then their cotangents in
        // reverse order: node h = F_a w + u passes h' w to F_a, h' F_a to w and
        // h' to u).  A group's terms are nested in parts of at most
        // kAdjLeafPartTerms (consecutive in canonical order), which bounds the
        // node values live in a sweep; each leaf is formed just before the
        // first part that reads it and its cotangent is scattered to the
        // energies and to beta just after the last one.
        std::vector<Part> parts;
        std::vector<int> first_use, last_use;
        build_parts(parts, first_use, last_use, kAdjLeafPartTerms);
        o << "__device__ __forceinline__ void leaf_pass(const double (&E)[NE], double beta, double e_reg, const double "
             "*ws, int64_t ld, uint32_t off, double (&gE)[NE], double &gbeta) {\n";
        o << kReverseContract;
        o << "  (void)e_reg;\n";
        // with Taylor-coefficient leaves DV holds dT/dx and DB dT/dbeta
        for (int l = 0; l < L; ++l)
            o << "  double F" << l << ", FB" << l << ", DV" << l << (taylor ? ", DB" + std::to_string(l) : "") << ";\n";
        auto leaf_arg = [&](int l) {
            Lin x;
            for (int i = 0; i < ne; ++i) x.add(tb.leaf_coef[static_cast<size_t>(l) * ne + i], idx("E", i));
            return x.str() + (tb.leaf_sigma[l] < 0 ? " + e_reg" : "");
        };
        auto fname = [](int l) { return "F" + std::to_string(l); };
        for (size_t p = 0; p < parts.size(); ++p) {
            const Part &pt = parts[p];
            for (int l : pt.leaves) {
                if (first_use[l] != static_cast<int>(p)) continue;
                if (taylor) {
                    const int jo = tb.leaf_order[l];
                    o << "  { const double x = " << leaf_arg(l) << ";\n    double f, m, tn = 0.0;\n    ami::leaf_pair("
                      << (tb.leaf_sigma[l] < 0 ? "true" : "false") << ", beta * x, f, m);\n";
                    o << taylor_expr(jo, "F" + std::to_string(l), "    ") << taylor_expr(jo + 1, "tn", "    ");
                    o << "    DV" << l << " = " << num(static_cast<double>(jo + 1)) << " * tn;\n    DB" << l << " = fma("
                      << num(static_cast<double>(jo)) << ", F" << l << ", x * DV" << l << ") / beta; }\n  FB" << l
                      << " = 0.0;\n";
                } else {
                    o << "  ami::leaf_and_slope(" << (tb.leaf_sigma[l] < 0 ? "true" : "false") << ", beta * ("
                      << leaf_arg(l) << "), F" << l << ", DV" << l << ");\n  FB" << l << " = 0.0;\n";
                }
            }
            o << "  { const double tb = ami::ws_load(ws, ld, " << ftb0 << " + " << pt.g << ", off);\n";
            horner_emit(pt.nodes, fname, o);
            const size_t nn = pt.nodes.size();
            for (size_t k = 0; k < nn; ++k) o << "    double hb" << k << " = 0.0;\n";
            // a cotangent c passed to reference r: hb += c (node) or FB += c (leaf)
            auto pass = [&](const HRef &r, const std::string &c) {
                if (r.kind == HRef::NODE) o << "    hb" << r.idx << (r.neg ? " -= " : " += ") << c << ";\n";
                else if (r.kind == HRef::LEAF) o << "    FB" << r.idx << (r.neg ? " -= " : " += ") << c << ";\n";
            };
            pass(pt.root, "tb");
            for (size_t kk = nn; kk-- > 0;) {
                const HNode &n = pt.nodes[kk];
                const std::string hb = "hb" + std::to_string(kk), fa = fname(n.a), fb = "FB" + std::to_string(n.a);
                if (n.w.kind == HRef::CONST) {
                    if (n.w.c == 1.0) o << "    " << fb << " += " << hb << ";\n";
                    else if (n.w.c == -1.0) o << "    " << fb << " -= " << hb << ";\n";
                    else o << "    " << fb << " = fma(" << num(n.w.c) << ", " << hb << ", " << fb << ");\n";
                } else {
                    const std::string wn = href_name(n.w, fname);
                    o << "    " << fb << " = fma(" << (n.w.neg ? "-" : "") << wn << ", " << hb << ", " << fb << ");\n";
                    pass(n.w, fa + " * " + hb);
                }
                pass(n.u, hb);
            }
            o << "  }\n";
            for (int l : pt.leaves) {
                if (last_use[l] != static_cast<int>(p)) continue;
                if (taylor)
                    o << "  { gbeta = fma(FB" << l << ", DB" << l << ", gbeta);\n    const double v = FB" << l << " * DV"
                      << l << ";\n";
                else
                    o << "  { const double fb = FB" << l << " * DV" << l << ";\n    gbeta = fma(fb, " << leaf_arg(l)
                      << ", gbeta);\n    const double v = fb * beta;\n";
                for (int i = 0; i < ne; ++i) {
                    const double c = tb.leaf_coef[static_cast<size_t>(l) * ne + i];
                    if (c == 1.0) o << "    gE[" << i << "] += v;\n";
                    else if (c == -1.0) o << "    gE[" << i << "] -= v;\n";
                    else if (c != 0.0) o << "    gE[" << i << "] = fma(" << num(c) << ", v, gE[" << i << "]);\n";
                }
                o << "  }\n";
            }
            if ((p + 1) % kAdjLeafFenceParts == 0 && p + 1 < parts.size()) o << "  AMI_SCHED_FENCE();\n";
        }
        o << "}\n";
    }

    // The adjoint at complex energies in passes (after the complex two-pass
    // forward's first pass stored FT_g and E_j, both complex, in the
    // workspace: columns [0, G) Re FT, [G, 2G) Im FT, [2G, 2G + NE) Re E,
    // [2G + NE, 2G + 2NE) Im E, then the denominators' energy cotangents
    // (re NE, im NE) and the group-sum cotangents FTB_g (re G, im G)).  The
    // cotangents are complex, Xbar = dL/dRe X + i dL/dIm X.
    const std::string cge0 = "(2 * G + 2 * NE)", cftb0 = "(2 * G + 4 * NE)";
    if (kernels & 2048) {
        // frequency pass, one frequency row: per chunk of groups its own
        // reciprocals (the energies' imaginary parts in the denominators),
        // each group's R_g, the value FT_g R_g, FTB_g += c conj(R_g) (stored;
        // added to the stored value after the first row), u_g = -FT_g conj(c)
        // R_g summed per denominator, then U_k rho_k = conj(Dbar_k) scattered:
        // its real part to Re Ebar and the frequencies, minus its imaginary
        // part to Im Ebar
        o << "template <bool FIRST>\n__device__ __forceinline__ void cadj_freq_row(const double (&Er)[NE], const double "
             "(&Ei)[NE], const double (&wr)["
          << NXA << "], const double (&wi)[" << NXA << "], double cr, double ci, double *ws, int64_t ld, uint32_t off, "
             "double &acc_re, double &acc_im, double (&gEr)[NE], double (&gEi)[NE], double (&gwr)["
          << NXA << "], double (&gwi)[" << NXA << "]) {\n";
        for (int g0 = 0; g0 < G; g0 += kAdjChunkGroups) {
            const int g1 = std::min(G, g0 + kAdjChunkGroups);
            std::vector<int> ks;
            for (int g = g0; g < g1; ++g)
                for (int j = gbegin(g); j < gend(g); ++j) ks.push_back(tb.group_den_list[j]);
            std::sort(ks.begin(), ks.end());
            ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
            o << "  {\n    double xr[D], xi[D];\n";
            for (int k : ks) {
                Lin re, im;
                for (int i = 0; i < ne; ++i) {
                    re.add(tb.den_coef[static_cast<size_t>(k) * nc + i], idx("Er", i));
                    im.add(tb.den_coef[static_cast<size_t>(k) * nc + i], idx("Ei", i));
                }
                for (int x = 0; x < nx; ++x) {
                    const double a = tb.den_coef[static_cast<size_t>(k) * nc + ne + x];
                    re.add(a, idx("wr", x));
                    im.add(a, idx("wi", x));
                }
                o << "    { const double dr = " << re.str() << ", di = " << im.str()
                  << ";\n      const double inv = ami::rcp_nr(fma(dr, dr, di * di));\n      xr[" << k
                  << "] = dr * inv;\n      xi[" << k << "] = -di * inv; }\n";
            }
            for (int k : ks) o << "    double Ur" << k << " = 0.0, Ui" << k << " = 0.0;\n";
            for (int g = g0; g < g1; ++g) {
                o << "    { const double ftr = ami::ws_load(ws, ld, " << g << ", off), fti = ami::ws_load(ws, ld, "
                  << G + g << ", off);\n";
                o << "      double rr = 1.0, ri = 0.0, nr = 0.0;\n";
                for (int j = gbegin(g); j < gend(g); ++j) {
                    const std::string k = std::to_string(tb.group_den_list[j]);
                    if (j == gbegin(g)) o << "      rr = xr[" << k << "]; ri = xi[" << k << "];\n";
                    else
                        o << "      nr = fma(rr, xr[" << k << "], -ri * xi[" << k << "]); ri = fma(rr, xi[" << k
                          << "], ri * xr[" << k << "]); rr = nr;\n";
                }
                o << "      (void)nr;\n";
                o << "      acc_re = fma(ftr, rr, fma(-fti, ri, acc_re));\n"
                     "      acc_im = fma(ftr, ri, fma(fti, rr, acc_im));\n";
                o << "      const double tbr = fma(cr, rr, ci * ri), tbi = fma(ci, rr, -cr * ri);\n";
                const std::string cr_ = cftb0 + " + " + std::to_string(g), ci_ = cftb0 + " + " + std::to_string(G + g);
                o << "      if constexpr (FIRST) {\n        ami::ws_store(ws, ld, " << cr_ << ", off, tbr);\n"
                  << "        ami::ws_store(ws, ld, " << ci_ << ", off, tbi);\n      } else {\n"
                  << "        ami::ws_store(ws, ld, " << cr_ << ", off, ami::ws_load(ws, ld, " << cr_ << ", off) + tbr);\n"
                  << "        ami::ws_store(ws, ld, " << ci_ << ", off, ami::ws_load(ws, ld, " << ci_
                  << ", off) + tbi);\n      }\n";
                o << "      const double qr = fma(ftr, cr, fti * ci), qi = fma(fti, cr, -ftr * ci);\n";
                o << "      const double ur = -fma(qr, rr, -qi * ri), ui = -fma(qr, ri, qi * rr);\n";
                for (int j = gbegin(g); j < gend(g); ++j) {
                    const std::string k = std::to_string(tb.group_den_list[j]);
                    o << "      Ur" << k << " += ur; Ui" << k << " += ui;\n";
                }
                o << "    }\n";
            }
            for (int k : ks) {
                o << "    { const double dR = fma(Ur" << k << ", xr[" << k << "], -Ui" << k << " * xi[" << k
                  << "]), dI = fma(Ur" << k << ", xi[" << k << "], Ui" << k << " * xr[" << k << "]);\n";
                for (int i = 0; i < ne; ++i) {
                    const double c = tb.den_coef[static_cast<size_t>(k) * nc + i];
                    if (c == 1.0) o << "      gEr[" << i << "] += dR; gEi[" << i << "] -= dI;\n";
                    else if (c == -1.0) o << "      gEr[" << i << "] -= dR; gEi[" << i << "] += dI;\n";
                    else if (c != 0.0)
                        o << "      gEr[" << i << "] = fma(" << num(c) << ", dR, gEr[" << i << "]); gEi[" << i
                          << "] = fma(" << num(-c) << ", dI, gEi[" << i << "]);\n";
                }
                for (int x = 0; x < nx; ++x) {
                    const double a = tb.den_coef[static_cast<size_t>(k) * nc + ne + x];
                    if (a == 0.0) continue;
                    o << "      gwr[" << x << "] = fma(" << num(a) << ", dR, gwr[" << x << "]);\n";
                    o << "      gwi[" << x << "] = fma(" << num(a) << ", dI, gwi[" << x << "]);\n";
                }
                o << "    }\n";
            }
            o << "  }\n";
            if (g1 < G) o << "  AMI_SCHED_FENCE();\n";
        }
        o << "}\n";
    }
    if (kernels & 4096) {
        // leaf pass at complex energies: the reverse sweep of each part of a
        // group's nested sum in complex arithmetic; a node h = F_a w + u
        // passes hbar conj(w) to F_a, hbar conj(F_a) to w and hbar to u.
        // Each leaf is formed just before the first part that reads it; after
        // the last one its pair again gives S = conj(f'(y)) = -conj(f(y) f(-y)),
        // and V = Fbar S gives xbar = beta V to the energies and
        // Re(conj(V) x) to beta.
        std::vector<Part> parts;
        std::vector<int> first_use, last_use;
        build_parts(parts, first_use, last_use, cadj_part_terms());
        o << "__device__ __forceinline__ void cleaf_pass(const double (&Er)[NE], const double (&Ei)[NE], double beta, "
             "double e_reg, const double *ws, int64_t ld, uint32_t off, double (&gEr)[NE], double (&gEi)[NE], "
             "double &gbeta) {\n";
        o << kReverseContract;
        o << "  (void)e_reg;\n";
        for (int l = 0; l < L; ++l)
            o << "  double Fr" << l << ", Fi" << l << ", FBr" << l << ", FBi" << l << ";\n";
        auto arg = [&](int l, bool imag) {
            Lin x;
            for (int i = 0; i < ne; ++i) x.add(tb.leaf_coef[static_cast<size_t>(l) * ne + i], idx(imag ? "Ei" : "Er", i));
            return x.str() + (!imag && tb.leaf_sigma[l] < 0 ? " + e_reg" : "");
        };
        // names of a reference's value: real and imaginary part (without its sign)
        auto vre = [&](const HRef &r) -> std::string {
            if (r.kind == HRef::LEAF) return "Fr" + std::to_string(r.idx);
            if (r.kind == HRef::NODE) return "h" + std::to_string(r.idx) + "r";
            return r.kind == HRef::CONST ? num(r.c) : std::string("0.0");
        };
        auto vim = [&](const HRef &r) -> std::string {
            if (r.kind == HRef::LEAF) return "Fi" + std::to_string(r.idx);
            if (r.kind == HRef::NODE) return "h" + std::to_string(r.idx) + "i";
            return std::string("0.0");
        };
        auto sg = [](const HRef &r, const std::string &e) { return r.neg ? "(-" + e + ")" : e; };
        for (size_t p = 0; p < parts.size(); ++p) {
            const Part &pt = parts[p];
            for (int l : pt.leaves) {
                if (first_use[l] != static_cast<int>(p)) continue;
                o << "  ami::leaf_complex(" << (tb.leaf_sigma[l] < 0 ? "true" : "false") << ", beta * ("
                  << arg(l, false) << "), beta * (" << arg(l, true) << "), Fr" << l << ", Fi" << l << ");\n  FBr" << l
                  << " = 0.0; FBi" << l << " = 0.0;\n";
            }
            o << "  { const double tbr = ami::ws_load(ws, ld, " << cftb0 << " + " << pt.g
              << ", off), tbi = ami::ws_load(ws, ld, " << cftb0 << " + " << G + pt.g << ", off);\n";
            // forward: node values
            const size_t nn = pt.nodes.size();
            for (size_t k = 0; k < nn; ++k) {
                const HNode &n = pt.nodes[k];
                const std::string far = "Fr" + std::to_string(n.a), fai = "Fi" + std::to_string(n.a);
                // u's parts (signed)
                std::string ur = "0.0", ui = "0.0";
                if (n.u.kind == HRef::CONST) ur = num(n.u.c);
                else if (n.u.kind != HRef::ZERO) {
                    ur = sg(n.u, vre(n.u));
                    ui = sg(n.u, vim(n.u));
                }
                std::string hr, hi;
                if (n.w.kind == HRef::CONST) {
                    hr = "fma(" + num(n.w.c) + ", " + far + ", " + ur + ")";
                    hi = "fma(" + num(n.w.c) + ", " + fai + ", " + ui + ")";
                } else {
                    const std::string wr = sg(n.w, vre(n.w)), wi = sg(n.w, vim(n.w));
                    hr = "fma(" + far + ", " + wr + ", fma(-" + fai + ", " + wi + ", " + ur + "))";
                    hi = "fma(" + far + ", " + wi + ", fma(" + fai + ", " + wr + ", " + ui + "))";
                }
                o << "    const double h" << k << "r = " << hr << ", h" << k << "i = " << hi << ";\n";
            }
            for (size_t k = 0; k < nn; ++k) o << "    double hb" << k << "r = 0.0, hb" << k << "i = 0.0;\n";
            // a cotangent (cr, ci) passed to reference r
            auto pass = [&](const HRef &r, const std::string &cr, const std::string &ci) {
                const char *op = r.neg ? " -= " : " += ";
                if (r.kind == HRef::NODE)
                    o << "    hb" << r.idx << "r" << op << cr << "; hb" << r.idx << "i" << op << ci << ";\n";
                else if (r.kind == HRef::LEAF)
                    o << "    FBr" << r.idx << op << cr << "; FBi" << r.idx << op << ci << ";\n";
            };
            pass(pt.root, "tbr", "tbi");
            for (size_t kk = nn; kk-- > 0;) {
                const HNode &n = pt.nodes[kk];
                const std::string br = "hb" + std::to_string(kk) + "r", bi = "hb" + std::to_string(kk) + "i";
                const std::string far = "Fr" + std::to_string(n.a), fai = "Fi" + std::to_string(n.a);
                const std::string fbr = "FBr" + std::to_string(n.a), fbi = "FBi" + std::to_string(n.a);
                if (n.w.kind == HRef::CONST) {
                    o << "    " << fbr << " = fma(" << num(n.w.c) << ", " << br << ", " << fbr << "); " << fbi
                      << " = fma(" << num(n.w.c) << ", " << bi << ", " << fbi << ");\n";
                } else {
                    // F_a += hbar conj(w) (w with its sign); w += hbar conj(F_a) (sign applied by pass)
                    const std::string wr = sg(n.w, vre(n.w)), wi = sg(n.w, vim(n.w));
                    o << "    " << fbr << " = fma(" << br << ", " << wr << ", fma(" << bi << ", " << wi << ", " << fbr
                      << ")); " << fbi << " = fma(" << bi << ", " << wr << ", fma(-" << br << ", " << wi << ", " << fbi
                      << "));\n";
                    pass(n.w, "fma(" + br + ", " + far + ", " + bi + " * " + fai + ")",
                         "fma(" + bi + ", " + far + ", -" + br + " * " + fai + ")");
                }
                pass(n.u, br, bi);
            }
            o << "  }\n";
            for (int l : pt.leaves) {
                if (last_use[l] != static_cast<int>(p)) continue;
                // the slope from the leaf pair formed again, from opaque copies of
                // its argument (else the compiler merges it with the first
                // evaluation and keeps that one's values live through the sweep)
                const std::string L_ = std::to_string(l);
                o << "  { double yr = beta * (" << arg(l, false) << "), yi = beta * (" << arg(l, true)
                  << ");\n    AMI_OPAQUE(yr); AMI_OPAQUE(yi);\n    double fr, fi, mr, mi;\n    ami::leaf_complex_pair("
                  << (tb.leaf_sigma[l] < 0 ? "true" : "false")
                  << ", yr, yi, fr, fi, mr, mi);\n    const double Sr = -fma(fr, mr, -fi * mi), Si = fma(fr, mi, fi * mr);\n";
                o << "    const double Vr = fma(FBr" << L_ << ", Sr, -FBi" << L_ << " * Si), Vi = fma(FBr" << L_
                  << ", Si, FBi" << L_ << " * Sr);\n";
                o << "    gbeta = fma(Vr, " << arg(l, false) << ", fma(Vi, " << arg(l, true) << ", gbeta));\n";
                o << "    const double vr = Vr * beta, vi = Vi * beta;\n";
                for (int i = 0; i < ne; ++i) {
                    const double c = tb.leaf_coef[static_cast<size_t>(l) * ne + i];
                    if (c == 1.0) o << "    gEr[" << i << "] += vr; gEi[" << i << "] += vi;\n";
                    else if (c == -1.0) o << "    gEr[" << i << "] -= vr; gEi[" << i << "] -= vi;\n";
                    else if (c != 0.0)
                        o << "    gEr[" << i << "] = fma(" << num(c) << ", vr, gEr[" << i << "]); gEi[" << i << "] = fma("
                          << num(c) << ", vi, gEi[" << i << "]);\n";
                }
                o << "  }\n";
            }
            if ((p + 1) % kAdjLeafFenceParts == 0 && p + 1 < parts.size()) o << "  AMI_SCHED_FENCE();\n";
        }
        o << "}\n";
    }

    if (adj_fns) {
    // U_k = sum over the occurrences of k in the groups of u_g
    std::vector<std::vector<int>> occ(D);
    for (int g = 0; g < G; ++g)
        for (int j = gbegin(g); j < gend(g); ++j) occ[tb.group_den_list[j]].push_back(g);
    o << "__device__ __forceinline__ void den_cotangents(const double (&ur)[G], const double (&ui)[G], double "
         "(&Ur)[D], double (&Ui)[D]) {\n";
    o << kReverseContract;
    for (int k = 0; k < D; ++k) {
        Lin r, i;
        for (int g : occ[k]) {
            r.add(1.0, idx("ur", g));
            i.add(1.0, idx("ui", g));
        }
        o << "  Ur[" << k << "] = " << r.str() << ";\n  Ui[" << k << "] = " << i.str() << ";\n";
    }
    o << "}\n";

    // dL/dE_i += e_ki dR_k ; dL/dw_x += a_kx (dR_k, dI_k)
    auto scatter = [&](std::ostream &os, double c, const std::string &dst, const std::string &v) {
        if (c == 0.0) return;
        if (c == 1.0) os << "  " << dst << " += " << v << ";\n";
        else if (c == -1.0) os << "  " << dst << " -= " << v << ";\n";
        else os << "  " << dst << " = fma(" << num(c) << ", " << v << ", " << dst << ");\n";
    };
    o << "__device__ __forceinline__ void den_scatter(const double (&dR)[D], const double (&dI)[D], double (&gE)[NE], "
         "double (&gwr)["
      << NXA << "], double (&gwi)[" << NXA << "]) {\n";
    o << kReverseContract;
    o << "  (void)dR; (void)dI; (void)gE; (void)gwr; (void)gwi;\n";
    for (int k = 0; k < tb.D; ++k) {
        for (int i = 0; i < ne; ++i) scatter(o, tb.den_coef[static_cast<size_t>(k) * nc + i], idx("gE", i), idx("dR", k));
        for (int x = 0; x < nx; ++x) {
            const double a = tb.den_coef[static_cast<size_t>(k) * nc + ne + x];
            scatter(o, a, idx("gwr", x), idx("dR", k));
            scatter(o, a, idx("gwi", x), idx("dI", k));
        }
    }
    o << "}\n";

    // leaf cotangents: by a reverse sweep of each group's nested sum (parts of
    // at most kAdjLeafPartTerms terms, as the leaf pass of the adjoint in
    // passes), or by prefix/suffix products over each term's leaves
    o << "__device__ __forceinline__ void leaf_cotangents(const double (&F)[L], const double (&FTB)[G], double "
         "(&FB)[L]) {\n";
    o << kReverseContract;
    if (nested_part > 0) {
        std::vector<Part> parts;
        std::vector<int> first_use, last_use;
        build_parts(parts, first_use, last_use, nested_part);
        auto fname = [](int l) { return "F[" + std::to_string(l) + "]"; };
        for (size_t p = 0; p < parts.size(); ++p) {
            const Part &pt = parts[p];
            if (p > 0) o << "  AMI_SCHED_FENCE();\n";
            o << "  {\n";
            horner_emit(pt.nodes, fname, o);
            const size_t nn = pt.nodes.size();
            for (size_t k = 0; k < nn; ++k) o << "    double hb" << k << " = 0.0;\n";
            auto pass = [&](const HRef &r, const std::string &c) {
                if (r.kind == HRef::NODE) o << "    hb" << r.idx << (r.neg ? " -= " : " += ") << c << ";\n";
                else if (r.kind == HRef::LEAF) o << "    FB[" << r.idx << "]" << (r.neg ? " -= " : " += ") << c << ";\n";
            };
            pass(pt.root, "FTB[" + std::to_string(pt.g) + "]");
            for (size_t kk = nn; kk-- > 0;) {
                const HNode &n = pt.nodes[kk];
                const std::string hb = "hb" + std::to_string(kk), fa = fname(n.a),
                                  fb = "FB[" + std::to_string(n.a) + "]";
                if (n.w.kind == HRef::CONST) {
                    if (n.w.c == 1.0) o << "    " << fb << " += " << hb << ";\n";
                    else if (n.w.c == -1.0) o << "    " << fb << " -= " << hb << ";\n";
                    else o << "    " << fb << " = fma(" << num(n.w.c) << ", " << hb << ", " << fb << ");\n";
                } else {
                    const std::string wn = href_name(n.w, fname);
                    o << "    " << fb << " = fma(" << (n.w.neg ? "-" : "") << wn << ", " << hb << ", " << fb << ");\n";
                    pass(n.w, fa + " * " + hb);
                }
                pass(n.u, hb);
            }
            o << "  }\n";
        }
        o << "}\n";
    } else {
    for (int g = 0; g < G; ++g) {
        for (int ti = tb.group_start[g]; ti < tb.group_start[g + 1]; ++ti) {
            const double s = tb.term_sign[ti];
            std::vector<int> lv(ni);
            for (int j = 0; j < ni; ++j) lv[j] = tb.term_leaf[static_cast<size_t>(ti) * ni + j];
            // a unit sign goes into the update (a free negation), so that terms
            // sharing leading leaves share their prefix products
            const bool unit = s == 1.0 || s == -1.0;
            const char *sg = s == -1.0 ? "-" : "";
            o << "  { const double p0 = ";
            if (unit) o << "FTB[" << g << "]";
            else o << "FTB[" << g << "] * " << num(s);
            o << ";\n";
            for (int j = 1; j < ni; ++j)
                o << "    const double p" << j << " = p" << j - 1 << " * F[" << lv[j - 1] << "];\n";
            o << "    double q = 1.0;\n";
            for (int j = ni - 1; j >= 0; --j) {
                if (j == ni - 1) o << "    FB[" << lv[j] << "] " << (s == -1.0 ? "-=" : "+=") << " p" << j << ";\n";
                else o << "    FB[" << lv[j] << "] = fma(" << sg << "p" << j << ", q, FB[" << lv[j] << "]);\n";
                if (j > 0) {
                    if (j == ni - 1) o << "    q = F[" << lv[j] << "];\n";
                    else o << "    q *= F[" << lv[j] << "];\n";
                }
            }
            o << "    (void)q; }\n";
        }
    }
    o << "}\n";
    }

    // the same at complex energies: FB_l += sum over the terms holding l of
    // s FTB_g prod_(others) F, in complex arithmetic (the caller passes
    // conj(F), which makes the update FTB_g conj(dFT_g/dF_l))
    if (kernels & 256) {
    o << "__device__ __forceinline__ void leaf_cotangents_c(const double (&Fr)[L], const double (&Fi)[L], const double "
         "(&FTBr)[G], const double (&FTBi)[G], double (&FBr)[L], double (&FBi)[L]) {\n";
    o << kReverseContract;
    if (nested_part > 0) {
        // the reverse sweep of each group's nested sum at the given conj(F):
        // its node values are the conjugates of the true ones (real
        // coefficients), so a node h = F_a w + u passes hbar w to F_a and
        // hbar F_a to w as plain complex products
        std::vector<Part> parts;
        std::vector<int> first_use, last_use;
        build_parts(parts, first_use, last_use, nested_part);
        auto vre = [&](const HRef &r) -> std::string {
            if (r.kind == HRef::LEAF) return "Fr[" + std::to_string(r.idx) + "]";
            if (r.kind == HRef::NODE) return "h" + std::to_string(r.idx) + "r";
            return r.kind == HRef::CONST ? num(r.c) : std::string("0.0");
        };
        auto vim = [&](const HRef &r) -> std::string {
            if (r.kind == HRef::LEAF) return "Fi[" + std::to_string(r.idx) + "]";
            if (r.kind == HRef::NODE) return "h" + std::to_string(r.idx) + "i";
            return std::string("0.0");
        };
        auto sg = [](const HRef &r, const std::string &e) { return r.neg ? "(-" + e + ")" : e; };
        for (size_t p = 0; p < parts.size(); ++p) {
            const Part &pt = parts[p];
            if (p > 0) o << "  AMI_SCHED_FENCE();\n";
            o << "  {\n";
            const size_t nn = pt.nodes.size();
            for (size_t k = 0; k < nn; ++k) {
                const HNode &n = pt.nodes[k];
                const std::string far = "Fr[" + std::to_string(n.a) + "]", fai = "Fi[" + std::to_string(n.a) + "]";
                std::string ur = "0.0", ui = "0.0";
                if (n.u.kind == HRef::CONST) ur = num(n.u.c);
                else if (n.u.kind != HRef::ZERO) {
                    ur = sg(n.u, vre(n.u));
                    ui = sg(n.u, vim(n.u));
                }
                std::string hr, hi;
                if (n.w.kind == HRef::CONST) {
                    hr = "fma(" + num(n.w.c) + ", " + far + ", " + ur + ")";
                    hi = "fma(" + num(n.w.c) + ", " + fai + ", " + ui + ")";
                } else {
                    const std::string wr = sg(n.w, vre(n.w)), wi = sg(n.w, vim(n.w));
                    hr = "fma(" + far + ", " + wr + ", fma(-" + fai + ", " + wi + ", " + ur + "))";
                    hi = "fma(" + far + ", " + wi + ", fma(" + fai + ", " + wr + ", " + ui + "))";
                }
                o << "    const double h" << k << "r = " << hr << ", h" << k << "i = " << hi << ";\n";
            }
            for (size_t k = 0; k < nn; ++k) o << "    double hb" << k << "r = 0.0, hb" << k << "i = 0.0;\n";
            auto pass = [&](const HRef &r, const std::string &cr, const std::string &ci) {
                const char *op = r.neg ? " -= " : " += ";
                if (r.kind == HRef::NODE)
                    o << "    hb" << r.idx << "r" << op << cr << "; hb" << r.idx << "i" << op << ci << ";\n";
                else if (r.kind == HRef::LEAF)
                    o << "    FBr[" << r.idx << "]" << op << cr << "; FBi[" << r.idx << "]" << op << ci << ";\n";
            };
            pass(pt.root, "FTBr[" + std::to_string(pt.g) + "]", "FTBi[" + std::to_string(pt.g) + "]");
            for (size_t kk = nn; kk-- > 0;) {
                const HNode &n = pt.nodes[kk];
                const std::string br = "hb" + std::to_string(kk) + "r", bi = "hb" + std::to_string(kk) + "i";
                const std::string far = "Fr[" + std::to_string(n.a) + "]", fai = "Fi[" + std::to_string(n.a) + "]";
                const std::string fbr = "FBr[" + std::to_string(n.a) + "]", fbi = "FBi[" + std::to_string(n.a) + "]";
                if (n.w.kind == HRef::CONST) {
                    o << "    " << fbr << " = fma(" << num(n.w.c) << ", " << br << ", " << fbr << "); " << fbi
                      << " = fma(" << num(n.w.c) << ", " << bi << ", " << fbi << ");\n";
                } else {
                    const std::string wr = sg(n.w, vre(n.w)), wi = sg(n.w, vim(n.w));
                    o << "    " << fbr << " = fma(" << br << ", " << wr << ", fma(-" << bi << ", " << wi << ", " << fbr
                      << ")); " << fbi << " = fma(" << br << ", " << wi << ", fma(" << bi << ", " << wr << ", " << fbi
                      << "));\n";
                    pass(n.w, "fma(" + br + ", " + far + ", -" + bi + " * " + fai + ")",
                         "fma(" + br + ", " + fai + ", " + bi + " * " + far + ")");
                }
                pass(n.u, br, bi);
            }
            o << "  }\n";
        }
        o << "}\n";
    } else {
    for (int g = 0; g < G; ++g) {
        for (int ti = tb.group_start[g]; ti < tb.group_start[g + 1]; ++ti) {
            const double s = tb.term_sign[ti];
            std::vector<int> lv(ni);
            for (int j = 0; j < ni; ++j) lv[j] = tb.term_leaf[static_cast<size_t>(ti) * ni + j];
            const bool unit = s == 1.0 || s == -1.0;
            const std::string sg = s == -1.0 ? "-" : "";
            auto F = [&](const char *part, int j) { return std::string(part) + "[" + std::to_string(lv[j]) + "]"; };
            o << "  { const double p0r = FTBr[" << g << "]" << (unit ? "" : " * " + num(s)) << ", p0i = FTBi[" << g
              << "]" << (unit ? "" : " * " + num(s)) << ";\n";
            for (int j = 1; j < ni; ++j) {
                const std::string pr = "p" + std::to_string(j - 1) + "r", pi = "p" + std::to_string(j - 1) + "i";
                o << "    const double p" << j << "r = fma(" << pr << ", " << F("Fr", j - 1) << ", -" << pi << " * "
                  << F("Fi", j - 1) << "), p" << j << "i = fma(" << pr << ", " << F("Fi", j - 1) << ", " << pi
                  << " * " << F("Fr", j - 1) << ");\n";
            }
            o << "    double qr = 1.0, qi = 0.0;\n";
            for (int j = ni - 1; j >= 0; --j) {
                const std::string pr = "p" + std::to_string(j) + "r", pi = "p" + std::to_string(j) + "i";
                const std::string fbr = F("FBr", j), fbi = F("FBi", j);
                if (j == ni - 1) {
                    o << "    " << fbr << (s == -1.0 ? " -= " : " += ") << pr << ";\n";
                    o << "    " << fbi << (s == -1.0 ? " -= " : " += ") << pi << ";\n";
                } else {
                    o << "    " << fbr << " = fma(" << sg << pr << ", qr, fma(" << (s == -1.0 ? "" : "-") << pi
                      << ", qi, " << fbr << "));\n";
                    o << "    " << fbi << " = fma(" << sg << pr << ", qi, fma(" << sg << pi << ", qr, " << fbi
                      << "));\n";
                }
                if (j > 0) {
                    if (j == ni - 1) {
                        o << "    qr = " << F("Fr", j) << "; qi = " << F("Fi", j) << ";\n";
                    } else {
                        o << "    { const double tr = fma(qr, " << F("Fr", j) << ", -qi * " << F("Fi", j)
                          << "); qi = fma(qr, " << F("Fi", j) << ", qi * " << F("Fr", j) << "); qr = tr; }\n";
                    }
                }
            }
            o << "    (void)qr; (void)qi; }\n";
        }
    }
    o << "}\n";
    }
    }
    }  // adj_fns

    // the leaves' and lines' scatters: every adjoint kernel (one pass, or the
    // leaf pass of large solutions)
    if (adj_fns || (kernels & 128)) {
    auto scatter = [&](std::ostream &os, double c, const std::string &dst, const std::string &v) {
        if (c == 0.0) return;
        if (c == 1.0) os << "  " << dst << " += " << v << ";\n";
        else if (c == -1.0) os << "  " << dst << " -= " << v << ";\n";
        else os << "  " << dst << " = fma(" << num(c) << ", " << v << ", " << dst << ");\n";
    };
    // dL/dE_i += sum_l c_li v_l
    o << "__device__ __forceinline__ void leaf_scatter(const double (&v)[L], double (&gE)[NE]) {\n";
    o << kReverseContract;
    for (int l = 0; l < L; ++l)
        for (int i = 0; i < ne; ++i) scatter(o, tb.leaf_coef[static_cast<size_t>(l) * ne + i], idx("gE", i), idx("v", l));
    o << "}\n";

    // dL/dk_l += sum_j alpha_jl dL/dK_j
    o << "__device__ __forceinline__ void line_scatter(const double (&gx)[" << NGA << "], const double (&gy)[" << NGA
      << "], double (&gkx)[" << NIA << "], double (&gky)[" << NIA << "]) {\n";
    o << kReverseContract;
    if (hub) {
        for (int j = 0; j < ng; ++j)
            for (int l = 0; l < ni; ++l) {
                const double a = tb.line_alpha[static_cast<size_t>(j) * nf + l];
                scatter(o, a, idx("gkx", l), idx("gx", j));
                scatter(o, a, idx("gky", l), idx("gy", j));
            }
    }
    o << "}\n";
    }  // adjoint scatters
    o << "}  // namespace amijit\n";
    o << "#include \"jit_kernel.hpp\"\n";
    return o.str();
}

std::string jit_batch_source(const std::vector<const AmiTerms *> &items, const std::vector<int> &two_pass,
                             const std::vector<int> &one_row, bool hub, int block, int phases,
                             const std::vector<int> &labels, bool claim_ahead, int waves) {
    std::ostringstream o;
    o << "// generated: persistent batch of " << items.size() << " specialized evaluators\n";
    o << "#include \"kargs.hpp\"\n";
    // the tile functions read the argument blocks through the constant address space
    o << "#define AMI_JIT_ARGS const __attribute__((address_space(4))) ami::KArgs\n";
    const char *const kSettings[] = {"AMI_JIT_HUB", "AMI_JIT_KERNELS", "AMI_JIT_BLOCK", "AMI_JIT_PARK_DV",
                                     "AMI_JIT_ADJ_WAVES", "AMI_JIT_CADJ_WAVES", "AMI_JIT_CADJL_WAVES"};
    bool any_two = false;
    for (size_t j = 0; j < items.size(); ++j) {
        any_two = any_two || two_pass[j];
        std::string src = jit_source(items[j], hub, two_pass[j] ? (16 | 32) : 1);
        // the diagram's functions in a namespace of its own, with its settings
        // and the block of the batch, followed by the tile functions
        std::istringstream in(src);
        std::string line;
        for (const char *m : kSettings) o << "#undef " << m << "\n";
        o << "#define amijit amijit_b" << j << "\n";
        while (std::getline(in, line)) {
            if (line == "#include \"kargs.hpp\"" || line == "#include \"jit_kernel.hpp\"") continue;
            if (line.rfind("#define AMI_JIT_BLOCK ", 0) == 0) line = "#define AMI_JIT_BLOCK " + std::to_string(block);
            o << line << "\n";
        }
        o << "#include \"jit_tiles.hpp\"\n#undef amijit\n";
    }
    // the persistent kernels: every block takes work items (item, first tile,
    // tile count, first frequency row, row count) from its counter until the
    // list is done (every wave sees the counter pass n_work and exits) and runs
    // the item's own tile function on each tile (and row); the first kernel
    // runs the one-pass forward tiles and the two-pass items' first pass, the
    // second their frequency pass.  With claim_ahead the claim of the next
    // work item is issued before the current one runs, so that its round trip
    // overlaps the work.
    o << "namespace amibatch {\n"
         "struct Work {\n  int32_t item, ntiles;\n  int64_t tile0;\n  int32_t f, nf;\n};\n"
         "typedef const __attribute__((address_space(4))) Work *cwork;\n"
         "typedef const __attribute__((address_space(4))) ami::KArgs *cargs;\n"
         "}  // namespace amibatch\n";
    const std::string stride = std::to_string(kBatchCounterStride);
    for (int phase = 1; phase <= 2; ++phase) {
        if (!(phases & phase) || (phase == 2 && !any_two)) continue;
        // eight work lists, one per XCD (xoff[x] .. xoff[x + 1] of work, with
        // their counters kBatchCounterStride apart): a block drains the list
        // of its own XCD first (block b runs on XCD b mod 8), then the others
        // in turn, so every block has tried every list before it exits
        if (waves > 0) o << "__attribute__((amdgpu_waves_per_eu(" << waves << ")))\n";
        o << "extern \"C\" __global__ __launch_bounds__(" << block << ") void ami_batch_p" << phase
          << "(const ami::KArgs *args, const amibatch::Work *work, const int *xoff, unsigned int *counter) {\n"
             "  __shared__ int next;\n"
             "  const amibatch::cwork cw = (amibatch::cwork)(work);\n"
             "  const amibatch::cargs ca = (amibatch::cargs)(args);\n"
             "  const int x0 = static_cast<int>(blockIdx.x & 7u);\n"
             "  for (int k = 0; k < 8; ++k) {\n"
             "   const int x = (x0 + k) & 7, begin = xoff[x], n_work = xoff[x + 1] - begin;\n"
             "   unsigned int *const ctr = counter + " << stride << " * x;\n"
             "   if (threadIdx.x == 0) next = static_cast<int>(atomicAdd(ctr, 1u));\n"
             "   __syncthreads();\n"
             "   int wj = __builtin_amdgcn_readfirstlane(next);\n"
             "   __syncthreads();\n"
             "   while (wj < n_work) {\n";
        if (claim_ahead)
            o << "    unsigned int claim = 0u;\n"
                 "    if (threadIdx.x == 0) claim = atomicAdd(ctr, 1u);\n";
        o << "    const int wi = begin + wj;\n"
             "    const int item = cw[wi].item, ntiles = cw[wi].ntiles, f = cw[wi].f, nf = cw[wi].nf;\n"
             "    const int64_t tile0 = cw[wi].tile0;\n"
             "    const __attribute__((address_space(4))) ami::KArgs &a = ca[item];\n"
             "    (void)f;\n"
             "    (void)nf;\n"
             "    switch (item) {\n";
        for (size_t j = 0; j < items.size(); ++j) {
            const std::string ns = "amijit_b" + std::to_string(j);
            const std::string h = hub ? "true" : "false";
            const int label = labels.empty() ? static_cast<int>(j) : labels[j];
            if (phase == 1) {
                o << "    case " << label << ":\n      for (int64_t t = tile0; t < tile0 + ntiles; ++t) {\n"
                  << "        asm volatile(\"\" ::: \"memory\");   // each tile loads its own inputs\n        ";
                if (two_pass[j]) o << ns << "::sums_tile<" << h << ">(a, t);\n";
                else o << ns << "::fwd_tile<" << h << ", " << (one_row[j] ? "true" : "false") << ">(a, t);\n";
                o << "      }\n      break;\n";
            } else if (two_pass[j]) {
                o << "    case " << label << ":\n      for (int64_t t = tile0; t < tile0 + ntiles; ++t)\n"
                  << "        for (int r = f; r < f + nf; ++r) {\n"
                  << "          asm volatile(\"\" ::: \"memory\");   // each row loads its own inputs\n"
                  << "          " << ns << "::freq_tile(a, t, r);\n        }\n      break;\n";
            }
        }
        o << "    default: break;\n    }\n";
        o << (claim_ahead ? "    if (threadIdx.x == 0) next = static_cast<int>(claim);\n"
                          : "    if (threadIdx.x == 0) next = static_cast<int>(atomicAdd(ctr, 1u));\n");
        o << "    __syncthreads();\n"
             "    wj = __builtin_amdgcn_readfirstlane(next);\n"
             "    __syncthreads();\n"
             "   }\n  }\n}\n";
    }
    return o.str();
}

}  // namespace ami

extern "C" AmiStatus amiBatchSource(AmiTerms *const *terms, int32_t n, const int64_t *n_f, int32_t momentum,
                                    int32_t compile, char *buf, int64_t cap, int64_t *len) {
    using namespace ami;
    clear_error();
    if (!terms || !n_f || !len || n < 1) return fail(AMI_E_ARG, "NULL argument or no items");
    const bool hub = momentum != 0;
    std::vector<const AmiTerms *> ts;
    std::vector<int> two, one;
    for (int i = 0; i < n; ++i) {
        if (!terms[i]) return fail(AMI_E_ARG, "terms[" + std::to_string(i) + "] is NULL");
        two.push_back(jit_prefers_two_pass(terms[i]) ? 1 : 0);
        std::string why;
        if (!jit_supported(terms[i], hub, &why, two.back() != 0))
            return fail(AMI_E_UNSUPPORTED, "item " + std::to_string(i) + ": no specialized kernel: " + why);
        ts.push_back(terms[i]);
        one.push_back(n_f[i] == 1 ? 1 : 0);
    }
    const std::string src = jit_batch_source(ts, two, one, hub, 256, 3, {});
    if (compile) {
        std::vector<char> code;
        std::string err;
        const AmiStatus st = code_from_source(src, code, err);
        if (st != AMI_OK) return fail(st, err);
    }
    *len = static_cast<int64_t>(src.size()) + 1;
    if (!buf) return AMI_OK;
    if (cap < *len) return fail(AMI_E_ARG, "buffer too small");
    std::memcpy(buf, src.c_str(), src.size() + 1);
    return AMI_OK;
}

extern "C" AmiStatus amiTermsSource(const AmiTerms *t, int32_t momentum, char *buf, int64_t cap, int64_t *len) {
    using namespace ami;
    clear_error();
    if (!t || !len) return fail(AMI_E_ARG, "NULL argument");
    if (momentum < 0 || momentum > 3) return fail(AMI_E_ARG, "momentum must be 0..3");
    const bool hub = (momentum & 1) != 0, two_pass = (momentum & 2) != 0;
    std::string why;
    if (!jit_supported(t, hub, &why, two_pass)) return fail(AMI_E_UNSUPPORTED, "no specialized kernel: " + why);
    int kernels = two_pass ? (hub ? 48 | 64 | 128 : 48 | 64 | 128 | 512 | 1024 | 2048 | 4096) : hub ? 7 : 11 | 256;
    for (int o : t->tab.leaf_order)
        if (o > 0) kernels &= ~(8 | 256 | 512 | 1024 | 2048 | 4096);   // Taylor-coefficient leaves: no complex energies
    const std::string src = jit_source(t, hub, kernels);
    *len = static_cast<int64_t>(src.size()) + 1;
    if (!buf) return AMI_OK;
    if (cap < *len) return fail(AMI_E_ARG, "buffer too small");
    std::memcpy(buf, src.c_str(), src.size() + 1);
    return AMI_OK;
}
