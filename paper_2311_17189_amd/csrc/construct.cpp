// Host-side symbolic construction of the AMI solution (Burke & LeBlanc,
// arXiv 2311.17189, Sec. 2.2) and its flattening into evaluation tables.
//
//  * Each Matsubara sum over nu_p (p = 0..n_int-1, in slot order, Sec. 5.1.1)
//    is done with the residue theorem Eq. (3): every denominator holding nu_p
//    with coefficient c = +-1 has a simple pole at
//        z = -c * (eps.E + sum_{l != p} alpha_l w_l)          (Eq. (4), sign of Eq. (2))
//    whose residue is 1/c = c times the other denominators evaluated at z.
//    The pole's Fermi function keeps only its energy part: for Matsubara
//    frequencies exp(beta i nu) is -1 (fermionic) or +1 (bosonic), so
//    f(z) = 1/(sigma exp(beta x) + 1) with sigma = (-1)^(sum of the pole's
//    fermionic frequency coefficients).
//  * Terms A * FT * R (Eq. (6)) are kept flat (FACTORIZE=false) and put in a
//    canonical order; with AMI_FACTORIZE the Fermi tree of Sec. 2.1 / Fig. 1 is
//    built as well by collecting, after every sum, the poles that leave equal
//    denominators.
//  * The canonical terms are flattened into tables with every distinct leaf
//    and denominator stored once, and terms grouped by their denominators
//    (FT_g * R_g), which is what the HIP kernels evaluate.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "ami_internal.hpp"

namespace ami {

namespace {

struct BuildError {
    AmiStatus st;
    std::string msg;
};

// A term during construction: prefactor, leaves so far, remaining denominators.
struct Work {
    int s = 1;
    std::vector<int> leaves;   // records of 1 + n_eps ints
    std::vector<int> dens;     // records of n_eps + n_freq ints
};

class Builder {
public:
    Builder(int n_eps, int n_freq, const std::vector<uint8_t> &fermionic, bool multipole = false)
        : ne_(n_eps), nf_(n_freq), rec_(n_eps + n_freq), ferm_(fermionic), multi_(multipole) {}

    int rec() const { return rec_; }

    // Residues of the sum over slot p of one product of denominators.  Each
    // result is (c, leaf record, remaining denominators after substitution).
    struct Child {
        int c;
        std::vector<int> leaf;
        std::vector<int> dens;
    };

    // Poles of slot p: each distinct pole z0 (the zero of the denominators
    // D_r = c_r (z - z0), c_r = +-1, that share it; M of them) gives, with
    // j + sum_q k_q = M - 1 over the other denominators q that hold nu_p
    // (coefficient a_q, multiplicity m_q after substitution), the residue term
    //   prod_r c_r * T_j(x0) * prod_q (-a_q)^k_q C(m_q + k_q - 1, k_q) D_q(z0)^-(m_q + k_q)
    // (Eq. (5) by the Leibniz rule; T_j the j-th Taylor coefficient of the
    // pole's Fermi/Bose function, leaf code sigma (1 + j)).  M = 1 is Eq. (3)
    // with Eq. (4).  Without multipole support a shared pole is an error.
    void residues(const std::vector<int> &dens, int p, std::vector<Child> &out) const {
        const int m = static_cast<int>(dens.size()) / rec_;
        std::vector<int> P;
        for (int r = 0; r < m; ++r)
            if (dens[r * rec_ + ne_ + p] != 0) P.push_back(r);
        if (P.empty())
            throw BuildError{AMI_E_LABEL, "summed frequency " + std::to_string(p) +
                                              " appears in no denominator of a term"};
        std::vector<std::vector<int>> poles;       // distinct pole records, first-appearance order
        std::vector<std::vector<int>> members;     // denominators of each pole
        for (int r : P) {
            const int c = dens[r * rec_ + ne_ + p];
            if (c != 1 && c != -1)
                throw BuildError{AMI_E_COEFF, "summed frequency " + std::to_string(p) +
                                                  " has coefficient " + std::to_string(c)};
            std::vector<int> z(rec_);
            for (int i = 0; i < rec_; ++i) z[i] = -c * dens[r * rec_ + i];
            z[ne_ + p] = 0;
            size_t k = 0;
            while (k < poles.size() && poles[k] != z) ++k;
            if (k < poles.size() && !multi_)
                throw BuildError{AMI_E_MULTIPOLE, "two denominators share a pole in frequency " +
                                                      std::to_string(p)};
            if (k == poles.size()) {
                poles.push_back(std::move(z));
                members.emplace_back();
            }
            members[k].push_back(r);
        }
        for (size_t k = 0; k < poles.size(); ++k) {
            const std::vector<int> &z = poles[k];
            const std::vector<int> &grp = members[k];
            const int M = static_cast<int>(grp.size());
            int pref = 1;
            for (int r : grp) pref *= dens[r * rec_ + ne_ + p];
            int parity = 0;
            for (int l = 0; l < nf_; ++l)
                if (ferm_[l]) parity += z[ne_ + l];
            const int sigma = (std::abs(parity) % 2 == 0) ? 1 : -1;
            // the other denominators at the pole: fixed ones (no nu_p) and
            // moving ones keyed by (substituted record, nu_p coefficient)
            std::vector<int> fixed;
            std::vector<std::pair<std::vector<int>, int>> mkey;   // (record, a_q)
            std::vector<int> mult;
            for (int q = 0; q < m; ++q) {
                if (std::find(grp.begin(), grp.end(), q) != grp.end()) continue;
                const int mq = dens[q * rec_ + ne_ + p];
                std::vector<int> rec(dens.begin() + q * rec_, dens.begin() + (q + 1) * rec_);
                if (mq == 0) {
                    fixed.insert(fixed.end(), rec.begin(), rec.end());
                    continue;
                }
                for (int i = 0; i < rec_; ++i) rec[i] += mq * z[i];
                rec[ne_ + p] = 0;
                size_t u = 0;
                while (u < mkey.size() && !(mkey[u].first == rec && mkey[u].second == mq)) ++u;
                if (u == mkey.size()) {
                    mkey.emplace_back(std::move(rec), mq);
                    mult.push_back(0);
                }
                ++mult[u];
            }
            // every split j + sum_u k_u = M - 1
            const int nu = static_cast<int>(mkey.size());
            std::vector<int> ks(nu, 0);
            for (;;) {
                int used = 0;
                for (int x : ks) used += x;
                if (used <= M - 1) {
                    const int j = M - 1 - used;
                    long long coef = pref;
                    Child ch;
                    ch.dens = fixed;
                    for (int u = 0; u < nu; ++u) {
                        const int a = mkey[u].second, kk = ks[u], mu = mult[u];
                        long long binom = 1;
                        for (int i = 0; i < kk; ++i) binom = binom * (mu + i) / (i + 1);
                        for (int i = 0; i < kk; ++i) coef *= -a;
                        coef *= binom;
                        for (int i = 0; i < mu + kk; ++i)
                            ch.dens.insert(ch.dens.end(), mkey[u].first.begin(), mkey[u].first.end());
                    }
                    if (coef > INT32_MAX || coef < INT32_MIN)
                        throw BuildError{AMI_E_COEFF, "residue prefactor overflows int32"};
                    ch.c = static_cast<int>(coef);
                    ch.leaf.resize(1 + ne_);
                    ch.leaf[0] = sigma * (1 + j);
                    for (int i = 0; i < ne_; ++i) ch.leaf[1 + i] = z[i];
                    out.push_back(std::move(ch));
                }
                // next tuple of ks (odometer over 0..M-1)
                int u = 0;
                while (u < nu && ks[u] == M - 1) ks[u++] = 0;
                if (u == nu) break;
                ++ks[u];
            }
        }
    }

    // Sign-normalize every denominator (first non-zero coefficient positive) and
    // sort them; returns the accumulated sign.
    int normalize_dens(std::vector<int> &dens) const {
        const int m = static_cast<int>(dens.size()) / rec_;
        int sign = 1;
        std::vector<std::vector<int>> recs(m);
        for (int r = 0; r < m; ++r) {
            recs[r].assign(dens.begin() + r * rec_, dens.begin() + (r + 1) * rec_);
            for (int i = 0; i < rec_; ++i) {
                if (recs[r][i] == 0) continue;
                if (recs[r][i] < 0) {
                    for (int &x : recs[r]) x = -x;
                    sign = -sign;
                }
                break;
            }
        }
        std::sort(recs.begin(), recs.end());
        dens.clear();
        for (auto &r : recs) dens.insert(dens.end(), r.begin(), r.end());
        return sign;
    }

    void sort_leaves(std::vector<int> &leaves) const {
        const int lr = 1 + ne_;
        const int m = static_cast<int>(leaves.size()) / lr;
        std::vector<std::vector<int>> recs(m);
        for (int r = 0; r < m; ++r) recs[r].assign(leaves.begin() + r * lr, leaves.begin() + (r + 1) * lr);
        std::sort(recs.begin(), recs.end());
        leaves.clear();
        for (auto &r : recs) leaves.insert(leaves.end(), r.begin(), r.end());
    }

private:
    int ne_, nf_, rec_;
    std::vector<uint8_t> ferm_;
    bool multi_;
};

std::vector<int> initial_dens(const AmiTerms *t) {
    std::vector<int> d;
    d.reserve(static_cast<size_t>(t->n_g) * (t->n_eps + t->n_freq));
    for (int j = 0; j < t->n_g; ++j) {
        for (int i = 0; i < t->n_eps; ++i) d.push_back(t->eps[j * t->n_eps + i]);
        for (int l = 0; l < t->n_freq; ++l) d.push_back(t->alpha[j * t->n_freq + l]);
    }
    return d;
}

// Canonical merge of flat terms: key = sorted leaves ++ normalized sorted dens.
std::vector<FlatTerm> canonicalize(const Builder &b, std::vector<Work> &work, int n_eps) {
    std::map<std::vector<int>, long long> merged;
    size_t leaf_len = 0;
    for (auto &w : work) {
        const int sign = b.normalize_dens(w.dens);
        b.sort_leaves(w.leaves);
        std::vector<int> key(w.leaves);
        key.insert(key.end(), w.dens.begin(), w.dens.end());
        leaf_len = w.leaves.size();
        merged[key] += static_cast<long long>(w.s) * sign;
    }
    (void)n_eps;
    std::vector<FlatTerm> out;
    out.reserve(merged.size());
    for (auto &kv : merged) {
        if (kv.second == 0) continue;
        if (kv.second > INT32_MAX || kv.second < INT32_MIN)
            throw BuildError{AMI_E_COEFF, "merged prefactor overflows int32"};
        FlatTerm ft;
        ft.s = static_cast<int>(kv.second);
        ft.leaves.assign(kv.first.begin(), kv.first.begin() + leaf_len);
        ft.dens.assign(kv.first.begin() + leaf_len, kv.first.end());
        out.push_back(std::move(ft));
    }
    return out;
}

void check_ranges(const std::vector<FlatTerm> &terms) {
    for (const auto &t : terms) {
        for (int x : t.leaves)
            if (x > 127 || x < -127) throw BuildError{AMI_E_COEFF, "leaf coefficient exceeds int8"};
        for (int x : t.dens)
            if (x > 127 || x < -127) throw BuildError{AMI_E_COEFF, "denominator coefficient exceeds int8"};
    }
}

void construct_flat(AmiTerms *t) {
    Builder b(t->n_eps, t->n_freq, t->fermionic, (t->flags & AMI_MULTIPOLE) != 0);
    std::vector<Work> cur(1);
    cur[0].s = 1;
    cur[0].dens = initial_dens(t);
    std::vector<Builder::Child> kids;
    for (int p = 0; p < t->n_int; ++p) {
        std::vector<Work> nxt;
        for (const Work &w : cur) {
            kids.clear();
            b.residues(w.dens, p, kids);
            for (auto &k : kids) {
                Work c;
                c.s = w.s * k.c;
                c.leaves = w.leaves;
                c.leaves.insert(c.leaves.end(), k.leaf.begin(), k.leaf.end());
                c.dens = std::move(k.dens);
                nxt.push_back(std::move(c));
            }
        }
        cur.swap(nxt);
    }
    const int rec = b.rec();
    for (const Work &w : cur) {
        const int m = static_cast<int>(w.dens.size()) / rec;
        for (int r = 0; r < m; ++r) {
            bool zero = true;
            for (int i = 0; i < rec; ++i) zero = zero && (w.dens[r * rec + i] == 0);
            if (zero) throw BuildError{AMI_E_MULTIPOLE, "a denominator vanished identically"};
        }
    }
    t->raw_terms = static_cast<int64_t>(cur.size());
    t->terms = canonicalize(b, cur, t->n_eps);
    check_ranges(t->terms);
}

// ---- factorized Fermi tree --------------------------------------------------

int add_node(AmiTerms *t, TreeNode n) {
    t->tree.push_back(std::move(n));
    return static_cast<int>(t->tree.size()) - 1;
}

void construct_tree(AmiTerms *t) {
    Builder b(t->n_eps, t->n_freq, t->fermionic);
    t->tree.clear();
    t->tree_terms.clear();
    TreeNode one;
    one.kind = TreeNode::ONE;
    const int one_id = add_node(t, one);
    std::vector<TreeTerm> cur(1);
    cur[0].node = one_id;
    cur[0].dens = initial_dens(t);
    std::vector<Builder::Child> kids;
    for (int p = 0; p < t->n_int; ++p) {
        std::map<std::vector<int>, size_t> gindex;
        std::vector<std::pair<std::vector<int>, std::vector<int>>> groups;  // key, part nodes
        for (const TreeTerm &tt : cur) {
            kids.clear();
            b.residues(tt.dens, p, kids);
            std::map<std::vector<int>, size_t> lindex;
            std::vector<std::pair<std::vector<int>, TreeNode>> local;  // key, ADD node
            for (auto &k : kids) {
                const int sign = b.normalize_dens(k.dens);
                TreeNode leaf;
                leaf.kind = TreeNode::LEAF;
                leaf.sigma = k.leaf[0];
                leaf.e.assign(k.leaf.begin() + 1, k.leaf.end());
                const int leaf_id = add_node(t, std::move(leaf));
                auto it = lindex.find(k.dens);
                size_t li;
                if (it == lindex.end()) {
                    li = local.size();
                    lindex.emplace(k.dens, li);
                    TreeNode add;
                    add.kind = TreeNode::ADD;
                    local.emplace_back(k.dens, std::move(add));
                } else {
                    li = it->second;
                }
                local[li].second.child.push_back(leaf_id);
                local[li].second.coef.push_back(k.c * sign);
            }
            for (auto &lg : local) {
                int factor = add_node(t, std::move(lg.second));
                int node = factor;
                if (t->tree[tt.node].kind != TreeNode::ONE) {
                    TreeNode mul;
                    mul.kind = TreeNode::MUL;
                    mul.child = {tt.node, factor};
                    node = add_node(t, std::move(mul));
                }
                auto git = gindex.find(lg.first);
                if (git == gindex.end()) {
                    gindex.emplace(lg.first, groups.size());
                    groups.emplace_back(lg.first, std::vector<int>{node});
                } else {
                    groups[git->second].second.push_back(node);
                }
            }
        }
        cur.clear();
        for (auto &g : groups) {
            TreeTerm tt;
            tt.dens = g.first;
            if (g.second.size() == 1) {
                tt.node = g.second[0];
            } else {
                TreeNode add;
                add.kind = TreeNode::ADD;
                add.child = g.second;
                add.coef.assign(g.second.size(), 1);
                tt.node = add_node(t, std::move(add));
            }
            cur.push_back(std::move(tt));
        }
    }
    t->tree_terms = std::move(cur);
}

void expand_node(const AmiTerms *t, int id, std::vector<std::pair<long long, std::vector<int>>> &out) {
    const TreeNode &n = t->tree[id];
    out.clear();
    switch (n.kind) {
    case TreeNode::ONE:
        out.emplace_back(1, std::vector<int>{});
        return;
    case TreeNode::LEAF: {
        std::vector<int> rec(1 + n.e.size());
        rec[0] = n.sigma;
        std::copy(n.e.begin(), n.e.end(), rec.begin() + 1);
        out.emplace_back(1, std::move(rec));
        return;
    }
    case TreeNode::MUL: {
        out.emplace_back(1, std::vector<int>{});
        std::vector<std::pair<long long, std::vector<int>>> sub, acc;
        for (int c : n.child) {
            expand_node(t, c, sub);
            acc.clear();
            for (auto &a : out)
                for (auto &s : sub) {
                    std::vector<int> l(a.second);
                    l.insert(l.end(), s.second.begin(), s.second.end());
                    acc.emplace_back(a.first * s.first, std::move(l));
                }
            out.swap(acc);
        }
        return;
    }
    case TreeNode::ADD: {
        std::vector<std::pair<long long, std::vector<int>>> sub;
        for (size_t k = 0; k < n.child.size(); ++k) {
            expand_node(t, n.child[k], sub);
            for (auto &s : sub) out.emplace_back(s.first * n.coef[k], std::move(s.second));
        }
        return;
    }
    }
}

std::vector<FlatTerm> expand_tree(const AmiTerms *t) {
    Builder b(t->n_eps, t->n_freq, t->fermionic);
    std::vector<Work> work;
    std::vector<std::pair<long long, std::vector<int>>> ex;
    for (const TreeTerm &tt : t->tree_terms) {
        expand_node(t, tt.node, ex);
        for (auto &e : ex) {
            Work w;
            w.s = static_cast<int>(e.first);
            w.leaves = std::move(e.second);
            w.dens = tt.dens;
            work.push_back(std::move(w));
        }
    }
    return canonicalize(b, work, t->n_eps);
}

void serialize(const AmiTerms *t, const std::vector<FlatTerm> &terms, std::vector<int32_t> &out) {
    out.clear();
    const size_t drec = static_cast<size_t>(t->n_eps + t->n_freq);
    bool extended = false;
    for (const auto &ft : terms) extended = extended || ft.dens.size() != terms[0].dens.size();
    out.push_back(t->n_int);
    out.push_back(t->n_eps);
    out.push_back(t->n_freq);
    out.push_back(extended ? -static_cast<int32_t>(terms.size()) : static_cast<int32_t>(terms.size()));
    for (const auto &ft : terms) {
        out.push_back(ft.s);
        if (extended) out.push_back(static_cast<int32_t>(ft.dens.size() / drec));
        out.insert(out.end(), ft.leaves.begin(), ft.leaves.end());
        out.insert(out.end(), ft.dens.begin(), ft.dens.end());
    }
}

}  // namespace

void pack_tables(AmiTerms *t);

// Flatten canonical terms: distinct leaves, distinct denominators (energy part
// and external-frequency part), groups of terms with equal denominators.
AmiStatus build_tables(AmiTerms *t) {
    Tables &tab = t->tab;
    tab = Tables();
    const int ne = t->n_eps, nf = t->n_freq, ni = t->n_int, nx = t->n_ext;
    const int lrec = 1 + ne, drec = ne + nf;
    tab.dpt = t->n_g - ni;
    // uniform: every term holds n_g - n_int denominators and plain leaves (no
    // pole of higher order); the table-driven kernels need it
    tab.uniform = true;
    std::map<std::vector<int>, int> leaf_id, den_id;
    for (const auto &ft : t->terms) {
        const int nd = static_cast<int>(ft.dens.size()) / drec;
        if (nd != tab.dpt) tab.uniform = false;
        for (int j = 0; j < ni; ++j) {
            const int code = ft.leaves[j * lrec];
            if (code != 1 && code != -1) tab.uniform = false;
            leaf_id.emplace(std::vector<int>(ft.leaves.begin() + j * lrec, ft.leaves.begin() + (j + 1) * lrec), 0);
        }
        for (int r = 0; r < nd; ++r) {
            std::vector<int> k(ft.dens.begin() + r * drec, ft.dens.begin() + r * drec + ne);
            k.insert(k.end(), ft.dens.begin() + r * drec + ne + ni, ft.dens.begin() + (r + 1) * drec);
            den_id.emplace(std::move(k), 0);
        }
    }
    int idx = 0;
    for (auto &kv : leaf_id) {
        kv.second = idx++;
        tab.leaf_sigma.push_back(kv.first[0] > 0 ? 1.0 : -1.0);
        tab.leaf_order.push_back(std::abs(kv.first[0]) - 1);
        for (int i = 0; i < ne; ++i) tab.leaf_coef.push_back(static_cast<double>(kv.first[1 + i]));
    }
    tab.L = idx;
    idx = 0;
    for (auto &kv : den_id) {
        kv.second = idx++;
        for (int v : kv.first) tab.den_coef.push_back(static_cast<double>(v));
    }
    tab.D = idx;
    // group terms by their (sorted) denominator indices, first-appearance order
    std::map<std::vector<int>, int> gid;
    std::vector<std::vector<int>> gdens;
    std::vector<std::vector<int>> gterms;
    for (size_t ti = 0; ti < t->terms.size(); ++ti) {
        const auto &ft = t->terms[ti];
        std::vector<int> ds;
        const int nd = static_cast<int>(ft.dens.size()) / drec;
        for (int r = 0; r < nd; ++r) {
            std::vector<int> k(ft.dens.begin() + r * drec, ft.dens.begin() + r * drec + ne);
            k.insert(k.end(), ft.dens.begin() + r * drec + ne + ni, ft.dens.begin() + (r + 1) * drec);
            ds.push_back(den_id.at(k));
        }
        std::sort(ds.begin(), ds.end());
        auto it = gid.find(ds);
        int g;
        if (it == gid.end()) {
            g = static_cast<int>(gdens.size());
            gid.emplace(ds, g);
            gdens.push_back(ds);
            gterms.emplace_back();
        } else {
            g = it->second;
        }
        gterms[g].push_back(static_cast<int>(ti));
    }
    tab.G = static_cast<int>(gdens.size());
    tab.group_start.push_back(0);
    tab.group_den_start.push_back(0);
    for (int g = 0; g < tab.G; ++g) {
        for (int d : gdens[g]) tab.group_den_list.push_back(d);
        tab.group_den_start.push_back(static_cast<int32_t>(tab.group_den_list.size()));
        if (tab.uniform)
            for (int d : gdens[g]) tab.group_dens.push_back(d);
        for (int ti : gterms[g]) {
            const auto &ft = t->terms[ti];
            tab.term_sign.push_back(static_cast<double>(ft.s));
            for (int j = 0; j < ni; ++j) {
                std::vector<int> k(ft.leaves.begin() + j * lrec, ft.leaves.begin() + (j + 1) * lrec);
                tab.term_leaf.push_back(leaf_id.at(k));
            }
        }
        tab.group_start.push_back(static_cast<int32_t>(tab.term_sign.size()));
    }
    tab.T = static_cast<int>(tab.term_sign.size());
    for (int j = 0; j < t->n_g; ++j)
        for (int l = 0; l < nf; ++l) tab.line_alpha.push_back(static_cast<double>(t->alpha[j * nf + l]));
    pack_tables(t);
    (void)nx;
    return AMI_OK;
}

// Packed tables for the specialized kernels: +-1 coefficients as bit masks,
// indices as bytes.  Left empty (packable = false) when the solution falls
// outside that form; the double tables above always exist.
void pack_tables(AmiTerms *t) {
    Tables &tab = t->tab;
    const int ne = t->n_eps, nf = t->n_freq, ni = t->n_int, nx = t->n_ext;
    tab.packable = false;
    tab.p_leaf.clear();
    tab.p_den.clear();
    tab.p_line.clear();
    tab.p_term.clear();
    tab.p_group.clear();
    tab.fermi_used = 0;
    tab.use_products = false;
    if (!tab.uniform) return;
    if (ne > 16 || nf > 16 || ni > 8 || tab.dpt > 8 || nx > 4 || tab.L > 255 || tab.D > 255) return;
    auto masks = [&](const double *c, int n, uint64_t &out) -> bool {
        uint32_t pos = 0, neg = 0;
        for (int i = 0; i < n; ++i) {
            if (c[i] == 1.0) pos |= 1u << i;
            else if (c[i] == -1.0) neg |= 1u << i;
            else if (c[i] != 0.0) return false;
        }
        out = static_cast<uint64_t>(pos) | (static_cast<uint64_t>(neg) << 16);
        return true;
    };
    int n_fermi = 0;
    for (int l = 0; l < tab.L; ++l) {
        uint64_t w = 0;
        if (!masks(&tab.leaf_coef[static_cast<size_t>(l) * ne], ne, w)) return;
        if (tab.leaf_sigma[l] < 0) {
            w |= 1ull << 32;
        } else {
            ++n_fermi;
            tab.fermi_used |= static_cast<uint32_t>((w & 0xffff) | ((w >> 16) & 0xffff));
        }
        tab.p_leaf.push_back(w);
    }
    const int nc = ne + nx;
    for (int r = 0; r < tab.D; ++r) {
        uint64_t w = 0;
        if (!masks(&tab.den_coef[static_cast<size_t>(r) * nc], ne, w)) return;
        for (int x = 0; x < nx; ++x) {
            const double a = tab.den_coef[static_cast<size_t>(r) * nc + ne + x];
            if (a < -127.0 || a > 127.0) return;
            const uint8_t b = static_cast<uint8_t>(static_cast<int8_t>(a));
            w |= static_cast<uint64_t>(b) << (32 + 8 * x);
        }
        tab.p_den.push_back(w);
    }
    for (int j = 0; j < t->n_g; ++j) {
        uint64_t w = 0;
        if (!masks(&tab.line_alpha[static_cast<size_t>(j) * nf], nf, w)) return;
        tab.p_line.push_back(static_cast<uint32_t>(w));
    }
    for (int ti = 0; ti < tab.T; ++ti) {
        uint64_t w = 0;
        for (int j = 0; j < ni; ++j) {
            const int32_t lj = tab.term_leaf[static_cast<size_t>(ti) * ni + j];
            for (int k = 0; k < j; ++k)   // the adjoint updates a term's leaves together
                if (tab.term_leaf[static_cast<size_t>(ti) * ni + k] == lj) return;
            w |= static_cast<uint64_t>(lj) << (8 * j);
        }
        tab.p_term.push_back(w);
    }
    for (int g = 0; g < tab.G; ++g) {
        uint64_t w = 0;
        for (int k = 0; k < tab.dpt; ++k)
            w |= static_cast<uint64_t>(tab.group_dens[static_cast<size_t>(g) * tab.dpt + k]) << (8 * k);
        tab.p_group.push_back(w);
    }
    // products of exp(beta E_i) pay off when Fermi leaves outnumber the energies they use
    tab.use_products = n_fermi > __builtin_popcount(tab.fermi_used);
    tab.packable = true;
}

}  // namespace ami

extern "C" {

AmiStatus amiConstruct(int32_t n_g, int32_t n_eps, int32_t n_freq, int32_t n_int,
                       const int8_t *alpha, const int8_t *eps, const uint8_t *fermionic,
                       uint32_t flags, AmiTerms **out) {
    using namespace ami;
    clear_error();
    if (!out) return fail(AMI_E_ARG, "out is NULL");
    *out = nullptr;
    if (!alpha || !eps) return fail(AMI_E_ARG, "alpha or eps is NULL");
    if (n_g < 1 || n_g > 64) return fail(AMI_E_ARG, "n_g must be in 1..64");
    if (n_eps < 1 || n_eps > kMaxEps) return fail(AMI_E_ARG, "n_eps must be in 1..32");
    if (n_freq < 1 || n_freq > kMaxFreq) return fail(AMI_E_ARG, "n_freq must be in 1..16");
    if (n_int < 0 || n_int > n_freq) return fail(AMI_E_ARG, "n_int must be in 0..n_freq");
    if (flags & ~(AMI_FACTORIZE | AMI_MULTIPOLE)) return fail(AMI_E_ARG, "unknown flag");
    if ((flags & AMI_FACTORIZE) && (flags & AMI_MULTIPOLE))
        return fail(AMI_E_UNSUPPORTED, "the factorized tree is built for simple poles only");
    AmiTerms *t = new (std::nothrow) AmiTerms();
    if (!t) return fail(AMI_E_OOM, "out of host memory");
    t->n_g = n_g;
    t->n_eps = n_eps;
    t->n_freq = n_freq;
    t->n_int = n_int;
    t->n_ext = n_freq - n_int;
    t->flags = flags;
    t->alpha.assign(alpha, alpha + static_cast<size_t>(n_g) * n_freq);
    t->eps.assign(eps, eps + static_cast<size_t>(n_g) * n_eps);
    t->fermionic.assign(n_freq, 1);
    if (fermionic)
        for (int l = 0; l < n_freq; ++l) t->fermionic[l] = fermionic[l] ? 1 : 0;
    for (int8_t v : t->alpha)
        if (v < -1 || v > 1) { delete t; return fail(AMI_E_LABEL, "alpha coefficients must be -1, 0 or 1"); }
    for (int8_t v : t->eps)
        if (v < -1 || v > 1) { delete t; return fail(AMI_E_LABEL, "epsilon coefficients must be -1, 0 or 1"); }
    for (int p = 0; p < n_int; ++p)
        if (!t->fermionic[p]) { delete t; return fail(AMI_E_LABEL, "only fermionic frequencies can be summed"); }
    try {
        construct_flat(t);
        if (flags & AMI_FACTORIZE) construct_tree(t);
        build_tables(t);
    } catch (const BuildError &e) {
        delete t;
        return fail(e.st, e.msg);
    } catch (const std::bad_alloc &) {
        delete t;
        return fail(AMI_E_OOM, "out of host memory during construction");
    }
    *out = t;
    return AMI_OK;
}

AmiStatus amiTermsInfo(const AmiTerms *t, int64_t info[16]) {
    using namespace ami;
    clear_error();
    if (!t || !info) return fail(AMI_E_ARG, "NULL argument");
    for (int i = 0; i < 16; ++i) info[i] = 0;
    info[0] = t->tab.T;
    info[1] = t->n_int;
    info[2] = t->n_eps;
    info[3] = t->n_freq;
    info[4] = t->n_ext;
    info[5] = t->tab.L;
    info[6] = t->tab.D;
    info[7] = t->tab.G;
    info[8] = static_cast<int64_t>(t->tree.size());
    info[9] = t->raw_terms;
    info[10] = t->n_int;
    info[11] = t->n_g - t->n_int;
    info[12] = t->tab.packable ? 1 : 0;
    info[13] = t->tab.use_products ? 1 : 0;
    info[14] = t->n_g;
    info[15] = t->tab.uniform ? 1 : 0;
    return AMI_OK;
}

AmiStatus amiTermsCanonical(const AmiTerms *t, int32_t from_tree, int32_t *buf, int64_t cap, int64_t *len) {
    using namespace ami;
    clear_error();
    if (!t || !len) return fail(AMI_E_ARG, "NULL argument");
    std::vector<int32_t> s;
    try {
        if (from_tree) {
            if (!(t->flags & AMI_FACTORIZE)) return fail(AMI_E_ARG, "handle was built without AMI_FACTORIZE");
            serialize(t, expand_tree(t), s);
        } else {
            serialize(t, t->terms, s);
        }
    } catch (const BuildError &e) {
        return fail(e.st, e.msg);
    }
    *len = static_cast<int64_t>(s.size());
    if (!buf) return AMI_OK;
    if (cap < *len) return fail(AMI_E_ARG, "buffer too small");
    std::memcpy(buf, s.data(), s.size() * sizeof(int32_t));
    return AMI_OK;
}

}  // extern "C"
