// Feynman-graph input (Sec. 2.5): the 4-column graph description (source,
// target, B/F, spin) read from text, momentum-conserving labels assigned to
// every line, and the labels of the fermionic lines handed to the
// construction as R0 (alpha, epsilon = one energy per propagator).
//
// Labelling: the external frequency/momentum enters at the vertex missing an
// incoming fermionic line and leaves at the one missing an outgoing line
// (self-energy legs; with no such vertices, at the two vertices missing a
// bosonic line, first in edge order entering).  A spanning tree is grown from
// the bosonic lines first, then the fermionic ones, in file order; every
// fermionic line outside it carries one summed frequency (slots in file
// order), flowing source -> target on that line and back through the tree;
// the external one flows along the tree path between the external vertices.
// So every summed frequency sits on a fermionic line (the sums of Eq. (3) are
// fermionic) whenever the bosonic lines hold no cycle.  Each line's label is
// the signed sum of the frequencies crossing it (Eq. (2)).
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "ami_internal.hpp"

namespace ami {

namespace {

struct Dsu {
    std::vector<int> p;
    explicit Dsu(int n) : p(n) {
        for (int i = 0; i < n; ++i) p[i] = i;
    }
    int find(int x) {
        while (p[x] != x) x = p[x] = p[p[x]];
        return x;
    }
    bool unite(int a, int b) {
        a = find(a);
        b = find(b);
        if (a == b) return false;
        p[a] = b;
        return true;
    }
};

// edges crossed from u to v through the tree, with +1 when an edge is
// traversed source -> target
bool tree_path(const std::vector<std::vector<std::pair<int, int>>> &adj, const std::vector<int> &src,
               int u, int v, std::vector<std::pair<int, int>> &path) {
    const int n = static_cast<int>(adj.size());
    std::vector<int> prev_v(n, -1), prev_e(n, -1);
    std::vector<int> stack{u};
    std::vector<char> seen(n, 0);
    seen[u] = 1;
    while (!stack.empty()) {
        const int x = stack.back();
        stack.pop_back();
        if (x == v) break;
        for (const auto &ye : adj[x]) {
            if (seen[ye.first]) continue;
            seen[ye.first] = 1;
            prev_v[ye.first] = x;
            prev_e[ye.first] = ye.second;
            stack.push_back(ye.first);
        }
    }
    if (!seen[v]) return false;
    path.clear();
    for (int x = v; x != u; x = prev_v[x]) {
        const int e = prev_e[x];
        path.emplace_back(e, src[e] == prev_v[x] ? +1 : -1);
    }
    return true;
}

}  // namespace

}  // namespace ami

extern "C" {

AmiStatus amiReadGraph(const char *path, int32_t *edges, int32_t cap, int32_t *n_edges, int32_t *n_vertices) {
    using namespace ami;
    clear_error();
    if (!path || !n_edges || !n_vertices) return fail(AMI_E_ARG, "NULL argument");
    std::ifstream f(path);
    if (!f) return fail(AMI_E_ARG, std::string("cannot open ") + path);
    std::vector<int32_t> rows;
    std::string line;
    int nv = 0, lineno = 0;
    while (std::getline(f, line)) {
        ++lineno;
        const size_t hash = line.find('#');
        if (hash != std::string::npos) line.resize(hash);
        std::istringstream is(line);
        long long v[4];
        int got = 0;
        while (got < 4 && (is >> v[got])) ++got;
        std::string rest;
        if (got == 0 && !(is.clear(), is >> rest)) continue;   // blank or comment line
        if (got != 4 || (is >> rest))
            return fail(AMI_E_ARG, "line " + std::to_string(lineno) + ": expected 4 integers");
        if (v[0] < 0 || v[1] < 0 || v[0] > 4095 || v[1] > 4095 || (v[2] != 0 && v[2] != 1) || v[3] < INT32_MIN ||
            v[3] > INT32_MAX)
            return fail(AMI_E_ARG, "line " + std::to_string(lineno) + ": bad vertex, B/F or spin value");
        for (int j = 0; j < 4; ++j) rows.push_back(static_cast<int32_t>(v[j]));
        nv = std::max<int>(nv, static_cast<int>(std::max(v[0], v[1])) + 1);
    }
    *n_edges = static_cast<int32_t>(rows.size() / 4);
    *n_vertices = nv;
    if (!edges) return AMI_OK;
    if (cap < *n_edges) return fail(AMI_E_ARG, "edge buffer too small");
    if (!rows.empty()) std::memcpy(edges, rows.data(), rows.size() * sizeof(int32_t));   // an empty file has no rows
    return AMI_OK;
}

AmiStatus amiConstructGraph(int32_t n_vertices, int32_t n_edges, const int32_t *edges, uint32_t flags,
                            AmiTerms **out) {
    using namespace ami;
    clear_error();
    if (!out) return fail(AMI_E_ARG, "out is NULL");
    *out = nullptr;
    if (!edges || n_vertices < 2 || n_vertices > 4096 || n_edges < 1 || n_edges > 4096)
        return fail(AMI_E_ARG, "need 2..4096 vertices and 1..4096 edges");
    std::vector<int> src(n_edges), dst(n_edges), bf(n_edges);
    std::vector<int> in_f(n_vertices, 0), out_f(n_vertices, 0), deg_b(n_vertices, 0);
    for (int e = 0; e < n_edges; ++e) {
        src[e] = edges[4 * e];
        dst[e] = edges[4 * e + 1];
        bf[e] = edges[4 * e + 2];
        if (src[e] < 0 || src[e] >= n_vertices || dst[e] < 0 || dst[e] >= n_vertices || (bf[e] != 0 && bf[e] != 1))
            return fail(AMI_E_ARG, "edge " + std::to_string(e) + ": vertex out of range or B/F not 0/1");
        if (bf[e]) {
            ++out_f[src[e]];
            ++in_f[dst[e]];
        } else {
            ++deg_b[src[e]];
            ++deg_b[dst[e]];
        }
    }
    // external vertices
    int ext_in = -1, ext_out = -1;
    bool ext_fermionic = true;
    for (int v = 0; v < n_vertices; ++v) {
        if (in_f[v] > 1 || out_f[v] > 1)
            return fail(AMI_E_LABEL, "vertex " + std::to_string(v) + " has more than one fermionic line in or out");
        if (in_f[v] == 0) {
            if (ext_in >= 0) return fail(AMI_E_LABEL, "more than one vertex without an incoming fermionic line");
            ext_in = v;
        }
        if (out_f[v] == 0) {
            if (ext_out >= 0) return fail(AMI_E_LABEL, "more than one vertex without an outgoing fermionic line");
            ext_out = v;
        }
    }
    if ((ext_in < 0) != (ext_out < 0)) return fail(AMI_E_LABEL, "unbalanced fermionic lines");
    if (ext_in < 0) {
        ext_fermionic = false;
        for (int v = 0; v < n_vertices; ++v)
            if (deg_b[v] == 0) {
                if (ext_in < 0) ext_in = v;
                else if (ext_out < 0) ext_out = v;
                else return fail(AMI_E_LABEL, "more than two vertices without a bosonic line");
            }
        if (ext_out < 0) return fail(AMI_E_LABEL, "no external legs (vacuum graphs are not supported)");
    }
    // spanning tree: bosonic lines first, then fermionic, in file order
    Dsu dsu(n_vertices);
    std::vector<char> in_tree(n_edges, 0);
    for (int pass = 0; pass < 2; ++pass)
        for (int e = 0; e < n_edges; ++e)
            if (bf[e] == pass && dsu.unite(src[e], dst[e])) in_tree[e] = 1;
    for (int v = 1; v < n_vertices; ++v)
        if (dsu.find(v) != dsu.find(0)) return fail(AMI_E_LABEL, "the graph is not connected");
    std::vector<int> loops;
    for (int e = 0; e < n_edges; ++e)
        if (!in_tree[e]) loops.push_back(e);
    const int n_int = static_cast<int>(loops.size());
    const int n_freq = n_int + 1;
    if (n_freq > kMaxFreq) return fail(AMI_E_UNSUPPORTED, "more than 15 independent loops");
    std::vector<std::vector<std::pair<int, int>>> adj(n_vertices);
    for (int e = 0; e < n_edges; ++e)
        if (in_tree[e]) {
            adj[src[e]].emplace_back(dst[e], e);
            adj[dst[e]].emplace_back(src[e], e);
        }
    std::vector<std::vector<int>> lab(n_edges, std::vector<int>(n_freq, 0));
    std::vector<std::pair<int, int>> path;
    for (int s = 0; s < n_int; ++s) {
        const int e = loops[s];
        lab[e][s] = 1;
        if (!tree_path(adj, src, dst[e], src[e], path)) return fail(AMI_E_LABEL, "no tree path");
        for (const auto &pe : path) lab[pe.first][s] += pe.second;
    }
    if (!tree_path(adj, src, ext_in, ext_out, path)) return fail(AMI_E_LABEL, "no tree path");
    for (const auto &pe : path) lab[pe.first][n_int] += pe.second;
    // R0: the fermionic lines in file order, one energy each
    std::vector<int> g_lines;
    for (int e = 0; e < n_edges; ++e)
        if (bf[e]) g_lines.push_back(e);
    const int n_g = static_cast<int>(g_lines.size());
    if (n_g < 1) return fail(AMI_E_LABEL, "no fermionic lines");
    if (n_g > kMaxEps) return fail(AMI_E_UNSUPPORTED, "more than 32 propagators");
    std::vector<int8_t> alpha(static_cast<size_t>(n_g) * n_freq), eps(static_cast<size_t>(n_g) * n_g, 0);
    for (int j = 0; j < n_g; ++j) {
        for (int s = 0; s < n_freq; ++s) {
            const int c = lab[g_lines[j]][s];
            if (c < -1 || c > 1) return fail(AMI_E_LABEL, "a label coefficient beyond +-1");
            alpha[static_cast<size_t>(j) * n_freq + s] = static_cast<int8_t>(c);
        }
        eps[static_cast<size_t>(j) * n_g + j] = 1;
    }
    std::vector<uint8_t> fermionic(n_freq, 1);
    for (int s = 0; s < n_int; ++s) fermionic[s] = static_cast<uint8_t>(bf[loops[s]]);
    fermionic[n_int] = ext_fermionic ? 1 : 0;
    return amiConstruct(n_g, n_g, n_freq, n_int, alpha.data(), eps.data(), fermionic.data(), flags, out);
}

AmiStatus amiTermsLabels(const AmiTerms *t, int8_t *alpha, int8_t *eps, uint8_t *fermionic) {
    using namespace ami;
    clear_error();
    if (!t) return fail(AMI_E_ARG, "terms is NULL");
    if (alpha) std::memcpy(alpha, t->alpha.data(), t->alpha.size());
    if (eps) std::memcpy(eps, t->eps.data(), t->eps.size());
    if (fermionic) std::memcpy(fermionic, t->fermionic.data(), t->fermionic.size());
    return AMI_OK;
}

}  // extern "C"
