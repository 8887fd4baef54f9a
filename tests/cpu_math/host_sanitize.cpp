// Host driver of the library's host code under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by the CPU tests with g++, from
// construct.cpp, graph.cpp, codegen.cpp and abi.cpp): construction in every
// mode, term information, the canonical streams (flat and expanded tree),
// labels, the generated sources of every kernel set and of a persistent batch
// module, and the graph reader on every file named on the command line (well
// formed or not).  The GPU side is absent: amiFree releases the host handle
// only, and code_from_source (run-time compilation) is refused.
//
// stdin: a count, then per diagram "n_g n_eps n_freq n_int" and the alpha and
// eps entries row-major.  argv[1..]: graph files.  Exit status 0 when every
// call returned a status (sanitizer reports abort the process).
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/amigpu.h"
#include "../../paper_2311_17189_amd/csrc/ami_internal.hpp"
#include "../../paper_2311_17189_amd/csrc/jit.hpp"

namespace ami {
AmiStatus code_from_source(const std::string &, std::vector<char> &, std::string &err) {
    err = "no run-time compiler in the host check";
    return AMI_E_UNSUPPORTED;
}
}  // namespace ami

extern "C" void amiFree(AmiTerms *t) { delete t; }

namespace {

int exercise(AmiTerms *t, std::vector<AmiTerms *> &keep) {
    int64_t info[16];
    if (amiTermsInfo(t, info) != AMI_OK) return 1;
    for (int tree = 0; tree <= 1; ++tree) {
        int64_t len = 0;
        const AmiStatus st = amiTermsCanonical(t, tree, nullptr, 0, &len);
        if (st != AMI_OK) continue;                  // no tree without AMI_FACTORIZE
        std::vector<int32_t> buf(static_cast<size_t>(len));
        if (amiTermsCanonical(t, tree, buf.data(), len, &len) != AMI_OK) return 1;
        // a buffer one short is refused, not overrun
        if (len > 0 && amiTermsCanonical(t, tree, buf.data(), len - 1, &len) == AMI_OK) return 1;
    }
    std::vector<int8_t> a(static_cast<size_t>(info[14] * info[3])), e(static_cast<size_t>(info[14] * info[2]));
    std::vector<uint8_t> f(static_cast<size_t>(info[3]));
    if (amiTermsLabels(t, a.data(), e.data(), f.data()) != AMI_OK) return 1;
    for (int sel = 0; sel < 4; ++sel) {
        int64_t len = 0;
        if (amiTermsSource(t, sel, nullptr, 0, &len) != AMI_OK) continue;    // outside the specialized form
        std::vector<char> src(static_cast<size_t>(len));
        if (amiTermsSource(t, sel, src.data(), len, &len) != AMI_OK) return 1;
        if (std::strlen(src.data()) + 1 != static_cast<size_t>(len)) return 1;
    }
    keep.push_back(t);
    return 0;
}

}  // namespace

int main(int argc, char **argv) {
    int n = 0;
    if (std::scanf("%d", &n) != 1) return 2;
    std::vector<AmiTerms *> keep;
    int bad = 0;
    for (int d = 0; d < n; ++d) {
        int ng, ne, nf, ni;
        if (std::scanf("%d %d %d %d", &ng, &ne, &nf, &ni) != 4) return 2;
        std::vector<int8_t> alpha(static_cast<size_t>(ng) * nf), eps(static_cast<size_t>(ng) * ne);
        for (auto &x : alpha) {
            int v;
            if (std::scanf("%d", &v) != 1) return 2;
            x = static_cast<int8_t>(v);
        }
        for (auto &x : eps) {
            int v;
            if (std::scanf("%d", &v) != 1) return 2;
            x = static_cast<int8_t>(v);
        }
        for (uint32_t flags : {0u, static_cast<unsigned>(AMI_FACTORIZE), static_cast<unsigned>(AMI_MULTIPOLE)}) {
            AmiTerms *t = nullptr;
            const AmiStatus st = amiConstruct(ng, ne, nf, ni, alpha.data(), eps.data(), nullptr, flags, &t);
            if (st == AMI_OK) bad += exercise(t, keep);
            else if (t) bad += 1;                    // a failure hands out no handle
        }
        // labels outside {-1, 0, 1} are refused
        std::vector<int8_t> wrong = alpha;
        wrong[0] = 2;
        AmiTerms *t = nullptr;
        if (amiConstruct(ng, ne, nf, ni, wrong.data(), eps.data(), nullptr, 0, &t) == AMI_OK) bad += 1;
    }
    if (keep.size() >= 2) {                          // a persistent batch module of the first few
        std::vector<AmiTerms *> items(keep.begin(), keep.begin() + std::min<size_t>(4, keep.size()));
        std::vector<int64_t> n_f(items.size(), 16);
        n_f[0] = 1;
        int64_t len = 0;
        if (amiBatchSource(items.data(), static_cast<int32_t>(items.size()), n_f.data(), 1, 0, nullptr, 0, &len) ==
            AMI_OK) {
            std::vector<char> src(static_cast<size_t>(len));
            if (amiBatchSource(items.data(), static_cast<int32_t>(items.size()), n_f.data(), 1, 0, src.data(), len,
                               &len) != AMI_OK)
                bad += 1;
        }
    }
    for (int k = 1; k < argc; ++k) {
        int32_t ne = 0, nv = 0;
        if (amiReadGraph(argv[k], nullptr, 0, &ne, &nv) != AMI_OK) continue;   // malformed: refused
        std::vector<int32_t> edges(static_cast<size_t>(ne) * 4 + 4);
        if (amiReadGraph(argv[k], edges.data(), ne, &ne, &nv) != AMI_OK) {
            bad += 1;
            continue;
        }
        if (ne > 0 && amiReadGraph(argv[k], edges.data(), ne - 1, &ne, &nv) == AMI_OK) bad += 1;   // too small
        AmiTerms *t = nullptr;
        if (amiConstructGraph(nv, ne, edges.data(), 0, &t) == AMI_OK) bad += exercise(t, keep);
    }
    for (AmiTerms *t : keep) amiFree(t);
    std::printf("checked %zu handles, %d failures\n", keep.size(), bad);
    return bad == 0 ? 0 : 1;
}
