// Compilation, caching and loading of the run-time specialized evaluator.
//
// The generated source (codegen.cpp) and the embedded device headers
// (device_common.hpp, kargs.hpp, jit_tiles.hpp, jit_kernel.hpp, built into the library as
// strings) are compiled for gfx950 with hipRTC under the flags the library
// itself is built with.  Code objects are kept per handle and on disk, keyed
// by a hash of everything that goes into the compilation, so a diagram is
// compiled once per machine; the source is stored beside each code object and
// compared on every hit.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iterator>
#include <mutex>
#include <string>
#include <vector>

#include "jit.hpp"
#include "runtime.hpp"

#include "jit_headers.inc"   // kJitHeaderCount, kJitHeaderNames[], kJitHeaderTexts[] (generated at build)

namespace ami {

namespace {

const char *const kOptions[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                                // keep the compiler away from packed FP32 instructions
                                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
constexpr int kNumOptions = static_cast<int>(sizeof(kOptions) / sizeof(kOptions[0]));

uint64_t fnv1a(const std::string &s, uint64_t h) {
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string cache_key(const std::string &src) {
    int major = 0, minor = 0;
    (void)hiprtcVersion(&major, &minor);
    std::string all = "amigpu-jit-1|" + std::to_string(major) + "." + std::to_string(minor) + "|";
    for (int i = 0; i < kNumOptions; ++i) all += std::string(kOptions[i]) + "|";
    for (int i = 0; i < kJitHeaderCount; ++i) all += std::string(kJitHeaderNames[i]) + "|" + kJitHeaderTexts[i] + "|";
    all += src;
    char b[40];
    std::snprintf(b, sizeof(b), "%016llx%016llx", static_cast<unsigned long long>(fnv1a(all, 1469598103934665603ull)),
                  static_cast<unsigned long long>(fnv1a(all, 0x9e3779b97f4a7c15ull)));
    return b;
}

bool make_dirs(const std::string &path) {
    std::string cur;
    for (size_t i = 0; i <= path.size(); ++i) {
        if (i == path.size() || path[i] == '/') {
            if (!cur.empty() && ::mkdir(cur.c_str(), 0755) != 0 && errno != EEXIST) return false;
        }
        if (i < path.size()) cur += path[i];
    }
    return true;
}

// AMIGPU_CACHE_DIR, else $HOME/.cache/amigpu/jit; empty (no disk cache) when
// neither can be created
std::string cache_dir() {
    std::string d;
    if (const char *e = std::getenv("AMIGPU_CACHE_DIR")) {
        d = e;
    } else if (const char *h = std::getenv("HOME")) {
        d = std::string(h) + "/.cache/amigpu/jit";
    }
    if (d.empty() || !make_dirs(d)) return std::string();
    return d;
}

bool read_file(const std::string &path, std::vector<char> &out) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    out.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
    return static_cast<bool>(f) || f.eof();
}

void write_file_atomic(const std::string &path, const char *data, size_t n) {
    const std::string tmp = path + ".tmp" + std::to_string(::getpid());
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return;
        f.write(data, static_cast<std::streamsize>(n));
        if (!f) {
            std::remove(tmp.c_str());
            return;
        }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

AmiStatus compile(const std::string &src, std::vector<char> &code, std::string &err) {
    hiprtcProgram prog;
    hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "ami_jit.hip", kJitHeaderCount, kJitHeaderTexts,
                                         kJitHeaderNames);
    if (r != HIPRTC_SUCCESS) {
        err = std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
        return AMI_E_HIP;
    }
    r = hiprtcCompileProgram(prog, kNumOptions, kOptions);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        std::string log;
        if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 0) {
            log.resize(n);
            (void)hiprtcGetProgramLog(prog, &log[0]);
        }
        if (log.size() > 4000) log.resize(4000);
        err = std::string("specialized kernel compilation failed: ") + hiprtcGetErrorString(r) + "\n" + log;
        (void)hiprtcDestroyProgram(&prog);
        return AMI_E_HIP;
    }
    size_t n = 0;
    r = hiprtcGetCodeSize(prog, &n);
    if (r == HIPRTC_SUCCESS) {
        code.resize(n);
        r = hiprtcGetCode(prog, code.data());
    }
    (void)hiprtcDestroyProgram(&prog);
    if (r != HIPRTC_SUCCESS || code.empty()) {
        err = std::string("hiprtcGetCode: ") + hiprtcGetErrorString(r);
        code.clear();
        return AMI_E_HIP;
    }
    return AMI_OK;
}

// Code object for (t, kind): from the handle, the disk cache, or a compilation.
static_assert(sizeof(AmiTerms::jit_code) / sizeof(AmiTerms::jit_code[0]) == 2 * kJitKinds,
              "one code object per input and kind");

// Whether the second of two compiled forms of one kernel is the better one:
// no more private (spill) memory, and at least the waves per SIMD its VGPRs
// allow; unreadable metadata keeps the first.
bool prefer_second(const std::vector<char> &a, const std::vector<char> &b) {
    const int64_t va = code_meta(a, ".vgpr_count"), vb = code_meta(b, ".vgpr_count");
    const int64_t pa = code_meta(a, ".private_segment_fixed_size"), pb = code_meta(b, ".private_segment_fixed_size");
    if (va <= 0 || vb <= 0 || pa < 0 || pb < 0) return false;
    auto waves = [](int64_t v) { return std::min<int64_t>(8, 512 / ((v + 7) / 8 * 8)); };
    return pb <= pa && waves(vb) >= waves(va);
}

AmiStatus code_object(AmiTerms *t, bool hub, int kind) {
    const int slot = kJitKinds * (hub ? 1 : 0) + kind;
    std::vector<char> &code = t->jit_code[slot];
    if (!code.empty()) return AMI_OK;
    std::string &err = t->jit_error[slot];
    if (!err.empty()) return fail(AMI_E_UNSUPPORTED, err);
    std::string why;
    const bool passes = kind == kJitSumsPass || kind == kJitFreqPass || kind == kJitAdjFreq || kind == kJitAdjLeaf ||
                        kind == kJitComplexSums || kind == kJitComplexFreq || kind == kJitComplexAdjFreq ||
                        kind == kJitComplexAdjLeaf;
    if (!jit_supported(t, hub, &why, passes)) {
        err = "no specialized kernel: " + why;
        return fail(AMI_E_UNSUPPORTED, err);
    }
    if (jit_kind_complex(kind))
        for (int o : t->tab.leaf_order)
            if (o > 0) {
                err = "no complex-energy kernel for Taylor-coefficient leaves (poles of higher order)";
                return fail(AMI_E_UNSUPPORTED, err);
            }
    if ((kind == kJitAdjoint || kind == kJitComplexAdj) && jit_nested_override() < 0) {
        // the one-pass adjoints in both forms of their leaf-cotangent sweep; the
        // nested one is kept where it spills no more and keeps the occupancy
        // (order 4, 52 terms: 63.5 -> 61.0 us per 10^6-sample step; where its
        // node values push the kernel over a register boundary it loses)
        std::vector<char> nested;
        AmiStatus st = code_from_source(jit_source(t, hub, 1 << kind, 0), code, err);
        if (st != AMI_OK) return fail(st, err);
        st = code_from_source(jit_source(t, hub, 1 << kind, kJitNestedPartTerms), nested, err);
        if (st != AMI_OK) return fail(st, err);
        if (prefer_second(code, nested)) code.swap(nested);
        return AMI_OK;
    }
    const AmiStatus st = code_from_source(jit_source(t, hub, 1 << kind), code, err);
    return st == AMI_OK ? AMI_OK : fail(st, err);
}

}  // namespace

// An unsigned value of a code object's kernel metadata built here (the
// AMDGPU msgpack note of its one kernel): the integer after the fixstr key,
// or -1.
int64_t code_meta(const std::vector<char> &code, const char *key) {
    const size_t n = std::strlen(key);
    if (n == 0 || n > 31) return -1;
    std::string pat(1, static_cast<char>(0xa0 | n));
    pat += key;
    const std::string bytes(code.begin(), code.end());
    const size_t at = bytes.find(pat);
    if (at == std::string::npos) return -1;
    size_t i = at + pat.size();
    auto byte = [&](size_t j) -> int64_t {
        return j < bytes.size() ? static_cast<unsigned char>(bytes[j]) : -1;
    };
    const int64_t tag = byte(i);
    if (tag < 0) return -1;
    if (tag <= 0x7f) return tag;                                        // positive fixint
    int len = tag == 0xcc ? 1 : tag == 0xcd ? 2 : tag == 0xce ? 4 : 0;  // uint8/16/32
    if (len == 0) return -1;
    int64_t v = 0;
    for (int k = 1; k <= len; ++k) {
        const int64_t b = byte(i + k);
        if (b < 0) return -1;
        v = (v << 8) | b;
    }
    return v;
}

AmiStatus code_from_source(const std::string &src, std::vector<char> &code, std::string &err) {
    const std::string dir = cache_dir();
    const std::string base = dir.empty() ? std::string() : dir + "/" + cache_key(src);
    if (!base.empty()) {
        std::vector<char> stored_src;
        if (read_file(base + ".hip", stored_src) && std::string(stored_src.begin(), stored_src.end()) == src &&
            read_file(base + ".hsaco", code) && !code.empty())
            return AMI_OK;
        code.clear();
    }
    const AmiStatus st = compile(src, code, err);
    if (st != AMI_OK) return st;
    if (!base.empty()) {
        write_file_atomic(base + ".hsaco", code.data(), code.size());
        write_file_atomic(base + ".hip", src.data(), src.size());
    }
    return AMI_OK;
}

AmiStatus jit_compile(AmiTerms *t, bool hub, int kind) {
    if (kind < kJitForward || kind >= kJitKinds || (kind == kJitMonteCarlo && !hub) ||
        (jit_kind_complex(kind) && hub))
        return fail(AMI_E_ARG, "no such specialized kernel");
    std::lock_guard<std::mutex> lock(t->jit_mu);
    return code_object(t, hub, kind);
}

AmiStatus jit_get(AmiTerms *t, bool hub, int kind, void **fn) {
    if (kind < kJitForward || kind >= kJitKinds || (kind == kJitMonteCarlo && !hub) ||
        (jit_kind_complex(kind) && hub))
        return fail(AMI_E_ARG, "no such specialized kernel");
    std::lock_guard<std::mutex> lock(t->jit_mu);
    const int slot = kJitKinds * (hub ? 1 : 0) + kind;
    // the compilation needs no device: do it first
    AmiStatus st = code_object(t, hub, kind);
    if (st != AMI_OK) return st;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    for (const auto &m : t->jit_mods)
        if (m.device == dev && m.kind == slot) {
            *fn = m.fn;
            return AMI_OK;
        }
    hipModule_t mod = nullptr;
    e = hipModuleLoadData(&mod, t->jit_code[slot].data());
    if (e != hipSuccess) return hip_fail(e, "hipModuleLoadData (specialized kernel)");
    hipFunction_t f = nullptr;
    static const char *const kNames[kJitKinds] = {"ami_jit_fwd",  "ami_jit_adj",   "ami_jit_mc",   "ami_jit_cfwd",
                                                  "ami_jit_sums", "ami_jit_freq",  "ami_jit_adjf", "ami_jit_adjl",
                                                  "ami_jit_cadj", "ami_jit_csums", "ami_jit_cfreq", "ami_jit_cadjf",
                                                  "ami_jit_cadjl"};
    e = hipModuleGetFunction(&f, mod, kNames[kind]);
    if (e != hipSuccess) {
        (void)hipModuleUnload(mod);
        return hip_fail(e, "hipModuleGetFunction (specialized kernel)");
    }
    AmiTerms::JitModule m;
    m.device = dev;
    m.kind = slot;
    m.module = mod;
    m.fn = reinterpret_cast<void *>(f);
    t->jit_mods.push_back(m);
    *fn = m.fn;
    return AMI_OK;
}

AmiStatus jit_loaded(AmiTerms *t, bool hub, int kind, void **fn) {
    if (kind < kJitForward || kind >= kJitKinds || (kind == kJitMonteCarlo && !hub) ||
        (jit_kind_complex(kind) && hub))
        return fail(AMI_E_ARG, "no such specialized kernel");
    std::lock_guard<std::mutex> lock(t->jit_mu);
    const int slot = kJitKinds * (hub ? 1 : 0) + kind;
    if (!t->jit_error[slot].empty()) return fail(AMI_E_UNSUPPORTED, t->jit_error[slot]);
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    for (const auto &m : t->jit_mods)
        if (m.device == dev && m.kind == slot) {
            *fn = m.fn;
            return AMI_OK;
        }
    return fail(AMI_E_ARG, "the specialized kernel is not loaded on this device: call amiTermsSpecialize first");
}

void jit_release(AmiTerms *t) {
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (auto &m : t->jit_mods)
        if (m.module && hipSetDevice(m.device) == hipSuccess) (void)hipModuleUnload(static_cast<hipModule_t>(m.module));
    t->jit_mods.clear();
    if (have_cur) (void)hipSetDevice(cur);
}

}  // namespace ami
