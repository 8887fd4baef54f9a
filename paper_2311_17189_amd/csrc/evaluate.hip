// Runtime side of the evaluators: table upload, launch shapes, kernel
// dispatch, deterministic reductions, and the evaluate entry points of the C
// ABI (include/amigpu.h).
//
// The evaluation (Burke & LeBlanc, arXiv 2311.17189, Sec. 2.3) maps one lane
// to one energy sample; the kernels are in kernels_packed.hpp (bit-mask tables,
// specialized per self-energy shape, forward and adjoint) and kernel_generic.hpp
// (double tables, forward only, any coefficients).  Sums over samples (the
// Monte-Carlo row sums of Sec. 2.3 and the reductions of the adjoint) are done
// per block with a fixed shuffle tree and then across blocks in a fixed order,
// so repeated calls are bitwise identical.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ami_internal.hpp"
#include "device_common.hpp"
#include "kernel_generic.hpp"
#include "jit.hpp"
#include "kernels_packed.hpp"
#include "runtime.hpp"

namespace ami {

AmiStatus hip_fail(hipError_t e, const char *what) {
    return fail(AMI_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

// out[j] = sum over rows of column j.  One block per column.
__global__ __launch_bounds__(kRedThreads) void ami_colsum_kernel(const double *partial, int64_t rows, int64_t rs,
                                                                 int64_t cs, double *out) {
    __shared__ double sh[kRedThreads / 64];
    const double r = column_sum(partial + blockIdx.x * cs, rows, rs, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// Same reduction for the adjoint partials, routing each column to its output:
// column 0 dL/dbeta, 1 dL/dmu, 2 dL/dt, 4.. dL/dw (complex [n_f][n_ext]).
// Blocks past the gradient columns reduce the forward values' row sums
// (partial sums of nval columns stored after the ncols gradient ones, in the
// same layout: column-major when colmajor, else row-major).
__global__ __launch_bounds__(kRedThreads) void ami_adj_finalize_kernel(const double *partial, int64_t rows, int ncols,
                                                                       int colmajor, double *gbeta, double *gmu,
                                                                       double *gt, double *gw, int nval,
                                                                       double *vsum) {
    __shared__ double sh[kRedThreads / 64];
    int j = blockIdx.x;
    double *dst = nullptr;
    const double *src = partial;
    int64_t width = ncols;
    if (j == 0) dst = gbeta;
    else if (j == 1) dst = gmu;
    else if (j == 2) dst = gt;
    else if (j >= kAdjScalars && j < ncols && gw) dst = gw + (j - kAdjScalars);
    else if (j >= ncols && vsum) {
        j -= ncols;
        dst = vsum + j;
        src = partial + rows * ncols;
        width = nval;
    }
    if (!dst) return;
    const double r = colmajor ? column_sum(src + j * rows, rows, 1, sh) : column_sum(src + j, rows, width, sh);
    if (threadIdx.x == 0) *dst = r;
}

__global__ void ami_fill_kernel(double *p, int64_t n, double v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

}  // namespace

AmiStatus fill(double *p, int64_t n, hipStream_t stream) {
    if (!p || n <= 0) return AMI_OK;
    hipLaunchKernelGGL(ami_fill_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, p, n,
                       0.0);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? AMI_OK : hip_fail(e, "fill launch");
}

// Upload (once per device) every table of a handle in one allocation.
AmiStatus upload(AmiTerms *t, DeviceTables **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(t->dev_mu);
    for (auto &d : t->dev)
        if (d.device == dev) {
            *out = &d;
            return AMI_OK;
        }
    const Tables &tb = t->tab;
    struct Piece {
        const void *src;
        size_t bytes;
        size_t off;
    };
    Piece pieces[13] = {
        {tb.leaf_coef.data(), tb.leaf_coef.size() * sizeof(double), 0},
        {tb.leaf_sigma.data(), tb.leaf_sigma.size() * sizeof(double), 0},
        {tb.den_coef.data(), tb.den_coef.size() * sizeof(double), 0},
        {tb.group_dens.data(), tb.group_dens.size() * sizeof(int32_t), 0},
        {tb.group_start.data(), tb.group_start.size() * sizeof(int32_t), 0},
        {tb.term_sign.data(), tb.term_sign.size() * sizeof(double), 0},
        {tb.term_leaf.data(), tb.term_leaf.size() * sizeof(int32_t), 0},
        {tb.line_alpha.data(), tb.line_alpha.size() * sizeof(double), 0},
        {tb.p_leaf.data(), tb.p_leaf.size() * sizeof(uint64_t), 0},
        {tb.p_den.data(), tb.p_den.size() * sizeof(uint64_t), 0},
        {tb.p_line.data(), tb.p_line.size() * sizeof(uint32_t), 0},
        {tb.p_term.data(), tb.p_term.size() * sizeof(uint64_t), 0},
        {tb.p_group.data(), tb.p_group.size() * sizeof(uint64_t), 0},
    };
    size_t total = 0;
    for (auto &pc : pieces) {
        pc.off = total;
        total += align256(std::max<size_t>(pc.bytes, 8));
    }
    std::vector<unsigned char> host(total, 0);
    for (auto &pc : pieces)
        if (pc.bytes) std::memcpy(host.data() + pc.off, pc.src, pc.bytes);
    void *blob = nullptr;
    e = hipMalloc(&blob, total);
    if (e != hipSuccess) return fail(AMI_E_OOM, std::string("hipMalloc of tables: ") + hipGetErrorString(e));
    e = hipMemcpy(blob, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(blob);
        return hip_fail(e, "hipMemcpy of tables");
    }
    DeviceTables d;
    d.device = dev;
    d.blob = blob;
    auto at = [&](int i) { return static_cast<unsigned char *>(blob) + pieces[i].off; };
    d.leaf_coef = reinterpret_cast<const double *>(at(0));
    d.leaf_sigma = reinterpret_cast<const double *>(at(1));
    d.den_coef = reinterpret_cast<const double *>(at(2));
    d.group_dens = reinterpret_cast<const int32_t *>(at(3));
    d.group_start = reinterpret_cast<const int32_t *>(at(4));
    d.term_sign = reinterpret_cast<const double *>(at(5));
    d.term_leaf = reinterpret_cast<const int32_t *>(at(6));
    d.line_alpha = reinterpret_cast<const double *>(at(7));
    d.p_leaf = reinterpret_cast<const uint64_t *>(at(8));
    d.p_den = reinterpret_cast<const uint64_t *>(at(9));
    d.p_line = reinterpret_cast<const uint32_t *>(at(10));
    d.p_term = reinterpret_cast<const uint64_t *>(at(11));
    d.p_group = reinterpret_cast<const uint64_t *>(at(12));
    t->dev.push_back(d);
    *out = &t->dev.back();
    return AMI_OK;
}

AmiStatus pick_shape(int slots, LaunchShape &ls) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    ls.slots = slots;
    const size_t per_lane = static_cast<size_t>(slots) * sizeof(double);
    // 256 lanes while a block stays within a quarter of the CU's LDS, else fewer
    const int blocks[3] = {256, 128, 64};
    for (int b : blocks) {
        const size_t lds = per_lane * b + 2 * sizeof(double) * (b / 64);
        if (lds <= static_cast<size_t>(max_lds) && (lds <= 40 * 1024 || b == 64)) {
            ls.block = b;
            ls.lds = lds;
            return AMI_OK;
        }
    }
    return fail(AMI_E_UNSUPPORTED, "solution too large for the LDS-resident evaluator (" +
                                       std::to_string(per_lane) + " B per sample)");
}

PackedTabs packed_tabs(const AmiTerms *t, const DeviceTables *dt) {
    const Tables &tb = t->tab;
    PackedTabs p;
    p.leaf = dt->p_leaf;
    p.den = dt->p_den;
    p.line = dt->p_line;
    p.term = dt->p_term;
    p.term_sign = dt->term_sign;
    p.group_start = dt->group_start;
    p.group = dt->p_group;
    p.L = tb.L;
    p.D = tb.D;
    p.G = tb.G;
    p.T = tb.T;
    p.n_eps = t->n_eps;
    p.n_int = t->n_int;
    p.n_ext = t->n_ext;
    p.n_freq = t->n_freq;
    p.n_g = t->n_g;
    p.dpt = tb.dpt;
    p.fermi_used = tb.fermi_used;
    p.use_products = tb.use_products ? 1 : 0;
    return p;
}

namespace {

template <bool ADJ, int NE, int NI, int DPT, bool EXACT, bool HUB>
void launch_packed_one(dim3 grid, dim3 block, size_t lds, hipStream_t stream, const KArgs &a) {
    if constexpr (ADJ)
        hipLaunchKernelGGL((ami_adj_packed<NE, NI, DPT, EXACT, HUB>), grid, block, lds, stream, a);
    else
        hipLaunchKernelGGL((ami_fwd_packed<NE, NI, DPT, EXACT, HUB>), grid, block, lds, stream, a);
}

// Self-energy shapes (order n: 2n-1 energies, n leaves and n-1 denominators
// per term) get exact instances; anything else the bounded generic one.
template <bool ADJ, bool HUB>
const char *launch_packed(const AmiTerms *t, dim3 grid, dim3 block, size_t lds, hipStream_t stream,
                          const KArgs &a) {
    const int ne = t->n_eps, ni = t->n_int, dpt = t->tab.dpt;
    const bool se = (ne == 2 * ni - 1) && (dpt == ni - 1) && (!HUB || t->n_g == ne);
#define AMI_SE(N)                                                                                 \
    if (se && ni == N) {                                                                          \
        launch_packed_one<ADJ, 2 * N - 1, N, N - 1, true, HUB>(grid, block, lds, stream, a);      \
        return "self-energy order " #N;                                                           \
    }
    AMI_SE(1)
    AMI_SE(2)
    AMI_SE(3)
    AMI_SE(4)
    AMI_SE(5)
    AMI_SE(6)
    AMI_SE(7)
#undef AMI_SE
    launch_packed_one<ADJ, 16, 8, 8, false, HUB>(grid, block, lds, stream, a);
    return "bounded generic";
}

}  // namespace

int fwd_slots(const Tables &tb) { return std::max(tb.L, 2 * tb.D) + tb.G; }

namespace {
int adj_slots(const Tables &tb) { return tb.L + 2 * tb.G + std::max(2 * tb.D, tb.L); }

AmiStatus launch_generic_forward(AmiTerms *t, DeviceTables *dt, bool hub, const KArgs &ka, double *partial,
                                 const LaunchShape &ls, dim3 grid, hipStream_t stream) {
    const Tables &tb = t->tab;
    FwdParams p;
    std::memset(&p, 0, sizeof(p));
    p.leaf_coef = dt->leaf_coef;
    p.leaf_sigma = dt->leaf_sigma;
    p.den_coef = dt->den_coef;
    p.group_dens = dt->group_dens;
    p.group_start = dt->group_start;
    p.term_sign = dt->term_sign;
    p.term_leaf = dt->term_leaf;
    p.line_alpha = dt->line_alpha;
    p.n_eps = t->n_eps;
    p.n_ext = t->n_ext;
    p.n_int = t->n_int;
    p.n_g = t->n_g;
    p.n_freq = t->n_freq;
    p.L = tb.L;
    p.D = tb.D;
    p.G = tb.G;
    p.dpt = tb.dpt;
    p.region_a = std::max(tb.L, 2 * tb.D);
    p.energies = ka.energies;
    p.stride_s = ka.stride_s;
    p.stride_i = ka.stride_i;
    p.k = ka.k;
    p.stride_k = ka.stride_k;
    for (int x = 0; x < 2 * kMaxExt; ++x) p.q[x] = ka.q[x];
    p.hop_t = ka.hop_t;
    p.mu = ka.mu;
    p.ext_freqs = ka.ext_freqs;
    p.n_f = ka.n_f;
    p.beta = ka.beta;
    p.e_reg = ka.e_reg;
    p.n_e = ka.n_e;
    p.out = ka.out;
    p.partial = partial;
    const int maxe = t->n_eps <= 4 ? 4 : (t->n_eps <= 8 ? 8 : 16);
    const dim3 block(ls.block);
#define AMI_LAUNCH(ME, H) hipLaunchKernelGGL((ami_fwd_kernel<ME, H>), grid, block, ls.lds, stream, p)
    if (hub) {
        if (maxe == 4) AMI_LAUNCH(4, true);
        else if (maxe == 8) AMI_LAUNCH(8, true);
        else AMI_LAUNCH(16, true);
    } else {
        if (maxe == 4) AMI_LAUNCH(4, false);
        else if (maxe == 8) AMI_LAUNCH(8, false);
        else AMI_LAUNCH(16, false);
    }
#undef AMI_LAUNCH
    return AMI_OK;
}

thread_local std::string g_last_variant;

// Optional HIP-event timing of the main evaluation kernel of each call on
// this thread (amiKernelTimerStart / amiKernelTimerStop).  The specialized
// kernels carry the events on their own dispatch (hipExtModuleLaunchKernel),
// so the pair brackets the kernel alone; the table-driven ones are bracketed
// by events recorded on the stream around the launch.
struct KernelTimer {
    bool on = false;
    std::vector<hipEvent_t> ev;      // start/stop pairs
    int used = 0;
};
thread_local KernelTimer g_timer;

void timer_mark(hipStream_t stream, bool stop) {
    if (!g_timer.on || g_timer.used >= static_cast<int>(g_timer.ev.size()) / 2) return;
    (void)hipEventRecord(g_timer.ev[2 * g_timer.used + (stop ? 1 : 0)], stream);
    if (stop) ++g_timer.used;
}

// The next start/stop pair for a dispatch, or false when the timer is off or full.
bool timer_pair(hipEvent_t &start, hipEvent_t &stop) {
    if (!g_timer.on || g_timer.used >= static_cast<int>(g_timer.ev.size()) / 2) return false;
    start = g_timer.ev[2 * g_timer.used];
    stop = g_timer.ev[2 * g_timer.used + 1];
    ++g_timer.used;
    return true;
}

enum class Path { TABLES, PACKED, SPECIALIZED, TWO_PASS, ADJ_PASSES };

// Workspace of one chunk of the two-pass forward and of the adjoint in passes
// (group sums, energies and their cotangents): 1 GiB unless
// amiSetTwoPassChunkBytes set another bound (a chunk never exceeds what the
// call's samples need).
std::atomic<int64_t> g_two_pass_chunk_bytes{int64_t(1) << 30};
// Frequency rows of one two-pass launch (its second kernel runs a block per
// tile and frequency row; the bound keeps that grid below 2^31 blocks).
constexpr int kTwoPassMaxFreqs = 65535;

// Which kernels serve a call (AMI_VARIANT_* of the handle); for the
// specialized path also loads them.  AUTO falls back and records why.
// With no_load the specialized kernels must already be loaded on the device
// (jit_loaded): nothing is compiled, loaded or allocated, and a kernel that
// the call would use but that is not loaded yet is an error, not a fallback.
// The adjoint of a large solution in passes (Path::ADJ_PASSES) takes three
// kernels: jit_fn (sums pass), jit_fn2 (frequency pass), jit_fn3 (leaf pass).
AmiStatus choose_path(AmiTerms *t, bool hub, bool adjoint, Path &p, void **jit_fn, std::string &note,
                      void **jit_fn2 = nullptr, int n_f = 1, int variant = -1, bool no_load = false,
                      void **jit_fn3 = nullptr) {
    const int v = variant >= 0 ? variant : t->variant;
    note.clear();
    auto get = [&](int kind, void **fn) {
        return no_load ? jit_loaded(t, hub, kind, fn) : jit_get(t, hub, kind, fn);
    };
    // the forward of a large solution: two passes (AUTO and SPECIALIZED when the
    // one-pass kernel would not fit its registers; TWO_PASS always)
    const bool two = !adjoint && jit_fn2 && n_f <= kTwoPassMaxFreqs &&
                     (v == AMI_VARIANT_TWO_PASS ||
                      ((v == AMI_VARIANT_AUTO || v == AMI_VARIANT_SPECIALIZED) && jit_prefers_two_pass(t)));
    const bool passes = adjoint && jit_fn2 && jit_fn3 &&
                        (v == AMI_VARIANT_TWO_PASS || (v == AMI_VARIANT_AUTO && t->tab.T > kJitAutoAdjointTerms));
    if (v == AMI_VARIANT_TWO_PASS && !two && !passes)
        return fail(AMI_E_UNSUPPORTED, adjoint ? "the two-pass variant of the adjoint runs in passes only"
                                               : "the two-pass variant takes at most 65535 frequency rows");
    if (passes) {
        std::string why;
        AmiStatus st = AMI_OK;
        if (!jit_adjoint_passes_supported(t, hub, &why)) st = fail(AMI_E_UNSUPPORTED, "no adjoint in passes: " + why);
        if (st == AMI_OK) st = get(kJitSumsPass, jit_fn);
        if (st == AMI_OK) st = get(kJitAdjFreq, jit_fn2);
        if (st == AMI_OK) st = get(kJitAdjLeaf, jit_fn3);
        if (st == AMI_OK) {
            p = Path::ADJ_PASSES;
            return AMI_OK;
        }
        if (v != AMI_VARIANT_AUTO || (no_load && st != AMI_E_UNSUPPORTED)) return st;
        note = std::string(" (not in passes: ") + amiLastError() + ")";
        clear_error();
    }
    if (two) {
        AmiStatus st = get(kJitSumsPass, jit_fn);
        if (st == AMI_OK) st = get(kJitFreqPass, jit_fn2);
        if (st == AMI_OK) {
            p = Path::TWO_PASS;
            return AMI_OK;
        }
        if (v != AMI_VARIANT_AUTO || (no_load && st != AMI_E_UNSUPPORTED)) return st;
        note = std::string(" (not two-pass: ") + amiLastError() + ")";
        clear_error();
    }
    const bool auto_skip = v == AMI_VARIANT_AUTO && adjoint && t->tab.T > kJitAutoAdjointTerms;
    if (auto_skip && note.empty())
        note = " (adjoint specialized in one pass up to " + std::to_string(kJitAutoAdjointTerms) + " terms)";
    if (v == AMI_VARIANT_SPECIALIZED || (v == AMI_VARIANT_AUTO && !auto_skip && !two)) {
        const AmiStatus st = get(adjoint ? kJitAdjoint : kJitForward, jit_fn);
        if (st == AMI_OK) {
            p = Path::SPECIALIZED;
            return AMI_OK;
        }
        if (v == AMI_VARIANT_SPECIALIZED || (no_load && st != AMI_E_UNSUPPORTED)) return st;
        note = std::string(" (not specialized: ") + amiLastError() + ")";
        clear_error();
    }
    if (!t->tab.uniform)
        return fail(AMI_E_UNSUPPORTED, "poles of higher order are evaluated by the specialized kernels only" + note);
    if (v == AMI_VARIANT_TABLES) {
        if (adjoint) return fail(AMI_E_UNSUPPORTED, "the double-table variant has no adjoint");
        p = Path::TABLES;
        return AMI_OK;
    }
    if (t->tab.packable) {
        p = Path::PACKED;
        return AMI_OK;
    }
    if (v == AMI_VARIANT_PACKED || adjoint)
        return fail(AMI_E_UNSUPPORTED,
                    "the packed kernels need +-1 coefficients and at most 255 leaves/denominators" + note);
    p = Path::TABLES;
    return AMI_OK;
}

// Partial-sum workspace of (handle, device, stream), at least `bytes` long:
// steady-state calls allocate nothing (and can be captured in a graph once a
// first call on the stream has sized it).
AmiStatus workspace(AmiTerms *t, DeviceTables *dt, hipStream_t stream, size_t bytes, double **out) {
    std::lock_guard<std::mutex> lk(t->dev_mu);
    DeviceTables::Workspace *w = nullptr;
    for (auto &x : dt->ws)
        if (x.stream == static_cast<void *>(stream)) w = &x;
    if (!w) {
        dt->ws.emplace_back();
        w = &dt->ws.back();
        w->stream = static_cast<void *>(stream);
    }
    if (w->bytes < bytes) {
        const size_t want = std::max(bytes, 2 * w->bytes);
        void *p = nullptr;
        const hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) return fail(AMI_E_OOM, std::string("workspace: ") + hipGetErrorString(e));
        if (w->ptr) dt->retired.push_back(w->ptr);     // a launch already queued may still read it
        w->ptr = p;
        w->bytes = want;
    }
    *out = static_cast<double *>(w->ptr);
    return AMI_OK;
}

// Launch of a specialized kernel on a grid of nblocks x gy blocks (timed by
// the kernel timer when it runs).
hipError_t launch_jit(void *fn, int64_t nblocks, int block, hipStream_t stream, KArgs &a, int gy = 1) {
    void *params[] = {&a};
    const hipFunction_t f = static_cast<hipFunction_t>(fn);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (g_timer.on) (void)hipStreamIsCapturing(stream, &cap);   // no timer events inside a capture
    if (nblocks * block <= 0xffffffffLL && cap == hipStreamCaptureStatusNone && timer_pair(t0, t1))
        return hipExtModuleLaunchKernel(f, static_cast<uint32_t>(nblocks * block), static_cast<uint32_t>(gy), 1,
                                        static_cast<uint32_t>(block), 1, 1, 0, stream, params, nullptr, t0, t1, 0);
    return hipModuleLaunchKernel(f, static_cast<unsigned>(nblocks), static_cast<unsigned>(gy), 1,
                                 static_cast<unsigned>(block), 1, 1, 0, stream, params, nullptr);
}

// The two-pass forward: the samples in chunks whose group sums and energies
// fit the chunk workspace; per chunk the sums pass (one lane per sample) and
// the frequency pass (a block per tile and frequency row), then one column reduction
// of the per-wave partial sums for the row sums.
// cplx: the complex-energy passes, whose group sums and energies take two
// columns each.
AmiStatus launch_two_pass(AmiTerms *t, DeviceTables *dt, bool hub, KArgs &a, double *out_sum, void *fn_sums,
                          void *fn_freq, hipStream_t stream, bool cplx = false) {
    const int B = jit_block(t, hub);
    const int64_t tiles = (a.n_e + B - 1) / B;
    if (tiles > 0x7fffffffLL) return fail(AMI_E_ARG, "n_e too large");
    const int64_t rows = tiles * (B / 64);
    const int64_t cols = (cplx ? 2 : 1) * (static_cast<int64_t>(t->tab.G) + t->n_eps);
    const int64_t chunk_bytes = g_two_pass_chunk_bytes.load();
    int64_t ld = chunk_bytes / (cols * static_cast<int64_t>(sizeof(double))) / B * B;
    ld = std::max<int64_t>(B, std::min<int64_t>(ld, tiles * B));
    ld = std::min<int64_t>(ld, int64_t(1) << 28);   // the kernels address a chunk with 32-bit byte offsets
    double *ws = nullptr;
    const int ncols = a.mc ? 4 * a.n_f : 2 * a.n_f;   // per-wave sums (Monte Carlo: with squares)
    const size_t n_part = out_sum ? static_cast<size_t>(rows) * ncols : 0;
    AmiStatus st = workspace(t, dt, stream, (static_cast<size_t>(cols) * ld + n_part) * sizeof(double), &ws);
    if (st != AMI_OK) return st;
    a.work = ws;
    a.ld = ld;
    a.partial = out_sum ? ws + static_cast<size_t>(cols) * ld : nullptr;
    a.nrows = rows;
    // the largest chunk's frequency pass: a block per tile and frequency row
    if ((std::min<int64_t>(ld, a.n_e) + B - 1) / B * a.n_f + 7 * a.n_f > 0x7fffffffLL)
        return fail(AMI_E_ARG, "two-pass chunk too large for its frequency rows");
    hipError_t e = hipSuccess;
    for (int64_t s0 = 0; s0 < a.n_e && e == hipSuccess; s0 += ld) {
        a.s0 = s0;
        a.n_chunk = std::min<int64_t>(ld, a.n_e - s0);
        const int64_t nb = (a.n_chunk + B - 1) / B;
        e = launch_jit(fn_sums, nb, B, stream, a);
        // (tile, frequency) blocks, tiles rounded up to a multiple of the 8 XCDs
        if (e == hipSuccess) e = launch_jit(fn_freq, (nb + 7) / 8 * 8 * a.n_f, B, stream, a);
    }
    if (e == hipSuccess) e = hipGetLastError();
    g_last_variant = cplx ? "specialized complex two-pass" : "specialized two-pass";
    if (e != hipSuccess) return hip_fail(e, "two-pass launch");
    if (out_sum) {
        hipLaunchKernelGGL(ami_colsum_kernel, dim3(ncols), dim3(kRedThreads), 0, stream, a.partial, rows,
                           static_cast<int64_t>(1), rows, out_sum);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "row-sum launch");
    }
    return AMI_OK;
}

AmiStatus launch_forward(AmiTerms *t, bool hub, KArgs &a, double *out_sum, hipStream_t stream, int variant = -1) {
    DeviceTables *dt = nullptr;
    AmiStatus st = upload(t, &dt);
    if (st != AMI_OK) return st;
    const Tables &tb = t->tab;
    if (a.n_e == 0) return fill(out_sum, 2 * static_cast<int64_t>(a.n_f), stream);
    Path path;
    void *jit_fn = nullptr, *jit_fn2 = nullptr;
    std::string note;
    st = choose_path(t, hub, false, path, &jit_fn, note, &jit_fn2, a.n_f, variant);
    if (st != AMI_OK) return st;
    if (path == Path::TWO_PASS) return launch_two_pass(t, dt, hub, a, out_sum, jit_fn, jit_fn2, stream);
    LaunchShape ls;
    if (path == Path::SPECIALIZED) {
        ls.block = jit_block(t, hub);
    } else {
        st = pick_shape(fwd_slots(tb), ls);
        if (st != AMI_OK) return st;
    }
    const int64_t nblocks = (a.n_e + ls.block - 1) / ls.block;
    if (nblocks > 0x7fffffffLL) return fail(AMI_E_ARG, "n_e too large");
    // partial-sum rows: one per wave for the specialized kernels, per block otherwise
    const int64_t rows = path == Path::SPECIALIZED ? nblocks * (ls.block / 64) : nblocks;
    double *partial = nullptr;
    hipError_t e;
    if (out_sum) {
        st = workspace(t, dt, stream, static_cast<size_t>(rows) * a.n_f * 2 * sizeof(double), &partial);
        if (st != AMI_OK) return st;
    }
    const dim3 grid(static_cast<unsigned>(nblocks)), block(ls.block);
    if (path != Path::SPECIALIZED) timer_mark(stream, false);
    if (path == Path::SPECIALIZED) {
        a.partial = partial;
        a.nrows = rows;
        e = launch_jit(jit_fn, nblocks, ls.block, stream, a);
        g_last_variant = "specialized";
        if (e == hipSuccess) e = hipGetLastError();
    } else if (path == Path::PACKED) {
        a.tb = packed_tabs(t, dt);
        a.slots = ls.slots;
        a.partial = partial;
        g_last_variant = std::string("packed ") +
                         (hub ? launch_packed<false, true>(t, grid, block, ls.lds, stream, a)
                              : launch_packed<false, false>(t, grid, block, ls.lds, stream, a)) + note;
        e = hipGetLastError();
    } else {
        launch_generic_forward(t, dt, hub, a, partial, ls, grid, stream);
        g_last_variant = "double tables" + note;
        e = hipGetLastError();
    }
    if (path != Path::SPECIALIZED) timer_mark(stream, true);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    if (out_sum) {
        const bool cm = path == Path::SPECIALIZED;
        hipLaunchKernelGGL(ami_colsum_kernel, dim3(2 * a.n_f), dim3(kRedThreads), 0, stream, partial, rows,
                           static_cast<int64_t>(cm ? 1 : 2 * a.n_f), cm ? rows : static_cast<int64_t>(1), out_sum);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "row-sum launch");
    }
    return AMI_OK;
}

// Scratch of the allocation-free entry point (amiEvaluateHubbardAdjointNoAlloc):
// the partial sums of one call.  Every device the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: kernels get the address hipGetSymbolAddress
// returns for the current device (scratch_address).
constexpr size_t kScratchBytes = AMI_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kScratchMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call there.
AmiStatus scratch_address(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kScratchMaxDevices) return fail(AMI_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (scratch)");
        if (!p) return fail(AMI_E_HIP, "hipGetSymbolAddress (scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return AMI_OK;
}

// The handle's tables on the current device when amiTermsUpload (or an
// earlier evaluate call) has put them there; uploads nothing.
AmiStatus find_uploaded(AmiTerms *t, DeviceTables **out) {
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(t->dev_mu);
    for (auto &d : t->dev)
        if (d.device == dev) {
            *out = &d;
            return AMI_OK;
        }
    return fail(AMI_E_ARG, "the tables are not on this device: call amiTermsUpload first");
}

struct AdjOut {
    double *grad_beta = nullptr, *grad_mu = nullptr, *grad_t = nullptr, *grad_freqs = nullptr;
    double *out_sum = nullptr;   // forward row sums computed on the way (optional)
};

// The adjoint of a large solution in passes, per chunk of samples: the
// two-pass forward's sums pass (FT_g and E_j into the workspace), the
// frequency pass (values, FTB_g and the denominators' energy cotangents into
// the workspace, wave sums of dL/dw and of the values), the leaf pass (leaf
// cotangents, per-sample gradients, wave sums of dL/dbeta, dL/dmu, dL/dt);
// then one reduction of the wave sums.  Workspace: the partial sums (rows x
// columns), then the chunk's 2 G + 2 NE columns of ld samples each.
// fixed_ws: both in the allocation-free scratch (the chunk sized to what is
// left), nothing allocated.
// cplx: the passes at complex energies, whose workspace columns are complex
// (4 G + 4 NE of them).
AmiStatus launch_adjoint_passes(AmiTerms *t, DeviceTables *dt, bool hub, KArgs &a, const AdjOut &o, void *fn_sums,
                                void *fn_freq, void *fn_leaf, hipStream_t stream, double *fixed_ws,
                                bool cplx = false) {
    const int B = jit_block(t, hub);
    const int64_t tiles = (a.n_e + B - 1) / B;
    if (tiles > 0x7fffffffLL) return fail(AMI_E_ARG, "n_e too large");
    const int64_t rows = tiles * (B / 64);
    const int ncols = kAdjScalars + 2 * a.n_f * t->n_ext;
    const int nval = o.out_sum ? 2 * a.n_f : 0;
    const int64_t cols = (cplx ? 2 : 1) * (2 * static_cast<int64_t>(t->tab.G) + 2 * t->n_eps);
    const size_t n_part = static_cast<size_t>(rows) * (ncols + nval);
    int64_t ld = 0;
    double *ws = nullptr;
    if (fixed_ws) {
        const int64_t left = static_cast<int64_t>(kScratchBytes / sizeof(double)) - static_cast<int64_t>(n_part);
        ld = left > 0 ? left / cols / B * B : 0;
        if (ld < B)
            return fail(AMI_E_ARG, "the partial sums and one chunk of samples do not fit the " +
                                       std::to_string(kScratchBytes) +
                                       "-byte scratch of the allocation-free entry point: split the samples");
        ld = std::min<int64_t>(ld, tiles * B);
        ws = fixed_ws;
    } else {
        ld = g_two_pass_chunk_bytes.load() / (cols * static_cast<int64_t>(sizeof(double))) / B * B;
        ld = std::max<int64_t>(B, std::min<int64_t>(ld, tiles * B));
    }
    ld = std::min<int64_t>(ld, int64_t(1) << 28);   // the kernels address a chunk with 32-bit byte offsets
    if (!fixed_ws) {
        const AmiStatus st = workspace(t, dt, stream, (n_part + static_cast<size_t>(cols) * ld) * sizeof(double), &ws);
        if (st != AMI_OK) return st;
    }
    a.gpartial = ws;
    a.partial = o.out_sum ? ws + static_cast<size_t>(rows) * ncols : nullptr;
    a.nrows = rows;
    a.work = ws + n_part;
    a.ld = ld;
    a.mc = 0;
    hipError_t e = hipSuccess;
    for (int64_t s0 = 0; s0 < a.n_e && e == hipSuccess; s0 += ld) {
        a.s0 = s0;
        a.n_chunk = std::min<int64_t>(ld, a.n_e - s0);
        const int64_t nb = (a.n_chunk + B - 1) / B;
        e = launch_jit(fn_sums, nb, B, stream, a);
        if (e == hipSuccess) e = launch_jit(fn_freq, nb, B, stream, a);
        if (e == hipSuccess) e = launch_jit(fn_leaf, nb, B, stream, a);
    }
    if (e == hipSuccess) e = hipGetLastError();
    g_last_variant = cplx ? "specialized complex passes" : "specialized passes";
    if (e != hipSuccess) return hip_fail(e, "adjoint passes launch");
    hipLaunchKernelGGL(ami_adj_finalize_kernel, dim3(ncols + nval), dim3(kRedThreads), 0, stream, a.gpartial, rows,
                       ncols, 1, o.grad_beta, o.grad_mu, o.grad_t, o.grad_freqs, 2 * a.n_f, o.out_sum);
    e = hipGetLastError();
    return e == hipSuccess ? AMI_OK : hip_fail(e, "adjoint reduction launch");
}

// fixed_ws: the partial sums go there (at most kScratchBytes), and nothing is
// uploaded, compiled, loaded or allocated (the allocation-free entry point);
// NULL: the handle's per-stream workspace.
AmiStatus launch_adjoint(AmiTerms *t, bool hub, KArgs &a, const AdjOut &o, hipStream_t stream,
                         double *fixed_ws = nullptr) {
    DeviceTables *dt = nullptr;
    AmiStatus st = fixed_ws ? find_uploaded(t, &dt) : upload(t, &dt);
    if (st != AMI_OK) return st;
    const Tables &tb = t->tab;
    const int nx = t->n_ext;
    const int ncols = kAdjScalars + 2 * a.n_f * nx;
    if (a.n_e == 0) {
        for (double *p : {o.grad_beta, o.grad_mu, o.grad_t}) {
            st = fill(p, 1, stream);
            if (st != AMI_OK) return st;
        }
        st = fill(o.out_sum, 2 * static_cast<int64_t>(a.n_f), stream);
        if (st != AMI_OK) return st;
        return fill(o.grad_freqs, 2 * static_cast<int64_t>(a.n_f) * nx, stream);
    }
    Path path;
    void *jit_fn = nullptr, *jit_fn2 = nullptr, *jit_fn3 = nullptr;
    std::string note;
    st = choose_path(t, hub, true, path, &jit_fn, note, &jit_fn2, a.n_f, -1, fixed_ws != nullptr, &jit_fn3);
    if (st != AMI_OK) return st;
    if (path == Path::ADJ_PASSES)
        return launch_adjoint_passes(t, dt, hub, a, o, jit_fn, jit_fn2, jit_fn3, stream, fixed_ws);
    LaunchShape ls;
    if (path == Path::SPECIALIZED) {
        ls.block = jit_block(t, hub);
    } else {
        st = pick_shape(adj_slots(tb), ls);
        if (st != AMI_OK) return st;
    }
    const int64_t nblocks = (a.n_e + ls.block - 1) / ls.block;
    if (nblocks > 0x7fffffffLL) return fail(AMI_E_ARG, "n_e too large");
    // partial-sum rows: one per wave for the specialized kernels, per block otherwise
    const int64_t rows = path == Path::SPECIALIZED ? nblocks * (ls.block / 64) : nblocks;
    double *partial = nullptr;
    const size_t n_grad = static_cast<size_t>(rows) * ncols;
    const size_t n_val = o.out_sum ? static_cast<size_t>(rows) * a.n_f * 2 : 0;
    const size_t ws_bytes = (n_grad + n_val) * sizeof(double);
    if (fixed_ws) {
        if (ws_bytes > kScratchBytes)
            return fail(AMI_E_ARG, "the partial sums need " + std::to_string(ws_bytes) +
                                       " bytes, more than the " + std::to_string(kScratchBytes) +
                                       "-byte scratch of the allocation-free entry point: split the samples");
        partial = fixed_ws;
    } else {
        st = workspace(t, dt, stream, ws_bytes, &partial);
        if (st != AMI_OK) return st;
    }
    hipError_t e;
    a.gpartial = partial;
    a.partial = o.out_sum ? partial + n_grad : nullptr;
    const dim3 grid(static_cast<unsigned>(nblocks)), block(ls.block);
    if (path == Path::SPECIALIZED) {
        a.nrows = rows;
        e = launch_jit(jit_fn, nblocks, ls.block, stream, a);
        g_last_variant = "specialized";
        if (e == hipSuccess) e = hipGetLastError();
    } else {
        a.tb = packed_tabs(t, dt);
        a.slots = ls.slots;
        timer_mark(stream, false);
        g_last_variant = std::string("packed ") +
                         (hub ? launch_packed<true, true>(t, grid, block, ls.lds, stream, a)
                              : launch_packed<true, false>(t, grid, block, ls.lds, stream, a)) + note;
        e = hipGetLastError();
        timer_mark(stream, true);
    }
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    // one launch for every reduction: gradient columns, then the value row sums
    const int n_red = ncols + (o.out_sum ? 2 * a.n_f : 0);
    hipLaunchKernelGGL(ami_adj_finalize_kernel, dim3(n_red), dim3(kRedThreads), 0, stream, partial, rows, ncols,
                       path == Path::SPECIALIZED ? 1 : 0, o.grad_beta, o.grad_mu, o.grad_t, o.grad_freqs, 2 * a.n_f,
                       o.out_sum);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "adjoint reduction launch");
    return AMI_OK;
}

AmiStatus check_common(const AmiTerms *t, int64_t n_e, const double *ext_freqs, int64_t n_f, double beta) {
    if (!t) return fail(AMI_E_ARG, "terms is NULL");
    if (n_e < 0) return fail(AMI_E_ARG, "n_e < 0");
    if (n_f < 1 || n_f > (1 << 24)) return fail(AMI_E_ARG, "n_f must be in 1..2^24");
    if (!ext_freqs && t->n_ext > 0) return fail(AMI_E_ARG, "ext_freqs is NULL");
    if (!(beta > 0.0)) return fail(AMI_E_ARG, "beta must be > 0");
    if (t->n_eps > kMaxEpsDev) return fail(AMI_E_UNSUPPORTED, "more than 16 energy placeholders");
    if (t->n_ext > kMaxExt) return fail(AMI_E_UNSUPPORTED, "more than 4 external frequency slots");
    return AMI_OK;
}

AmiStatus check_energies(const AmiTerms *, int64_t n_e, const double *energies, int64_t stride_s,
                         int64_t stride_i) {
    if (n_e > 0 && !energies) return fail(AMI_E_ARG, "energies is NULL");
    if (n_e > 0 && (stride_i < 1 || stride_s < 1)) return fail(AMI_E_ARG, "strides must be >= 1");
    return AMI_OK;
}

AmiStatus check_momenta(const AmiTerms *t, int64_t n_e, const double *k, int64_t stride_k, const double *q) {
    if (t->n_eps != t->n_g) return fail(AMI_E_ARG, "the momentum path needs one energy per propagator");
    if (t->n_int > kMaxInt) return fail(AMI_E_UNSUPPORTED, "more than 12 summed frequencies on the momentum path");
    if (n_e > 0 && !k) return fail(AMI_E_ARG, "k is NULL");
    if (n_e > 0 && stride_k < 2 * t->n_int) return fail(AMI_E_ARG, "stride_k < 2*n_int");
    if (t->n_ext > 0 && !q) return fail(AMI_E_ARG, "q is NULL");
    return AMI_OK;
}

void set_momenta(KArgs &a, const AmiTerms *t, const double *k, int64_t stride_k, const double *q, double hop_t,
                 double mu) {
    a.k = k;
    a.stride_k = stride_k;
    a.q_big = 0;
    if (k && (reinterpret_cast<uintptr_t>(k) & 15u) == 0 && (stride_k & 1) == 0) a.vec_io |= 1;
    for (int x = 0; x < t->n_ext && x < kMaxExtDev; ++x)
        for (int c = 0; c < 2; ++c) {
            const double r = std::remainder(q[2 * x + c], 2.0 * M_PI);
            a.q[2 * x + c] = r;
            a.qs[2 * x + c] = std::sin(r);
            a.qc[2 * x + c] = std::cos(r);
        }
    a.hop_t = hop_t;
    a.mu = mu;
}

void set_common(KArgs &a, const double *ext_freqs, int64_t n_f, double beta, double e_reg, int64_t n_e) {
    a.ext_freqs = ext_freqs;
    a.n_f = static_cast<int>(n_f);
    a.beta = beta;
    a.e_reg = e_reg;
    a.n_e = n_e;
}

}  // namespace

AmiStatus launch_forward_as(AmiTerms *t, bool hub, KArgs &a, double *out_sum, hipStream_t stream, int variant) {
    return launch_forward(t, hub, a, out_sum, stream, variant);
}

bool specialized_forward_ready(AmiTerms *t, bool hub, int n_f) {
    Path p;
    void *f1 = nullptr, *f2 = nullptr;
    std::string note;
    const AmiStatus st = choose_path(t, hub, false, p, &f1, note, &f2, n_f, AMI_VARIANT_AUTO);
    clear_error();
    return st == AMI_OK && (p == Path::SPECIALIZED || p == Path::TWO_PASS);
}

void set_inputs(KArgs &a, const AmiTerms *t, const double *k, int64_t stride_k, const double *q, double hop_t,
                double mu, const double *energies, int64_t stride_s, int64_t stride_i, const double *ext_freqs,
                int64_t n_f, double beta, double e_reg, int64_t n_e) {
    if (k) set_momenta(a, t, k, stride_k, q, hop_t, mu);
    a.energies = energies;
    a.stride_s = stride_s;
    a.stride_i = stride_i;
    set_common(a, ext_freqs, n_f, beta, e_reg, n_e);
}

}  // namespace ami

extern "C" {

AmiStatus amiTermsUpload(AmiTerms *t) {
    ami::clear_error();
    if (!t) return ami::fail(AMI_E_ARG, "terms is NULL");
    ami::DeviceTables *dt = nullptr;
    return ami::upload(t, &dt);
}

void amiFree(AmiTerms *t) {
    if (!t) return;
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (auto &d : t->dev)
        if (hipSetDevice(d.device) == hipSuccess) {
            if (d.blob) (void)hipFree(d.blob);
            for (auto &w : d.ws) (void)hipFree(w.ptr);
            for (void *p : d.retired) (void)hipFree(p);
        }
    if (have_cur) (void)hipSetDevice(cur);
    ami::jit_release(t);
    delete t;
}

AmiStatus amiEvaluate(AmiTerms *t, const double *energies, int64_t n_e, int64_t stride_s, int64_t stride_i,
                      const double *ext_freqs, int64_t n_f, double beta, double e_reg, double *out,
                      double *out_sum, void *hip_stream) {
    using namespace ami;
    clear_error();
    AmiStatus st = check_common(t, n_e, ext_freqs, n_f, beta);
    if (st == AMI_OK) st = check_energies(t, n_e, energies, stride_s, stride_i);
    if (st != AMI_OK) return st;
    if (!out && !out_sum) return fail(AMI_E_ARG, "out and out_sum are both NULL");
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.energies = energies;
    a.stride_s = stride_s;
    a.stride_i = stride_i;
    set_common(a, ext_freqs, n_f, beta, e_reg, n_e);
    a.out = out;
    return launch_forward(t, false, a, out_sum, static_cast<hipStream_t>(hip_stream));
}

AmiStatus amiEvaluateComplex(AmiTerms *t, const double *energies, int64_t n_e, int64_t stride_s, int64_t stride_i,
                             const double *ext_freqs, int64_t n_f, double beta, double e_reg, double *out,
                             double *out_sum, void *hip_stream) {
    using namespace ami;
    clear_error();
    AmiStatus st = check_common(t, n_e, ext_freqs, n_f, beta);
    if (st == AMI_OK) st = check_energies(t, n_e, energies, stride_s, stride_i);
    if (st != AMI_OK) return st;
    if (!out && !out_sum) return fail(AMI_E_ARG, "out and out_sum are both NULL");
    const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    DeviceTables *dt = nullptr;
    st = upload(t, &dt);
    if (st != AMI_OK) return st;
    // solutions above the one-pass size (or the forced two-pass variant): the
    // complex group sums stored per sample, then evaluated per frequency row
    if (t->tab.T > kJitMaxTerms || t->variant == AMI_VARIANT_TWO_PASS) {
        void *fs = nullptr, *ff = nullptr;
        st = jit_get(t, false, kJitComplexSums, &fs);
        if (st == AMI_OK) st = jit_get(t, false, kJitComplexFreq, &ff);
        if (st != AMI_OK) return st;
        if (n_e == 0) return fill(out_sum, 2 * n_f, stream);
        if (n_f > kTwoPassMaxFreqs) return fail(AMI_E_ARG, "the two-pass variant takes at most 65535 frequency rows");
        KArgs a;
        std::memset(&a, 0, sizeof(a));
        a.energies = energies;
        a.stride_s = stride_s;
        a.stride_i = stride_i;
        set_common(a, ext_freqs, n_f, beta, e_reg, n_e);
        a.out = out;
        return launch_two_pass(t, dt, false, a, out_sum, fs, ff, stream, true);
    }
    void *fn = nullptr;
    st = jit_get(t, false, kJitComplex, &fn);
    if (st != AMI_OK) return st;
    if (n_e == 0) return fill(out_sum, 2 * n_f, stream);
    const int block = jit_block(t, false);
    const int64_t nblocks = (n_e + block - 1) / block;
    if (nblocks > 0x7fffffffLL) return fail(AMI_E_ARG, "n_e too large");
    const int64_t rows = nblocks * (block / 64);   // partial sums per wave
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.energies = energies;
    a.stride_s = stride_s;
    a.stride_i = stride_i;
    set_common(a, ext_freqs, n_f, beta, e_reg, n_e);
    a.out = out;
    a.nrows = rows;
    if (out_sum) {
        st = workspace(t, dt, stream, static_cast<size_t>(rows) * n_f * 2 * sizeof(double), &a.partial);
        if (st != AMI_OK) return st;
    }
    hipError_t e = launch_jit(fn, nblocks, block, stream, a);
    if (e == hipSuccess) e = hipGetLastError();
    g_last_variant = "specialized complex";
    if (e != hipSuccess) return hip_fail(e, "complex-energy launch");
    if (out_sum) {
        hipLaunchKernelGGL(ami_colsum_kernel, dim3(static_cast<unsigned>(2 * n_f)), dim3(kRedThreads), 0, stream,
                           a.partial, rows, static_cast<int64_t>(1), rows, out_sum);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "row-sum launch");
    }
    return AMI_OK;
}

AmiStatus amiEvaluateComplexAdjoint(AmiTerms *t, const double *energies, int64_t n_e, int64_t stride_s,
                                    int64_t stride_i, const double *ext_freqs, int64_t n_f, double beta, double e_reg,
                                    const double *grad_out, const double *grad_sum, double *grad_energies,
                                    double *grad_beta, double *grad_freqs, double *out, double *out_sum,
                                    void *hip_stream) {
    using namespace ami;
    clear_error();
    AmiStatus st = check_common(t, n_e, ext_freqs, n_f, beta);
    if (st == AMI_OK) st = check_energies(t, n_e, energies, stride_s, stride_i);
    if (st != AMI_OK) return st;
    if (!grad_out && !grad_sum) return fail(AMI_E_ARG, "grad_out and grad_sum are both NULL");
    const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    DeviceTables *dt = nullptr;
    st = upload(t, &dt);
    if (st != AMI_OK) return st;
    // above the one-pass complex adjoint's automatic size (unless the handle
    // forces the specialized variant), or under the forced two-pass variant:
    // the adjoint in passes at complex energies
    if (t->variant == AMI_VARIANT_TWO_PASS ||
        (t->variant != AMI_VARIANT_SPECIALIZED && t->tab.T > kJitAutoComplexAdjointTerms)) {
        void *fs = nullptr, *ff = nullptr, *fl = nullptr;
        st = jit_get(t, false, kJitComplexSums, &fs);
        if (st == AMI_OK) st = jit_get(t, false, kJitComplexAdjFreq, &ff);
        if (st == AMI_OK) st = jit_get(t, false, kJitComplexAdjLeaf, &fl);
        if (st != AMI_OK) return st;
        if (n_e == 0) {
            st = fill(grad_beta, 1, stream);
            if (st == AMI_OK) st = fill(out_sum, 2 * n_f, stream);
            if (st == AMI_OK) st = fill(grad_freqs, 2 * n_f * t->n_ext, stream);
            return st;
        }
        KArgs a;
        std::memset(&a, 0, sizeof(a));
        a.energies = energies;
        a.stride_s = stride_s;
        a.stride_i = stride_i;
        set_common(a, ext_freqs, n_f, beta, e_reg, n_e);
        a.g_out = grad_out;
        a.g_sum = grad_sum;
        a.grad_e = grad_energies;
        a.out = out;
        AdjOut o;
        o.grad_beta = grad_beta;
        o.grad_freqs = grad_freqs;
        o.out_sum = out_sum;
        return launch_adjoint_passes(t, dt, false, a, o, fs, ff, fl, stream, nullptr, true);
    }
    void *fn = nullptr;
    st = jit_get(t, false, kJitComplexAdj, &fn);
    if (st != AMI_OK) return st;
    const int nx = t->n_ext;
    const int ncols = kAdjScalars + 2 * static_cast<int>(n_f) * nx;
    if (n_e == 0) {
        st = fill(grad_beta, 1, stream);
        if (st == AMI_OK) st = fill(out_sum, 2 * n_f, stream);
        if (st == AMI_OK) st = fill(grad_freqs, 2 * n_f * nx, stream);
        return st;
    }
    const int block = jit_block(t, false);
    const int64_t nblocks = (n_e + block - 1) / block;
    if (nblocks > 0x7fffffffLL) return fail(AMI_E_ARG, "n_e too large");
    const int64_t rows = nblocks * (block / 64);   // partial sums per wave
    const size_t n_grad = static_cast<size_t>(rows) * ncols;
    const size_t n_val = out_sum ? static_cast<size_t>(rows) * n_f * 2 : 0;
    double *partial = nullptr;
    st = workspace(t, dt, stream, (n_grad + n_val) * sizeof(double), &partial);
    if (st != AMI_OK) return st;
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.energies = energies;
    a.stride_s = stride_s;
    a.stride_i = stride_i;
    set_common(a, ext_freqs, n_f, beta, e_reg, n_e);
    a.g_out = grad_out;
    a.g_sum = grad_sum;
    a.grad_e = grad_energies;
    a.out = out;
    a.nrows = rows;
    a.gpartial = partial;
    a.partial = out_sum ? partial + n_grad : nullptr;
    hipError_t e = launch_jit(fn, nblocks, block, stream, a);
    if (e == hipSuccess) e = hipGetLastError();
    g_last_variant = "specialized complex";
    if (e != hipSuccess) return hip_fail(e, "complex-energy adjoint launch");
    const int n_red = ncols + (out_sum ? 2 * static_cast<int>(n_f) : 0);
    hipLaunchKernelGGL(ami_adj_finalize_kernel, dim3(n_red), dim3(kRedThreads), 0, stream, partial, rows, ncols, 1,
                       grad_beta, static_cast<double *>(nullptr), static_cast<double *>(nullptr), grad_freqs,
                       2 * static_cast<int>(n_f), out_sum);
    e = hipGetLastError();
    return e == hipSuccess ? AMI_OK : hip_fail(e, "adjoint reduction launch");
}

AmiStatus amiEvaluateHubbard(AmiTerms *t, const double *k, int64_t n_e, int64_t stride_k, const double *q,
                             double hop_t, double mu, const double *ext_freqs, int64_t n_f, double beta,
                             double e_reg, double *out, double *out_sum, void *hip_stream) {
    using namespace ami;
    clear_error();
    AmiStatus st = check_common(t, n_e, ext_freqs, n_f, beta);
    if (st == AMI_OK) st = check_momenta(t, n_e, k, stride_k, q);
    if (st != AMI_OK) return st;
    if (!out && !out_sum) return fail(AMI_E_ARG, "out and out_sum are both NULL");
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    set_momenta(a, t, k, stride_k, q, hop_t, mu);
    set_common(a, ext_freqs, n_f, beta, e_reg, n_e);
    a.out = out;
    return launch_forward(t, true, a, out_sum, static_cast<hipStream_t>(hip_stream));
}

AmiStatus amiEvaluateAdjoint(AmiTerms *t, const double *energies, int64_t n_e, int64_t stride_s,
                             int64_t stride_i, const double *ext_freqs, int64_t n_f, double beta, double e_reg,
                             const double *grad_out, const double *grad_sum, double *grad_energies,
                             double *grad_beta, double *grad_freqs, double *out, double *out_sum,
                             void *hip_stream) {
    using namespace ami;
    clear_error();
    AmiStatus st = check_common(t, n_e, ext_freqs, n_f, beta);
    if (st == AMI_OK) st = check_energies(t, n_e, energies, stride_s, stride_i);
    if (st != AMI_OK) return st;
    if (!grad_out && !grad_sum) return fail(AMI_E_ARG, "grad_out and grad_sum are both NULL");
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.energies = energies;
    a.stride_s = stride_s;
    a.stride_i = stride_i;
    set_common(a, ext_freqs, n_f, beta, e_reg, n_e);
    a.g_out = grad_out;
    a.g_sum = grad_sum;
    a.grad_e = grad_energies;
    a.out = out;
    AdjOut o;
    o.grad_beta = grad_beta;
    o.grad_freqs = grad_freqs;
    o.out_sum = out_sum;
    return launch_adjoint(t, false, a, o, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

namespace ami {
namespace {

AmiStatus hubbard_adjoint(AmiTerms *t, const double *k, int64_t n_e, int64_t stride_k, const double *q,
                          double hop_t, double mu, const double *ext_freqs, int64_t n_f, double beta, double e_reg,
                          const double *grad_out, const double *grad_sum, double *grad_k, double *grad_mu,
                          double *grad_t, double *grad_beta, double *grad_freqs, double *out, double *out_sum,
                          void *hip_stream, bool no_alloc) {
    clear_error();
    AmiStatus st = check_common(t, n_e, ext_freqs, n_f, beta);
    if (st == AMI_OK) st = check_momenta(t, n_e, k, stride_k, q);
    if (st != AMI_OK) return st;
    if (!grad_out && !grad_sum) return fail(AMI_E_ARG, "grad_out and grad_sum are both NULL");
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    set_momenta(a, t, k, stride_k, q, hop_t, mu);
    set_common(a, ext_freqs, n_f, beta, e_reg, n_e);
    a.g_out = grad_out;
    a.g_sum = grad_sum;
    a.grad_k = grad_k;
    if (grad_k && (reinterpret_cast<uintptr_t>(grad_k) & 15u) == 0) a.vec_io |= 2;
    a.out = out;
    AdjOut o;
    o.grad_beta = grad_beta;
    o.grad_mu = grad_mu;
    o.grad_t = grad_t;
    o.grad_freqs = grad_freqs;
    o.out_sum = out_sum;
    double *ws = nullptr;
    if (no_alloc) {
        st = scratch_address(&ws);
        if (st != AMI_OK) return st;
    }
    return launch_adjoint(t, true, a, o, static_cast<hipStream_t>(hip_stream), ws);
}

}  // namespace
}  // namespace ami

extern "C" {

AmiStatus amiEvaluateHubbardAdjoint(AmiTerms *t, const double *k, int64_t n_e, int64_t stride_k, const double *q,
                                    double hop_t, double mu, const double *ext_freqs, int64_t n_f, double beta,
                                    double e_reg, const double *grad_out, const double *grad_sum, double *grad_k,
                                    double *grad_mu, double *grad_t, double *grad_beta, double *grad_freqs,
                                    double *out, double *out_sum, void *hip_stream) {
    return ami::hubbard_adjoint(t, k, n_e, stride_k, q, hop_t, mu, ext_freqs, n_f, beta, e_reg, grad_out, grad_sum,
                                grad_k, grad_mu, grad_t, grad_beta, grad_freqs, out, out_sum, hip_stream, false);
}

AmiStatus amiEvaluateHubbardAdjointNoAlloc(AmiTerms *t, const double *k, int64_t n_e, int64_t stride_k,
                                           const double *q, double hop_t, double mu, const double *ext_freqs,
                                           int64_t n_f, double beta, double e_reg, const double *grad_out,
                                           const double *grad_sum, double *grad_k, double *grad_mu, double *grad_t,
                                           double *grad_beta, double *grad_freqs, double *out, double *out_sum,
                                           void *hip_stream) {
    return ami::hubbard_adjoint(t, k, n_e, stride_k, q, hop_t, mu, ext_freqs, n_f, beta, e_reg, grad_out, grad_sum,
                                grad_k, grad_mu, grad_t, grad_beta, grad_freqs, out, out_sum, hip_stream, true);
}

AmiStatus amiIntegrateHubbard(AmiTerms *t, int64_t n_samples, uint64_t seed, const double *q, double hop_t,
                              double mu, const double *ext_freqs, int64_t n_f, double beta, double e_reg,
                              double *sums, void *hip_stream) {
    using namespace ami;
    clear_error();
    AmiStatus st = check_common(t, n_samples, ext_freqs, n_f, beta);
    if (st != AMI_OK) return st;
    if (n_f > kMcMaxFreqs) return fail(AMI_E_ARG, "at most 8 frequency rows per Monte-Carlo call");
    if (!sums) return fail(AMI_E_ARG, "sums is NULL");
    if (t->n_eps != t->n_g) return fail(AMI_E_ARG, "the momentum path needs one energy per propagator");
    if (t->n_ext > 0 && !q) return fail(AMI_E_ARG, "q is NULL");
    const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    DeviceTables *dt = nullptr;
    st = upload(t, &dt);
    if (st != AMI_OK) return st;
    if (jit_prefers_two_pass(t)) {
        // large solutions: the two-pass kernels, momenta drawn in the first
        void *f1 = nullptr, *f2 = nullptr;
        st = jit_get(t, true, kJitSumsPass, &f1);
        if (st == AMI_OK) st = jit_get(t, true, kJitFreqPass, &f2);
        if (st != AMI_OK) return st;
        if (n_samples == 0) return fill(sums, 4 * n_f, stream);
        KArgs a;
        std::memset(&a, 0, sizeof(a));
        set_momenta(a, t, nullptr, 0, q, hop_t, mu);
        set_common(a, ext_freqs, n_f, beta, e_reg, n_samples);
        a.seed = seed;
        a.mc = 1;
        return launch_two_pass(t, dt, true, a, sums, f1, f2, stream);
    }
    void *fn = nullptr;
    st = jit_get(t, true, kJitMonteCarlo, &fn);
    if (st != AMI_OK) return st;
    if (n_samples == 0) return fill(sums, 4 * n_f, stream);
    int dev = 0, n_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    // a fixed grid per device (the sums are reduced in a fixed order for it):
    // eight blocks per CU, or fewer when there are fewer samples
    const int block = jit_block(t, true);
    const int64_t grid = std::min<int64_t>((n_samples + block - 1) / block, 8 * static_cast<int64_t>(n_cu));
    const int64_t rows = grid * (block / 64);   // partial sums per wave
    double *partial = nullptr;
    st = workspace(t, dt, stream, static_cast<size_t>(rows) * n_f * 4 * sizeof(double), &partial);
    if (st != AMI_OK) return st;
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    set_momenta(a, t, nullptr, 0, q, hop_t, mu);
    set_common(a, ext_freqs, n_f, beta, e_reg, n_samples);
    a.seed = seed;
    a.partial = partial;
    a.nrows = rows;
    e = launch_jit(fn, grid, block, stream, a);
    if (e == hipSuccess) e = hipGetLastError();
    g_last_variant = "specialized";
    if (e != hipSuccess) return hip_fail(e, "Monte-Carlo launch");
    hipLaunchKernelGGL(ami_colsum_kernel, dim3(static_cast<unsigned>(4 * n_f)), dim3(kRedThreads), 0, stream, partial,
                       rows, static_cast<int64_t>(1), rows, sums);
    e = hipGetLastError();
    return e == hipSuccess ? AMI_OK : hip_fail(e, "Monte-Carlo reduction launch");
}

AmiStatus amiSetTwoPassChunkBytes(int64_t bytes) {
    ami::clear_error();
    if (bytes < (int64_t(1) << 16)) return ami::fail(AMI_E_ARG, "the chunk bound must be at least 64 KiB");
    ami::g_two_pass_chunk_bytes.store(bytes);
    return AMI_OK;
}

AmiStatus amiSetVariant(AmiTerms *t, int32_t variant) {
    ami::clear_error();
    if (!t) return ami::fail(AMI_E_ARG, "terms is NULL");
    if (variant < AMI_VARIANT_AUTO || variant > AMI_VARIANT_TWO_PASS)
        return ami::fail(AMI_E_ARG, "variant must be one of AMI_VARIANT_*");
    t->variant = variant;
    return AMI_OK;
}

AmiStatus amiTermsSpecialize(AmiTerms *t, int32_t momentum) {
    ami::clear_error();
    if (!t) return ami::fail(AMI_E_ARG, "terms is NULL");
    using namespace ami;
    const bool hub = momentum != 0;
    bool taylor = false;                    // Taylor-coefficient leaves: no complex energies
    for (int o : t->tab.leaf_order) taylor = taylor || o > 0;
    // the kernels for this input: forward, adjoint, and the complex-energy
    // forward for the energy input; all compiled before any device is touched
    const bool small = t->tab.T <= kJitMaxTerms;
    std::vector<int> kinds;
    if (jit_prefers_two_pass(t)) {
        kinds.push_back(kJitSumsPass);
        kinds.push_back(kJitFreqPass);
    } else {
        kinds.push_back(kJitForward);
    }
    if (t->tab.T <= kJitAutoAdjointTerms) kinds.push_back(kJitAdjoint);
    if (t->tab.T > kJitAutoAdjointTerms && jit_adjoint_passes_supported(t, hub, nullptr)) {
        if (!jit_prefers_two_pass(t)) kinds.push_back(kJitSumsPass);
        kinds.push_back(kJitAdjFreq);
        kinds.push_back(kJitAdjLeaf);
    }
    // the complex-energy kernels AUTO uses: forward in one pass up to 1024
    // terms, in two above; the adjoint in one pass up to 512 terms, in passes
    // above
    if (!taylor && !hub && t->tab.T <= kJitTwoPassMaxTerms) {
        if (small) {
            kinds.push_back(kJitComplex);
        } else {
            kinds.push_back(kJitComplexSums);
            kinds.push_back(kJitComplexFreq);
        }
        if (t->tab.T <= kJitAutoComplexAdjointTerms) {
            kinds.push_back(kJitComplexAdj);
        } else {
            if (small) kinds.push_back(kJitComplexSums);
            kinds.push_back(kJitComplexAdjFreq);
            kinds.push_back(kJitComplexAdjLeaf);
        }
    }
    for (int k : kinds) {
        const AmiStatus st = jit_compile(t, hub, k);
        if (st != AMI_OK) return st;
    }
    for (int k : kinds) {
        void *fn = nullptr;
        const AmiStatus st = jit_get(t, hub, k, &fn);
        if (st != AMI_OK) return st;
    }
    return AMI_OK;
}

const char *amiLastVariant(void) { return ami::g_last_variant.c_str(); }

AmiStatus amiKernelTimerStart(int32_t capacity) {
    using namespace ami;
    clear_error();
    if (capacity < 1 || capacity > (1 << 20)) return fail(AMI_E_ARG, "capacity must be in 1..2^20");
    if (g_timer.on) return fail(AMI_E_ARG, "the kernel timer is already running on this thread");
    g_timer.ev.assign(2 * static_cast<size_t>(capacity), nullptr);
    for (size_t i = 0; i < g_timer.ev.size(); ++i) {
        const hipError_t e = hipEventCreate(&g_timer.ev[i]);
        if (e != hipSuccess) {
            for (size_t j = 0; j < i; ++j) (void)hipEventDestroy(g_timer.ev[j]);
            g_timer.ev.clear();
            return hip_fail(e, "hipEventCreate");
        }
    }
    g_timer.used = 0;
    g_timer.on = true;
    return AMI_OK;
}

AmiStatus amiKernelTimerStop(float *ms, int32_t cap, int32_t *count) {
    using namespace ami;
    clear_error();
    if (!g_timer.on) return fail(AMI_E_ARG, "the kernel timer is not running on this thread");
    AmiStatus st = AMI_OK;
    int n = 0;
    for (int i = 0; i < g_timer.used; ++i) {
        hipError_t e = hipEventSynchronize(g_timer.ev[2 * i + 1]);
        float v = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&v, g_timer.ev[2 * i], g_timer.ev[2 * i + 1]);
        if (e != hipSuccess) {
            st = hip_fail(e, "kernel timer events");
            break;
        }
        if (ms && n < cap) ms[n] = v;
        ++n;
    }
    for (hipEvent_t ev : g_timer.ev) (void)hipEventDestroy(ev);
    g_timer.ev.clear();
    g_timer.used = 0;
    g_timer.on = false;
    if (count) *count = n;
    return st;
}

}  // extern "C"
