// Persistent mixed-diagram batch: many diagrams of different order and term
// count, each with its own samples and frequency rows, evaluated by one
// persistent kernel launch that pulls (diagram, tile range) work items from a
// queue, replayed as one HIP graph (reset counter -> persistent kernel ->
// fixed-order row sums).
//
// Items are first split into LDS classes (the block size and the number of
// blocks per CU of their own packed launch), so that no item runs below the
// occupancy of its own launch: each class has its own block size, LDS size,
// grid, work queue and counter, and its persistent kernel is a graph node of
// its own between the counter reset and the row sums.  Within a class, work items are
// built on the host: a diagram's sample tiles are grouped so that every item
// costs about the same (a multiple, the tuning's tile factor, of the class's
// most expensive single tile, estimated from the solution's table sizes), and
// the items are queued from the most to the least expensive (largest-first
// list scheduling).  Each item is evaluated by the same tile
// function as the per-diagram kernel (fwd_tile), so every output value is
// bitwise the one the per-diagram launch computes; the row sums are reduced
// over the same tiles in the same order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include <thread>

#include "ami_internal.hpp"
#include "device_common.hpp"
#include "jit.hpp"
#include "kernels_packed.hpp"
#include "runtime.hpp"

namespace ami {

namespace {

// Shapes with their own instance in the batch kernel: self-energy order n
// (2n-1 energies, n leaves and n-1 denominators per term), n = 1..7, then the
// bounded generic instance (index 0).
constexpr int kShapeGeneric = 0;

struct BatchDesc {
    KArgs a;
    int32_t shape;
    int32_t pad;
};

struct Work {
    int32_t item;
    int32_t ntiles;
    int64_t tile0;
};

struct RowSumJob {
    const double *partial;   // [nblocks][ncols] of one item
    double *dst;             // one double of out_sum
    int64_t nblocks;
    int32_t ncols;
    int32_t col;
};

typedef const __attribute__((address_space(4))) BatchDesc *cdesc;
typedef const __attribute__((address_space(4))) Work *cwork;

// ALL: every shape; otherwise self-energy orders 1..6 only (fewer registers,
// chosen when every item of the batch has one of those shapes).
template <bool HUB, bool ALL>
__device__ __forceinline__ void run_item(const KArgs &a, int shape, int64_t tile0, int ntiles, double *sm) {
    for (int64_t tile = tile0; tile < tile0 + ntiles; ++tile) {
        switch (shape) {
        case 1: fwd_tile<1, 1, 0, true, HUB>(a, tile, sm); break;
        case 2: fwd_tile<3, 2, 1, true, HUB>(a, tile, sm); break;
        case 3: fwd_tile<5, 3, 2, true, HUB>(a, tile, sm); break;
        case 4: fwd_tile<7, 4, 3, true, HUB>(a, tile, sm); break;
        case 5: fwd_tile<9, 5, 4, true, HUB>(a, tile, sm); break;
        case 6: fwd_tile<11, 6, 5, true, HUB>(a, tile, sm); break;
        default:
            if constexpr (ALL) {
                if (shape == 7) fwd_tile<13, 7, 6, true, HUB>(a, tile, sm);
                else fwd_tile<16, 8, 8, false, HUB>(a, tile, sm);
            }
            break;
        }
        __syncthreads();   // the next tile reuses the LDS columns
    }
}

// Every block takes work items from the counter until the queue is empty;
// each block sees the counter pass n_work, so every wave exits.
template <bool HUB, bool ALL>
__global__ __launch_bounds__(256) void ami_batch_kernel(const BatchDesc *desc, const Work *work, int n_work,
                                                        unsigned int *counter) {
    extern __shared__ double sm[];
    __shared__ int next;
    cdesc cd = (cdesc)(desc);
    cwork cw = (cwork)(work);
    for (;;) {
        if (threadIdx.x == 0) next = static_cast<int>(atomicAdd(counter, 1u));
        __syncthreads();
        const int wi = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        if (wi >= n_work) break;
        const int item = cw[wi].item;
        const int ntiles = cw[wi].ntiles;
        const int64_t tile0 = cw[wi].tile0;
        // fields are read on demand through the constant address space
        const KArgs &a = *(const KArgs *)((const void *)&cd[item].a);
        run_item<HUB, ALL>(a, cd[item].shape, tile0, ntiles, sm);
    }
}

// counters are kCounterStride apart (one per class or work list)
constexpr int kCounterStride = kBatchCounterStride;
constexpr int kMaxClasses = 16;

__global__ void ami_batch_reset_kernel(unsigned int *counters, int n) {
    if (blockIdx.x == 0 && static_cast<int>(threadIdx.x) < n) counters[threadIdx.x * kCounterStride] = 0u;
}

__global__ __launch_bounds__(256) void ami_batch_rowsum_kernel(const RowSumJob *jobs) {
    __shared__ double sh[256];
    const RowSumJob j = jobs[blockIdx.x];
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int64_t b = tid; b < j.nblocks; b += 256) acc += j.partial[b * j.ncols + j.col];
    sh[tid] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    if (tid == 0) *j.dst = sh[0];
}

// Cost of one sample of an item: leaves and term products once, denominators
// and group products per frequency row (relative units).
double sample_cost(const AmiTerms *t, int64_t n_f) {
    const Tables &tb = t->tab;
    const double per_sample = 50.0 * tb.L + (t->n_int + 1.0) * tb.T + 44.0 * 2 * t->n_g;
    const double per_point = 30.0 * tb.D + (6.0 * std::max(tb.dpt - 1, 0) + 4.0) * tb.G;
    return per_sample + per_point * static_cast<double>(n_f);
}

int shape_of(const AmiTerms *t, bool hub) {
    const int ne = t->n_eps, ni = t->n_int, dpt = t->tab.dpt;
    const bool se = (ne == 2 * ni - 1) && (dpt == ni - 1) && (!hub || t->n_g == ne);
    return (se && ni >= 1 && ni <= 7) ? ni : kShapeGeneric;
}

}  // namespace

}  // namespace ami

struct AmiBatch {
    int device = -1;
    bool hub = false;
    int n_items = 0;
    int n_classes = 0;
    int block = 0;                         // of the class with the most work
    int grid = 0;                          // summed over the classes
    size_t lds = 0;                        // largest over the classes
    int64_t n_work = 0;
    int64_t n_jobs = 0;
    int n_spec = 0;                        // items on their specialized kernels
    int n_streams = 0;                     // streams their launches were captured from
    hipStream_t streams[4] = {};           // kept until the batch is freed (their workspaces)
    void *blob = nullptr;                  // descriptors, work list, jobs, counter, partial sums
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipModule_t> modules;      // persistent specialized batch: its compiled groups
};

namespace ami {
namespace {

AmiStatus batch_fail_free(AmiBatch *b, AmiStatus st);

// The items on their specialized kernels: each item's forward (as an AUTO
// evaluate call launches it, row sums included) recorded from up to four
// streams -- items assigned largest first to the least loaded stream, so
// small diagrams run side by side -- into a graph added to the batch graph as
// a child node beside the persistent kernels.  One eager run first sizes the
// items' per-stream workspaces and loads their kernels, so the recorded
// launches allocate nothing; the streams stay with the batch (its items'
// workspaces are keyed by them).
AmiStatus capture_specialized(AmiBatch *b, const AmiBatchItem *items, const std::vector<char> &spec, bool hub) {
    std::vector<int> ids;
    for (size_t i = 0; i < spec.size(); ++i)
        if (spec[i]) ids.push_back(static_cast<int>(i));
    std::vector<double> cost(spec.size(), 0.0);
    for (int i : ids) cost[i] = sample_cost(items[i].terms, items[i].n_f) * static_cast<double>(items[i].n_e);
    std::stable_sort(ids.begin(), ids.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    b->n_streams = std::min<int>(4, static_cast<int>(ids.size()));
    for (int k = 0; k < b->n_streams; ++k) {
        const hipError_t e = hipStreamCreateWithFlags(&b->streams[k], hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    }
    std::vector<int> stream_of(spec.size(), 0);
    std::vector<double> load(b->n_streams, 0.0);
    for (int i : ids) {
        const int k = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
        stream_of[i] = k;
        load[k] += cost[i];
    }
    auto launch_all = [&]() -> AmiStatus {
        for (int i : ids) {
            const AmiBatchItem &it = items[i];
            KArgs a;
            std::memset(&a, 0, sizeof(a));
            set_inputs(a, it.terms, it.k, it.stride_k, it.q, it.t, it.mu, it.energies, it.stride_s, it.stride_i,
                       it.ext_freqs, it.n_f, it.beta, it.e_reg, it.n_e);
            a.out = it.out;
            const AmiStatus st = launch_forward_as(it.terms, hub, a, it.out_sum, b->streams[stream_of[i]],
                                                   AMI_VARIANT_AUTO);
            if (st != AMI_OK) return st;
        }
        return AMI_OK;
    };
    AmiStatus st = launch_all();   // eager: workspaces sized, kernels loaded
    for (int k = 0; k < b->n_streams && st == AMI_OK; ++k) {
        const hipError_t e = hipStreamSynchronize(b->streams[k]);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    if (st != AMI_OK) return st;
    hipEvent_t ev[5] = {};
    for (int k = 0; k <= b->n_streams; ++k) {
        const hipError_t e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
        if (e != hipSuccess) {
            for (int j = 0; j < k; ++j) (void)hipEventDestroy(ev[j]);
            return hip_fail(e, "hipEventCreateWithFlags");
        }
    }
    hipStream_t s0 = b->streams[0];
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s0, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        e = hipEventRecord(ev[0], s0);                                  // fork
        for (int k = 1; k < b->n_streams && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->streams[k], ev[0], 0);
        if (e == hipSuccess) st = launch_all();
        for (int k = 1; k < b->n_streams && e == hipSuccess; ++k) {   // join
            e = hipEventRecord(ev[k], b->streams[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s0, ev[k], 0);
        }
        const hipError_t e2 = hipStreamEndCapture(s0, &g);                // always ends the capture
        if (e == hipSuccess) e = e2;
    }
    for (int k = 0; k <= b->n_streams; ++k) (void)hipEventDestroy(ev[k]);
    if (e == hipSuccess && st == AMI_OK) {
        hipGraphNode_t node = nullptr;
        e = hipGraphAddChildGraphNode(&node, b->graph, nullptr, 0, g);
    }
    if (g) (void)hipGraphDestroy(g);
    if (st != AMI_OK) return st;
    return e == hipSuccess ? AMI_OK : hip_fail(e, "capture of the specialized items");
}

AmiStatus batch_fail_free(AmiBatch *b, AmiStatus st) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->blob) (void)hipFree(b->blob);
    for (hipModule_t m : b->modules) (void)hipModuleUnload(m);
    for (int k = 0; k < b->n_streams; ++k)
        if (b->streams[k]) (void)hipStreamDestroy(b->streams[k]);
    delete b;
    return st;
}

// Row sums of the persistent specialized batch: per item and column, the
// column's per-wave partial sums reduced by column_sum, the routine (and
// block size) of the per-diagram row-sum kernel, so out_sum is bitwise the
// per-diagram call's.
struct ColJob {
    const double *col;
    double *dst;
    int64_t rows;
};

__global__ __launch_bounds__(kRedThreads) void ami_batch_colsum_kernel(const ColJob *jobs) {
    __shared__ double sh[kRedThreads / 64];
    const ColJob j = jobs[blockIdx.x];
    const double r = column_sum(j.col, j.rows, 1, sh);
    if (threadIdx.x == 0) *j.dst = r;
}

// Work item of the persistent specialized kernels (the layout of
// amibatch::Work in the generated source).
struct SpecWork {
    int32_t item, ntiles;
    int64_t tile0;
    int32_t f, nf;
};

// Terms per compiled group of the persistent specialized batch (groups are
// compiled side by side; one group per occupancy class below this bound).
constexpr int64_t kSpecGroupTerms = 16000;
constexpr int kSpecBlock = 256;

// The persistent specialized batch (tuning.kernels = 2): every item runs its
// own generated tile functions inside persistent kernels.  Per pass (the
// one-pass tiles with the two-pass items' first pass, then the two-pass
// items' frequency pass) the items are grouped by the occupancy (VGPRs) of
// their own kernel of that pass, groups cut at about kSpecGroupTerms terms;
// each group is one module compiled at run time whose kernel pulls work items
// from its own counter.  The graph: counter reset -> every first-pass kernel
// (side by side) -> every frequency-pass kernel -> row sums.
AmiStatus create_spec_persistent(const AmiBatchItem *items, int n_items, const AmiBatchTuning &tun, bool hub,
                                 int dev, AmiBatch **out) {
    int n_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    const int B = kSpecBlock;
    // per item: one or two passes (as AUTO), and the occupancy (waves per
    // SIMD) of its own kernel of each pass: the forward, or the first and the
    // frequency pass
    std::vector<int> two(n_items, 0), waves1(n_items, 8), waves2(n_items, 8);
    std::vector<int64_t> tiles(n_items, 0);
    auto waves_of = [&](AmiTerms *t, int kind, int &w) -> AmiStatus {
        void *fn = nullptr;
        AmiStatus st = jit_get(t, hub, kind, &fn);
        if (st != AMI_OK) return st;
        int r = 0;
        const hipError_t e2 = hipFuncGetAttribute(&r, HIP_FUNC_ATTRIBUTE_NUM_REGS, static_cast<hipFunction_t>(fn));
        if (e2 != hipSuccess) return hip_fail(e2, "hipFuncGetAttribute");
        w = std::max(1, std::min(8, 512 / std::max(8, (r + 7) / 8 * 8)));
        return AMI_OK;
    };
    for (int i = 0; i < n_items; ++i) {
        AmiTerms *t = items[i].terms;
        if (!specialized_forward_ready(t, hub, static_cast<int>(items[i].n_f)))
            return fail(AMI_E_UNSUPPORTED, "item " + std::to_string(i) + ": no specialized forward");
        two[i] = jit_prefers_two_pass(t) ? 1 : 0;
        if (two[i] && items[i].n_f > 65535) return fail(AMI_E_UNSUPPORTED, "more than 65535 frequency rows");
        AmiStatus st = waves_of(t, two[i] ? kJitSumsPass : kJitForward, waves1[i]);
        if (st == AMI_OK && two[i]) st = waves_of(t, kJitFreqPass, waves2[i]);
        if (st != AMI_OK) return st;
        tiles[i] = (items[i].n_e + B - 1) / B;
    }
    std::vector<double> cost(n_items);
    for (int i = 0; i < n_items; ++i) cost[i] = sample_cost(items[i].terms, items[i].n_f) * items[i].n_e;
    // kernel groups: per pass, the items by the occupancy of their own kernel
    // of that pass (most waves first, then by cost), cut at kSpecGroupTerms
    // terms; a group's kernel runs at the occupancy its own code allows.  In
    // the first pass the two-pass items' groups come first and hold no
    // one-pass item, so that their frequency passes wait for them alone.
    struct KGroup {
        int pass;
        std::vector<int> items;
    };
    std::vector<KGroup> groups;
    for (int pass = 1; pass <= 2; ++pass) {
        const std::vector<int> &wv = pass == 1 ? waves1 : waves2;
        std::vector<int> order;
        for (int i = 0; i < n_items; ++i)
            if (pass == 1 || two[i]) order.push_back(i);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            if (pass == 1 && two[x] != two[y]) return two[x] > two[y];
            return wv[x] != wv[y] ? wv[x] > wv[y] : cost[x] > cost[y];
        });
        int64_t terms_in = 0;
        bool fresh = true;
        for (int i : order) {
            const int64_t T = items[i].terms->tab.T;
            const int head = fresh ? -1 : groups.back().items[0];
            if (fresh || wv[head] != wv[i] || two[head] != two[i] || terms_in + T > kSpecGroupTerms) {
                groups.push_back(KGroup{pass, {}});
                terms_in = 0;
                fresh = false;
            }
            groups.back().items.push_back(i);
            terms_in += T;
        }
    }
    // generated sources, compiled side by side (no device needed), then loaded
    const size_t G = groups.size();
    std::vector<std::string> srcs(G), forced(G), plain(G), errs(G);
    std::vector<int> own(G, 1);
    std::vector<std::vector<char>> codes(G);
    std::vector<AmiStatus> sts(G, AMI_OK);
    for (size_t g = 0; g < G; ++g) {
        std::vector<const AmiTerms *> ts;
        std::vector<int> tp, one, labels;
        for (int i : groups[g].items) {
            ts.push_back(items[i].terms);
            tp.push_back(two[i]);
            one.push_back(items[i].n_f == 1 ? 1 : 0);
            labels.push_back(i);
        }
        own[g] = (groups[g].pass == 1 ? waves1 : waves2)[groups[g].items[0]];
        srcs[g] = jit_batch_source(ts, tp, one, hub, B, groups[g].pass, labels, true, 0);
        forced[g] = jit_batch_source(ts, tp, one, hub, B, groups[g].pass, labels, true, own[g]);
        plain[g] = jit_batch_source(ts, tp, one, hub, B, groups[g].pass, labels, false, 0);
    }
    {
        // a group's kernel as it compiles, claiming work ahead, where that
        // keeps the occupancy of its items' own kernels of the pass (read from
        // the compiled code's metadata); else compiled for that occupancy,
        // where that spills nothing; else without the claim ahead, where that
        // keeps more waves
        auto waves_meta = [](const std::vector<char> &code) {
            const int64_t v = code_meta(code, ".vgpr_count");
            return v <= 0 ? int64_t(0) : std::min<int64_t>(8, 512 / ((v + 7) / 8 * 8));
        };
        std::vector<std::thread> pool;
        std::atomic<size_t> next{0};
        const unsigned n_thr = std::max(1u, std::min<unsigned>(8u, static_cast<unsigned>(G)));
        for (unsigned k = 0; k < n_thr; ++k)
            pool.emplace_back([&]() {
                for (size_t g = next++; g < G; g = next++) {
                    sts[g] = code_from_source(srcs[g], codes[g], errs[g]);
                    if (sts[g] != AMI_OK || waves_meta(codes[g]) >= own[g]) continue;
                    std::vector<char> alt;
                    std::string alt_err;
                    if (code_from_source(forced[g], alt, alt_err) == AMI_OK && waves_meta(alt) >= own[g] &&
                        code_meta(alt, ".private_segment_fixed_size") == 0) {
                        codes[g].swap(alt);
                        continue;
                    }
                    alt.clear();
                    if (code_from_source(plain[g], alt, alt_err) == AMI_OK && waves_meta(alt) > waves_meta(codes[g]))
                        codes[g].swap(alt);
                }
            });
        for (auto &th : pool) th.join();
    }
    for (size_t g = 0; g < G; ++g)
        if (sts[g] != AMI_OK) return fail(sts[g], "persistent batch group " + std::to_string(g) + ": " + errs[g]);

    AmiBatch *b = new (std::nothrow) AmiBatch();
    if (!b) return fail(AMI_E_OOM, "out of host memory");
    b->device = dev;
    b->hub = hub;
    b->n_items = n_items;
    b->n_spec = n_items;
    b->block = B;
    std::vector<hipFunction_t> kfn(G, nullptr);
    for (size_t g = 0; g < G; ++g) {
        hipModule_t m = nullptr;
        e = hipModuleLoadData(&m, codes[g].data());
        if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "hipModuleLoadData (persistent batch)"));
        b->modules.push_back(m);
        const char *name = groups[g].pass == 1 ? "ami_batch_p1" : "ami_batch_p2";
        e = hipModuleGetFunction(&kfn[g], m, name);
        if (e != hipSuccess) return batch_fail_free(b, fail(AMI_E_HIP, std::string("hipModuleGetFunction ") + name));
    }

    // resident blocks per CU of each group's kernel, from its own VGPRs (one
    // wave of each block per SIMD), capped by the tuning
    std::vector<int> per_cu(G, 1);
    for (size_t g = 0; g < G; ++g) {
        int regs = 0;
        e = hipFuncGetAttribute(&regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, kfn[g]);
        if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "hipFuncGetAttribute"));
        const int gw = std::max(1, std::min(8, 512 / std::max(8, (regs + 7) / 8 * 8)));
        per_cu[g] = std::max(1, std::min(gw, tun.waves_per_cu / (B / 64)));
    }

    // work lists: per group, each item's tiles (and, in the frequency pass,
    // rows) in work items of about tile_factor times the group's most
    // expensive unit -- a tile, or a tile at one row -- but no larger than a
    // quarter of the group's work per resident block, so that a list has work
    // for every block and its tail stays short; the items from the most to
    // the least expensive with their work items together (a CU then mostly
    // runs one item's code at a time); in the frequency pass a work item is a
    // tile range at a range of rows, the rows of a tile range queued one
    // after another
    std::vector<double> tile_cost(n_items);
    for (int i = 0; i < n_items; ++i) tile_cost[i] = sample_cost(items[i].terms, items[i].n_f) * B;
    // Each group's work goes into eight lists, one per XCD: a unit (an
    // item's tile range with all its frequency rows in the second pass) goes
    // to the list with the least cost so far, so the rows of a tile read its
    // stored group sums through one XCD's L2.
    std::vector<SpecWork> wl;
    std::vector<int64_t> w0(G, 0), nw(G, 0);
    std::vector<int> xoffs(G * 9, 0);
    for (size_t g = 0; g < G; ++g) {
        const int pass = groups[g].pass;
        // pass 1 of a two-pass item: leaves and group sums only (about a
        // fifth of its tile's cost); pass 2: one frequency row
        auto unit = [&](int i) {
            return !two[i] ? tile_cost[i] : pass == 1 ? tile_cost[i] / 5 : tile_cost[i] / items[i].n_f;
        };
        auto rows_of = [&](int i) { return pass == 2 ? static_cast<int64_t>(items[i].n_f) : int64_t(1); };
        double max_unit = 0.0, total = 0.0;
        for (int i : groups[g].items) {
            max_unit = std::max(max_unit, unit(i));
            total += unit(i) * static_cast<double>(tiles[i] * rows_of(i));
        }
        const double slots = static_cast<double>(n_cu) * per_cu[g];
        const double target = std::min(max_unit * tun.tile_factor, total / (4.0 * slots));
        std::vector<int> by_cost = groups[g].items;
        std::stable_sort(by_cost.begin(), by_cost.end(), [&](int x, int y) { return cost[x] > cost[y]; });
        w0[g] = static_cast<int64_t>(wl.size());
        std::vector<SpecWork> lists[8];
        double load[8] = {0.0};
        for (int i : by_cost) {
            // units per work item: rows first, then whole tiles of all rows
            const int64_t per = std::max<int64_t>(1, static_cast<int64_t>(target / unit(i)));
            const int64_t rows = rows_of(i);
            const int64_t nr = std::min(per, rows);
            const int64_t per_t = nr < rows ? 1 : std::max<int64_t>(1, per / rows);
            for (int64_t t0 = 0; t0 < tiles[i]; t0 += per_t) {
                const int64_t nt = std::min<int64_t>(per_t, tiles[i] - t0);
                const int x = static_cast<int>(std::min_element(load, load + 8) - load);
                load[x] += unit(i) * static_cast<double>(nt * rows);
                for (int64_t f0 = 0; f0 < rows; f0 += nr) {
                    SpecWork w;
                    std::memset(&w, 0, sizeof(w));
                    w.item = i;
                    w.tile0 = t0;
                    w.ntiles = static_cast<int32_t>(nt);
                    w.f = pass == 2 ? static_cast<int32_t>(f0) : -1;
                    w.nf = pass == 2 ? static_cast<int32_t>(std::min(nr, rows - f0)) : 0;
                    lists[x].push_back(w);
                }
            }
        }
        for (int x = 0; x < 8; ++x) {
            xoffs[g * 9 + x] = static_cast<int>(static_cast<int64_t>(wl.size()) - w0[g]);
            wl.insert(wl.end(), lists[x].begin(), lists[x].end());
        }
        nw[g] = static_cast<int64_t>(wl.size()) - w0[g];
        xoffs[g * 9 + 8] = static_cast<int>(nw[g]);
    }
    if (wl.size() > 0x7fffffffu - 65536u) return batch_fail_free(b, fail(AMI_E_ARG, "too many work items"));

    // one allocation: argument blocks (item order) | work |
    // column jobs | counters | per-wave partial sums | two-pass workspaces
    std::vector<int64_t> rows(n_items), part_off(n_items, -1), ws_off(n_items, -1), ld(n_items, 0);
    int64_t part_total = 0, ws_total = 0, n_jobs = 0;
    for (int i = 0; i < n_items; ++i) {
        rows[i] = tiles[i] * (B / 64);
        if (items[i].out_sum) {
            part_off[i] = part_total;
            part_total += rows[i] * 2 * items[i].n_f;
            n_jobs += 2 * items[i].n_f;
        }
        if (two[i]) {
            ld[i] = tiles[i] * B;
            ws_off[i] = ws_total;
            ws_total += (static_cast<int64_t>(items[i].terms->tab.G) + items[i].terms->n_eps) * ld[i];
        }
    }
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t sz_args = sizeof(KArgs) * n_items;
    const size_t off_work = al(sz_args);
    const size_t off_xoff = al(off_work + sizeof(SpecWork) * std::max<size_t>(wl.size(), 1));
    const size_t off_jobs = al(off_xoff + sizeof(int) * xoffs.size());
    const size_t off_ctr = al(off_jobs + sizeof(ColJob) * std::max<int64_t>(n_jobs, 1));
    const size_t off_part = al(off_ctr + sizeof(unsigned int) * kCounterStride * 8 * G);
    const size_t off_ws = al(off_part + sizeof(double) * std::max<int64_t>(part_total, 1));
    const size_t total = off_ws + sizeof(double) * std::max<int64_t>(ws_total, 1);
    e = hipMalloc(&b->blob, total);
    if (e != hipSuccess) return batch_fail_free(b, fail(AMI_E_OOM, "persistent batch workspace"));
    unsigned char *base = static_cast<unsigned char *>(b->blob);
    double *partial = reinterpret_cast<double *>(base + off_part);
    double *wsp = reinterpret_cast<double *>(base + off_ws);
    std::vector<KArgs> args(n_items);
    std::vector<ColJob> jobs;
    for (int i = 0; i < n_items; ++i) {
        const AmiBatchItem &it = items[i];
        KArgs &a = args[i];
        std::memset(&a, 0, sizeof(a));
        set_inputs(a, it.terms, it.k, it.stride_k, it.q, it.t, it.mu, it.energies, it.stride_s, it.stride_i,
                   it.ext_freqs, it.n_f, it.beta, it.e_reg, it.n_e);
        a.out = it.out;
        a.nrows = rows[i];
        a.partial = it.out_sum ? partial + part_off[i] : nullptr;
        if (two[i]) {
            a.work = wsp + ws_off[i];
            a.ld = ld[i];
            a.s0 = 0;
            a.n_chunk = it.n_e;
        }
        if (it.out_sum)
            for (int c = 0; c < 2 * it.n_f; ++c) jobs.push_back(ColJob{partial + part_off[i] + c * rows[i], it.out_sum + c, rows[i]});
        if (two[i] && ld[i] > (int64_t(1) << 28))
            return batch_fail_free(b, fail(AMI_E_ARG, "item " + std::to_string(i) + ": more than 2^28 samples in two passes"));
    }
    // work items name their item; the kernels index the argument blocks by it
    std::vector<unsigned char> host(off_part, 0);
    std::memcpy(host.data(), args.data(), sz_args);
    if (!wl.empty()) std::memcpy(host.data() + off_work, wl.data(), sizeof(SpecWork) * wl.size());
    std::memcpy(host.data() + off_xoff, xoffs.data(), sizeof(int) * xoffs.size());
    if (!jobs.empty()) std::memcpy(host.data() + off_jobs, jobs.data(), sizeof(ColJob) * jobs.size());
    e = hipMemcpy(b->blob, host.data(), off_part, hipMemcpyHostToDevice);
    if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "persistent batch upload"));
    b->n_work = static_cast<int64_t>(wl.size());
    b->n_jobs = n_jobs;
    b->n_classes = static_cast<int>(G);

    // graph
    e = hipGraphCreate(&b->graph, 0);
    if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "hipGraphCreate"));
    unsigned int *d_ctr = reinterpret_cast<unsigned int *>(base + off_ctr);
    hipGraphNode_t n_reset = nullptr;
    {
        if (8 * G > 1024) return batch_fail_free(b, fail(AMI_E_ARG, "too many groups"));
        int n_ctr = static_cast<int>(8 * G);     // eight per group, one per work list
        void *kp[] = {&d_ctr, &n_ctr};
        hipKernelNodeParams p;
        std::memset(&p, 0, sizeof(p));
        p.func = reinterpret_cast<void *>(&ami_batch_reset_kernel);
        p.gridDim = dim3(1);
        p.blockDim = dim3(static_cast<unsigned>(std::max<size_t>(64, (8 * G + 63) / 64 * 64)));
        p.kernelParams = kp;
        e = hipGraphAddKernelNode(&n_reset, b->graph, nullptr, 0, &p);
        if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "graph reset node"));
    }
    // every first-pass kernel after the reset, side by side; each frequency-
    // pass kernel after the first-pass kernels that hold its items' first
    // passes; the row sums after everything
    std::vector<hipGraphNode_t> first_of(static_cast<size_t>(n_items), nullptr), all;
    for (int pass = 1; pass <= 2; ++pass)
        for (size_t g = 0; g < G; ++g) {
            if (groups[g].pass != pass || nw[g] == 0) continue;
            const KArgs *d_args = reinterpret_cast<const KArgs *>(base);
            const SpecWork *d_work = reinterpret_cast<const SpecWork *>(base + off_work) + w0[g];
            const int *d_xoff = reinterpret_cast<const int *>(base + off_xoff) + g * 9;
            unsigned int *ctr = d_ctr + g * 8 * kCounterStride;
            void *kp[] = {&d_args, &d_work, &d_xoff, &ctr};
            hipKernelNodeParams p;
            std::memset(&p, 0, sizeof(p));
            p.func = reinterpret_cast<void *>(kfn[g]);
            p.gridDim = dim3(static_cast<unsigned>(std::min<int64_t>(static_cast<int64_t>(n_cu) * per_cu[g], nw[g])));
            p.blockDim = dim3(B);
            p.kernelParams = kp;
            hipGraphNode_t node = nullptr;
            std::vector<hipGraphNode_t> deps;
            if (pass == 1) {
                deps.push_back(n_reset);
            } else {
                for (int i : groups[g].items)
                    if (first_of[i] && std::find(deps.begin(), deps.end(), first_of[i]) == deps.end())
                        deps.push_back(first_of[i]);
                if (deps.empty()) deps.push_back(n_reset);
            }
            e = hipGraphAddKernelNode(&node, b->graph, deps.data(), deps.size(), &p);
            if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "graph persistent node"));
            if (pass == 1)
                for (int i : groups[g].items) first_of[i] = node;
            all.push_back(node);
            b->grid += static_cast<int>(p.gridDim.x);
        }
    std::vector<hipGraphNode_t> &last = all;
    if (n_jobs > 0) {
        const ColJob *d_jobs = reinterpret_cast<const ColJob *>(base + off_jobs);
        void *kp[] = {&d_jobs};
        hipKernelNodeParams p;
        std::memset(&p, 0, sizeof(p));
        p.func = reinterpret_cast<void *>(&ami_batch_colsum_kernel);
        p.gridDim = dim3(static_cast<unsigned>(n_jobs));
        p.blockDim = dim3(kRedThreads);
        p.kernelParams = kp;
        hipGraphNode_t node = nullptr;
        e = hipGraphAddKernelNode(&node, b->graph, last.data(), last.size(), &p);
        if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "graph row-sum node"));
    }
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "hipGraphInstantiate"));
    *out = b;
    return AMI_OK;
}

}  // namespace
}  // namespace ami

extern "C" {

AmiStatus amiBatchCreate(const AmiBatchItem *items, int32_t n_items, const AmiBatchTuning *tuning,
                         AmiBatch **out) {
    using namespace ami;
    clear_error();
    if (!out) return fail(AMI_E_ARG, "out is NULL");
    *out = nullptr;
    if (!items || n_items < 1) return fail(AMI_E_ARG, "no items");
    AmiBatchTuning tun = {0, 8, 1, 0};
    if (tuning) tun = *tuning;
    if (tun.waves_per_cu < 1 || tun.waves_per_cu > 32) return fail(AMI_E_ARG, "waves_per_cu must be in 1..32");
    if (tun.tile_factor < 1 || tun.tile_factor > 1024) return fail(AMI_E_ARG, "tile_factor must be in 1..1024");
    if (tun.block != 0 && tun.block != 64 && tun.block != 128 && tun.block != 256)
        return fail(AMI_E_ARG, "block must be 0 (automatic), 64, 128 or 256");
    if (tun.kernels < 0 || tun.kernels > 2) return fail(AMI_E_ARG, "kernels must be 0, 1 or 2");
    const bool hub = items[0].k != nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");

    // per-item checks and descriptors; with kernels = 0 an item whose
    // specialized forward AUTO would run takes it (compiled and loaded here)
    std::vector<BatchDesc> desc(n_items);
    std::vector<char> spec(n_items, 0);
    for (int i = 0; i < n_items; ++i) {
        const AmiBatchItem &it = items[i];
        AmiTerms *t = it.terms;
        if (!t) return fail(AMI_E_ARG, "item " + std::to_string(i) + ": terms is NULL");
        if ((it.k != nullptr) != hub)
            return fail(AMI_E_ARG, "all items must use the same path (momenta or energies)");
        if (t->n_eps > kMaxEpsDev || t->n_ext > kMaxExt) return fail(AMI_E_UNSUPPORTED, "item shape too large");
        if (it.n_e < 1) return fail(AMI_E_ARG, "item " + std::to_string(i) + ": n_e must be >= 1");
        if (it.n_f < 1 || it.n_f > (1 << 24)) return fail(AMI_E_ARG, "n_f must be in 1..2^24");
        if (!(it.beta > 0.0)) return fail(AMI_E_ARG, "beta must be > 0");
        if (!it.out && !it.out_sum) return fail(AMI_E_ARG, "item " + std::to_string(i) + ": no output");
        if (t->n_ext > 0 && !it.ext_freqs) return fail(AMI_E_ARG, "ext_freqs is NULL");
        if (hub) {
            if (t->n_eps != t->n_g) return fail(AMI_E_ARG, "the momentum path needs one energy per propagator");
            if (it.stride_k < 2 * t->n_int) return fail(AMI_E_ARG, "stride_k < 2*n_int");
        } else {
            if (!it.energies || it.stride_s < 1 || it.stride_i < 1) return fail(AMI_E_ARG, "bad energies");
        }
        DeviceTables *dt = nullptr;
        AmiStatus st = upload(t, &dt);
        if (st != AMI_OK) return st;
        if (tun.kernels == 2) continue;
        spec[i] = tun.kernels == 0 && specialized_forward_ready(t, hub, static_cast<int>(it.n_f));
        if (!spec[i] && !t->tab.packable)
            return fail(AMI_E_UNSUPPORTED, "item " + std::to_string(i) + ": no specialized kernel and not in packed form");
        BatchDesc &d = desc[i];
        std::memset(&d, 0, sizeof(d));
        d.a.tb = packed_tabs(t, dt);
        d.a.energies = it.energies;
        d.a.stride_s = it.stride_s;
        d.a.stride_i = it.stride_i;
        d.a.k = it.k;
        d.a.stride_k = it.stride_k;
        for (int x = 0; x < t->n_ext && x < kMaxExtDev; ++x) {
            d.a.q[2 * x] = std::remainder(it.q[2 * x], 2.0 * M_PI);
            d.a.q[2 * x + 1] = std::remainder(it.q[2 * x + 1], 2.0 * M_PI);
        }
        d.a.hop_t = it.t;
        d.a.mu = it.mu;
        d.a.ext_freqs = it.ext_freqs;
        d.a.n_f = static_cast<int>(it.n_f);
        d.a.beta = it.beta;
        d.a.e_reg = it.e_reg;
        d.a.n_e = it.n_e;
        d.a.out = it.out;
        d.shape = shape_of(t, hub);
    }
    if (tun.kernels == 2) return create_spec_persistent(items, n_items, tun, hub, dev, out);
    int max_lds = 0, cu_lds = 0, n_cu = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    if (cu_lds < max_lds) cu_lds = max_lds;

    // LDS classes: items with the launch shape (block, LDS) the packed
    // per-diagram call picks, grouped by (block, resident blocks per CU), so
    // that every item runs at the occupancy of its own launch; classes in
    // order of per-lane LDS need, the last one taking the rest past kMaxClasses
    std::vector<int> order;
    std::vector<int> slots(n_items, 0);
    std::vector<LaunchShape> own(n_items);
    for (int i = 0; i < n_items; ++i) {
        if (spec[i]) continue;
        order.push_back(i);
        slots[i] = fwd_slots(items[i].terms->tab);
        AmiStatus st = pick_shape(slots[i], own[i]);
        if (st != AMI_OK) return st;
        if (tun.block != 0) {
            own[i].block = tun.block;
            own[i].lds = static_cast<size_t>(slots[i]) * sizeof(double) * tun.block +
                         2 * sizeof(double) * (tun.block / 64);
        }
    }
    auto resident = [&](size_t lds) { return static_cast<int>(cu_lds / (lds + 64)); };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return slots[x] < slots[y]; });
    struct Class {
        std::vector<int> items;
        int max_slots = 0;
        LaunchShape ls;
        int grid = 0;
        int64_t work0 = 0, n_work = 0;
    };
    std::vector<Class> cls;
    for (int i : order) {
        const bool same = !cls.empty() && own[cls.back().items[0]].block == own[i].block &&
                          resident(own[cls.back().items[0]].lds) == resident(own[i].lds);
        if (cls.empty() || (!same && static_cast<int>(cls.size()) < kMaxClasses)) cls.emplace_back();
        cls.back().items.push_back(i);
        cls.back().max_slots = std::max(cls.back().max_slots, slots[i]);
    }
    std::vector<int> cls_of(n_items, -1);
    for (size_t c = 0; c < cls.size(); ++c) {
        Class &k = cls[c];
        for (int i : k.items) cls_of[i] = static_cast<int>(c);
        k.ls.block = own[k.items[0]].block;
        for (int i : k.items) k.ls.block = std::min(k.ls.block, own[i].block);   // merged tail classes
        k.ls.slots = k.max_slots;
        k.ls.lds = static_cast<size_t>(k.max_slots) * sizeof(double) * k.ls.block +
                   2 * sizeof(double) * (k.ls.block / 64);
        if (k.ls.lds + 64 > static_cast<size_t>(max_lds))     // the kernel's own queue slot
            return fail(AMI_E_UNSUPPORTED, "batch items too large for the LDS of one block");
        for (int i : k.items) desc[i].a.slots = k.max_slots;
    }

    // work items per class and row-sum jobs
    std::vector<double> tile_cost(n_items, 0.0);
    std::vector<int64_t> tiles(n_items, 0);
    for (int i = 0; i < n_items; ++i) {
        if (spec[i]) continue;
        const int blk = cls[cls_of[i]].ls.block;
        tiles[i] = (items[i].n_e + blk - 1) / blk;
        tile_cost[i] = sample_cost(items[i].terms, items[i].n_f) * blk;
    }
    struct HostWork {
        Work w;
        double cost;
    };
    std::vector<Work> wl;
    size_t partial_total = 0;
    std::vector<size_t> partial_off(n_items, 0);
    for (int i = 0; i < n_items; ++i)
        if (items[i].out_sum && !spec[i]) {
            partial_off[i] = partial_total;
            partial_total += static_cast<size_t>(tiles[i]) * items[i].n_f * 2;
        }
    for (Class &k : cls) {
        double max_tile = 0.0;
        for (int i : k.items) max_tile = std::max(max_tile, tile_cost[i]);
        const double target = max_tile * tun.tile_factor;
        std::vector<HostWork> hw;
        for (int i : k.items) {
            const int64_t per = std::max<int64_t>(1, static_cast<int64_t>(target / tile_cost[i]));
            for (int64_t t0 = 0; t0 < tiles[i]; t0 += per) {
                HostWork h;
                h.w.item = i;
                h.w.tile0 = t0;
                h.w.ntiles = static_cast<int32_t>(std::min<int64_t>(per, tiles[i] - t0));
                h.cost = tile_cost[i] * h.w.ntiles;
                hw.push_back(h);
            }
        }
        std::stable_sort(hw.begin(), hw.end(), [](const HostWork &x, const HostWork &y) { return x.cost > y.cost; });
        k.work0 = static_cast<int64_t>(wl.size());
        k.n_work = static_cast<int64_t>(hw.size());
        for (const auto &h : hw) wl.push_back(h.w);
        // resident blocks per CU: the tuning's waves, within the CU's LDS
        const int waves_per_block = k.ls.block / 64;
        const int by_waves = std::max(1, tun.waves_per_cu / waves_per_block);
        const int by_lds = std::max<int>(1, static_cast<int>(cu_lds / (k.ls.lds + 64)));
        k.grid = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(n_cu) * std::min(by_waves, by_lds),
                                                    k.n_work));
    }
    if (wl.size() > 0x7fffffffu - 65536u) return fail(AMI_E_ARG, "too many work items");

    // one device allocation: descriptors | work | jobs | counters | partials
    const size_t sz_desc = sizeof(BatchDesc) * n_items;
    const size_t off_work = (sz_desc + 255) & ~size_t(255);
    const size_t sz_work = sizeof(Work) * wl.size();
    const size_t off_jobs = (off_work + sz_work + 255) & ~size_t(255);
    size_t n_jobs = 0;
    for (int i = 0; i < n_items; ++i)
        if (items[i].out_sum && !spec[i]) n_jobs += 2 * static_cast<size_t>(items[i].n_f);
    const size_t sz_jobs = sizeof(RowSumJob) * std::max<size_t>(n_jobs, 1);
    const size_t off_ctr = (off_jobs + sz_jobs + 255) & ~size_t(255);
    const size_t off_part = off_ctr + ((sizeof(unsigned int) * kCounterStride * kMaxClasses + 255) & ~size_t(255));
    const size_t total = off_part + sizeof(double) * std::max<size_t>(partial_total, 1);

    AmiBatch *b = new (std::nothrow) AmiBatch();
    if (!b) return fail(AMI_E_OOM, "out of host memory");
    b->device = dev;
    b->hub = hub;
    b->n_items = n_items;
    b->n_classes = static_cast<int>(cls.size());
    b->n_work = static_cast<int64_t>(wl.size());
    b->n_jobs = static_cast<int64_t>(n_jobs);
    int n_spec = 0;
    for (int i = 0; i < n_items; ++i) n_spec += spec[i] ? 1 : 0;
    b->n_spec = n_spec;
    int64_t most = -1;
    for (const Class &k : cls) {
        b->grid += k.grid;
        b->lds = std::max(b->lds, k.ls.lds);
        if (k.n_work > most) {
            most = k.n_work;
            b->block = k.ls.block;
        }
    }
    e = hipMalloc(&b->blob, total);
    if (e != hipSuccess) return batch_fail_free(b, fail(AMI_E_OOM, "batch workspace"));
    unsigned char *base = static_cast<unsigned char *>(b->blob);
    double *partial = reinterpret_cast<double *>(base + off_part);
    std::vector<RowSumJob> jobs;
    for (int i = 0; i < n_items; ++i) {
        desc[i].a.partial = items[i].out_sum && !spec[i] ? partial + partial_off[i] : nullptr;
        if (items[i].out_sum && !spec[i])
            for (int c = 0; c < 2 * items[i].n_f; ++c) {
                RowSumJob j;
                j.partial = partial + partial_off[i];
                j.dst = items[i].out_sum + c;
                j.nblocks = tiles[i];
                j.ncols = static_cast<int32_t>(2 * items[i].n_f);
                j.col = c;
                jobs.push_back(j);
            }
    }
    std::vector<unsigned char> host(off_part, 0);
    std::memcpy(host.data(), desc.data(), sz_desc);
    if (sz_work) std::memcpy(host.data() + off_work, wl.data(), sz_work);
    if (!jobs.empty()) std::memcpy(host.data() + off_jobs, jobs.data(), sizeof(RowSumJob) * jobs.size());
    e = hipMemcpy(b->blob, host.data(), off_part, hipMemcpyHostToDevice);
    if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "batch upload"));

    // graph: reset counters -> one persistent kernel per class -> row sums
    const BatchDesc *d_desc = reinterpret_cast<const BatchDesc *>(base);
    const RowSumJob *d_jobs = reinterpret_cast<const RowSumJob *>(base + off_jobs);
    unsigned int *d_ctr = reinterpret_cast<unsigned int *>(base + off_ctr);
    e = hipGraphCreate(&b->graph, 0);
    if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "hipGraphCreate"));
    hipGraphNode_t n_reset = nullptr, n_sum = nullptr;
    std::vector<hipGraphNode_t> n_main;
    {
        int n_ctr = static_cast<int>(cls.size());
        void *args[] = {&d_ctr, &n_ctr};
        hipKernelNodeParams p;
        std::memset(&p, 0, sizeof(p));
        p.func = reinterpret_cast<void *>(&ami_batch_reset_kernel);
        p.gridDim = dim3(1);
        p.blockDim = dim3(64);
        p.kernelParams = args;
        e = hipGraphAddKernelNode(&n_reset, b->graph, nullptr, 0, &p);
        if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "graph reset node"));
    }
    for (size_t c = 0; c < cls.size(); ++c) {
        const Class &k = cls[c];
        if (k.n_work == 0) continue;
        const Work *d_work = reinterpret_cast<const Work *>(base + off_work) + k.work0;
        int n_work = static_cast<int>(k.n_work);
        unsigned int *ctr = d_ctr + c * kCounterStride;
        void *args[] = {&d_desc, &d_work, &n_work, &ctr};
        hipKernelNodeParams p;
        std::memset(&p, 0, sizeof(p));
        bool all = false;
        for (int i : k.items) all = all || desc[i].shape == kShapeGeneric || desc[i].shape > 6;
        if (hub) p.func = all ? reinterpret_cast<void *>(&ami_batch_kernel<true, true>)
                              : reinterpret_cast<void *>(&ami_batch_kernel<true, false>);
        else p.func = all ? reinterpret_cast<void *>(&ami_batch_kernel<false, true>)
                          : reinterpret_cast<void *>(&ami_batch_kernel<false, false>);
        p.gridDim = dim3(static_cast<unsigned>(k.grid));
        p.blockDim = dim3(static_cast<unsigned>(k.ls.block));
        p.sharedMemBytes = static_cast<unsigned>(k.ls.lds);
        p.kernelParams = args;
        hipGraphNode_t node = nullptr;
        e = hipGraphAddKernelNode(&node, b->graph, &n_reset, 1, &p);
        if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "graph batch node"));
        n_main.push_back(node);
    }
    if (n_jobs > 0) {
        void *args[] = {&d_jobs};
        hipKernelNodeParams p;
        std::memset(&p, 0, sizeof(p));
        p.func = reinterpret_cast<void *>(&ami_batch_rowsum_kernel);
        p.gridDim = dim3(static_cast<unsigned>(n_jobs));
        p.blockDim = dim3(256);
        p.kernelParams = args;
        e = hipGraphAddKernelNode(&n_sum, b->graph, n_main.data(), n_main.size(), &p);
        if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "graph row-sum node"));
    }
    if (n_spec > 0) {
        const AmiStatus st = capture_specialized(b, items, spec, hub);
        if (st != AMI_OK) return batch_fail_free(b, st);
    }
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return batch_fail_free(b, hip_fail(e, "hipGraphInstantiate"));
    *out = b;
    return AMI_OK;
}

AmiStatus amiBatchRun(AmiBatch *b, void *hip_stream) {
    using namespace ami;
    clear_error();
    if (!b || !b->exec) return fail(AMI_E_ARG, "batch is NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != b->device) return fail(AMI_E_ARG, "batch was created on another device");
    e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return AMI_OK;
}

AmiStatus amiBatchInfo(const AmiBatch *b, int64_t info[10]) {
    using namespace ami;
    clear_error();
    if (!b || !info) return fail(AMI_E_ARG, "NULL argument");
    info[0] = b->n_items;
    info[1] = b->n_work;
    info[2] = b->grid;
    info[3] = b->block;
    info[4] = static_cast<int64_t>(b->lds);
    info[5] = b->n_jobs;
    info[6] = b->hub ? 1 : 0;
    info[7] = b->n_classes;
    info[8] = b->n_spec;
    info[9] = b->n_streams;
    return AMI_OK;
}

void amiBatchFree(AmiBatch *b) {
    if (!b) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    (void)hipSetDevice(b->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->blob) (void)hipFree(b->blob);
    for (hipModule_t m : b->modules) (void)hipModuleUnload(m);
    for (int k = 0; k < b->n_streams; ++k)
        if (b->streams[k]) (void)hipStreamDestroy(b->streams[k]);
    if (have) (void)hipSetDevice(cur);
    delete b;
}

}  // extern "C"
