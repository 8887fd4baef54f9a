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
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ami_internal.hpp"
#include "device_common.hpp"
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

// counters are kCounterStride apart (one per class)
constexpr int kCounterStride = 16;
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
    for (int k = 0; k < b->n_streams; ++k)
        if (b->streams[k]) (void)hipStreamDestroy(b->streams[k]);
    delete b;
    return st;
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
    if (tun.kernels != 0 && tun.kernels != 1) return fail(AMI_E_ARG, "kernels must be 0 or 1");
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
    for (int k = 0; k < b->n_streams; ++k)
        if (b->streams[k]) (void)hipStreamDestroy(b->streams[k]);
    if (have) (void)hipSetDevice(cur);
    delete b;
}

}  // extern "C"
