// ppc_batch.hip -- batched pospopcnt: many arrays of uneven length and mixed
// width in one persistent launch.
//
// The same per-wave tile walk as the plain call (CSA bit planes, cross-lane
// reduction) runs over a table of work items (array, tile range).  Waves of
// a persistent grid take items from a global atomic cursor, largest items
// first, so a few huge arrays and thousands of tiny ones share the device
// evenly.  The width is applied only when an item's 64 address-position
// counts are folded into its array's w counters (Section 5: one kernel,
// the accumulation function picks the width).  Each item's fold ends in at
// most w 64-bit atomics into that array's counters, so results are exact
// and independent of the order in which items run.
//
// A plan is built once per batch (validation, work split, autotuned tile
// and grid sizes) and replayed as a captured hipGraph.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <vector>

#include "ppc.h"
#include "ppc_batch.hpp"
#include "ppc_device.hpp"
#include "ppc_host.hpp"

namespace ppc {

// Resets the work cursor before a persistent launch that uses it (a
// kernel, not a memset, so the sequence can live in a hipGraph).
__global__ void prologue_kernel(uint32_t *cursor) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *cursor = 0u;
}

// The persistent loop of one wave (index gw of nw): group gw first, then
// groups nw + ticket while the cursor hands out tickets below the end.  A
// wave's first group needs no ticket, so the launch does not start with
// every wave queueing on one atomic.  The next ticket is taken only once
// the current group is done: a ticket taken in advance reserves a group
// for the whole of the current one, and near the end short groups then
// wait behind long ones while other waves are idle (10,000-array mix, 4 MiB
// items: a ~190 us tail, 6.6 against 6.9 TB/s).  The ticket's latency is
// small against a group, which closes at 16 or 32 tiles' worth of work
// unless the batch is small enough to give every wave one group.  If there
// are no more groups
// than waves, a wave's first group is its only one and the cursor is not
// touched: otherwise every wave's last atomic, which finds nothing, would
// queue on the one address at the same moment.
__device__ __forceinline__ void run_groups(const ArrayInfo *__restrict__ arrays, const WorkItem *__restrict__ items,
                                           const uint32_t *__restrict__ groups, uint32_t n_groups, uint32_t *cursor,
                                           uint32_t gw, uint32_t nw) {
    const uint32_t lane = __lane_id();
    uint32_t grp = gw;
    while (grp < n_groups) {
        const uint32_t i0 = groups[grp], i1 = groups[grp + 1];
        run_items(arrays, items, i0, i1);
        if (n_groups <= nw) break;
        uint32_t ticket = 0;
        if (lane == 0) ticket = atomicAdd(cursor, 1u);
        grp = nw + (uint32_t)__builtin_amdgcn_readfirstlane((int)ticket);
    }
}

template <int WPB>
__global__ __launch_bounds__(WPB *kWave) void batched_kernel(const ArrayInfo *__restrict__ arrays,
                                                             const WorkItem *__restrict__ items,
                                                             const uint32_t *__restrict__ groups, uint32_t n_groups,
                                                             uint32_t *cursor) {
    run_groups(arrays, items, groups, n_groups, cursor, blockIdx.x * WPB + wave_in_block(), gridDim.x * WPB);
}

// Small arrays (see is_small_array): wave g of nw takes entries g, g + nw,
// ... of the index table, loading the next entry's descriptor while the
// current array runs.  WPE waves per SIMD: 8 for at most two chunks per
// lane (63-64 VGPRs), 4 above (69-108 VGPRs).
template <int K, int WPE>
__global__ __launch_bounds__(kSmallWpb *kWave) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void
small_arrays_kernel(const ArrayInfo *__restrict__ arrays, const uint32_t *__restrict__ idx, uint32_t n) {
    const uint32_t nw = gridDim.x * kSmallWpb;
    uint32_t i = blockIdx.x * kSmallWpb + wave_in_block();
    if (i >= n) return;
    ArrayInfo ai = arrays[idx[i]];
    for (; i < n; i += nw) {
        const ArrayInfo nai = arrays[idx[min(i + nw, n - 1u)]];  // the last entry again past the end
        run_small_array<K>(ai);
        ai = nai;
    }
}

hipError_t launch_small_arrays(const ArrayInfo *arrays_dev, const uint32_t *idx_dev, uint32_t n, uint32_t k_max,
                               int cus, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const uint32_t k = small_k_class(k_max);
    const uint32_t wpe = k <= 2u ? 8u : 4u;
    // one round of resident blocks at most: 4 SIMDs x wpe waves per CU
    const uint32_t blocks =
        std::max<uint32_t>(1u, std::min<uint32_t>((uint32_t)std::max(cus, 1) * wpe, (n + kSmallWpb - 1) / kSmallWpb));
    const dim3 grid(blocks), block(kSmallWpb * kWave);
    switch (k) {
    case 1: hipLaunchKernelGGL((small_arrays_kernel<1, 8>), grid, block, 0, st, arrays_dev, idx_dev, n); break;
    case 2: hipLaunchKernelGGL((small_arrays_kernel<2, 8>), grid, block, 0, st, arrays_dev, idx_dev, n); break;
    case 4: hipLaunchKernelGGL((small_arrays_kernel<4, 4>), grid, block, 0, st, arrays_dev, idx_dev, n); break;
    case 8: hipLaunchKernelGGL((small_arrays_kernel<8, 4>), grid, block, 0, st, arrays_dev, idx_dev, n); break;
    default:
        hipLaunchKernelGGL((small_arrays_kernel<kSmallMaxK, 4>), grid, block, 0, st, arrays_dev, idx_dev, n);
        break;
    }
    return hipGetLastError();
}

// ---- server batch sequence (captured once per stream) ---------------------
__global__ void stage_copy_kernel(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst, uint32_t items_off,
                                  uint32_t groups_off) {
    const BatchHeader h = *reinterpret_cast<const BatchHeader *>(src);
    const uint32_t n4_head = (uint32_t)((sizeof(BatchHeader) + (size_t)h.n_arrays * sizeof(ArrayInfo)) / 4u);
    const uint32_t n4_items = (uint32_t)((size_t)h.n_items * sizeof(WorkItem) / 4u);
    const uint32_t n4_groups = h.n_groups + 1u;
    const uint32_t *s4 = reinterpret_cast<const uint32_t *>(src);
    uint32_t *d4 = reinterpret_cast<uint32_t *>(dst);
    const uint32_t io = items_off / 4u, go = groups_off / 4u;
    const uint32_t total = n4_head + n4_items + n4_groups;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const uint32_t j = i < n4_head ? i : (i < n4_head + n4_items ? io + (i - n4_head) : go + (i - n4_head - n4_items));
        d4[j] = s4[j];
    }
}

template <int WPB>
__global__ __launch_bounds__(WPB *kWave) void served_batch_kernel(const uint8_t *__restrict__ stage, uint32_t items_off,
                                                                  uint32_t groups_off, uint32_t *cursor) {
    const BatchHeader *h = reinterpret_cast<const BatchHeader *>(stage);
    run_groups(reinterpret_cast<const ArrayInfo *>(stage + sizeof(BatchHeader)),
               reinterpret_cast<const WorkItem *>(stage + items_off),
               reinterpret_cast<const uint32_t *>(stage + groups_off), h->n_groups, cursor,
               blockIdx.x * WPB + wave_in_block(), gridDim.x * WPB);
}

__global__ void served_epilogue_kernel(const uint8_t *__restrict__ stage, unsigned long long *counts,
                                       uint64_t *results, uint32_t *cursor) {
    const uint32_t n = reinterpret_cast<const BatchHeader *>(stage)->n_arrays * 64u;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        results[i] = counts[i];
        counts[i] = 0ull;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *cursor = 0u;
}

hipError_t enqueue_served_batch(hipStream_t st, const uint8_t *stage_host, uint8_t *stage_dev, size_t items_off,
                                size_t groups_off, unsigned long long *counts_dev, uint64_t *results_host,
                                uint32_t *cursor_dev, uint32_t waves) {
    constexpr int kWpb = 4;
    hipLaunchKernelGGL(stage_copy_kernel, dim3(16), dim3(256), 0, st, stage_host, stage_dev, (uint32_t)items_off,
                       (uint32_t)groups_off);
    hipLaunchKernelGGL(served_batch_kernel<kWpb>, dim3((waves + kWpb - 1) / kWpb), dim3(kWpb * kWave), 0, st,
                       (const uint8_t *)stage_dev, (uint32_t)items_off, (uint32_t)groups_off, cursor_dev);
    hipLaunchKernelGGL(served_epilogue_kernel, dim3(64), dim3(256), 0, st, (const uint8_t *)stage_dev, counts_dev,
                       results_host, cursor_dev);
    return hipGetLastError();
}

hipError_t capture_served_graph(hipGraph_t *graph, hipGraphExec_t *exec, const uint8_t *stage_host,
                                uint8_t *stage_dev, size_t items_off, size_t groups_off,
                                unsigned long long *counts_dev, uint64_t *results_host, uint32_t *cursor_dev,
                                uint32_t waves) {
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t launched = enqueue_served_batch(cap, stage_host, stage_dev, items_off, groups_off,
                                                         counts_dev, results_host, cursor_dev, waves);
        e = hipStreamEndCapture(cap, graph);
        if (e == hipSuccess) e = launched;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    return e;
}

void append_items(std::vector<WorkItem> &items, const ArrayInfo &ai, uint32_t idx, uint32_t tiles_per_item) {
    const uint32_t p = std::max(1u, std::min(tiles_per_item, kMaxItemTiles));
    const bool edges = ai.edge0_len + ai.edge1_len > 0;
    if (ai.n_tiles == 0) {
        if (edges) items.push_back(WorkItem{idx, 0u, 0u, 1u});
        return;
    }
    for (uint32_t t = 0; t < ai.n_tiles; t += p) {
        const uint32_t t1 = (uint32_t)std::min<uint64_t>((uint64_t)t + p, ai.n_tiles);
        items.push_back(WorkItem{idx, t, t1, (t == 0 && edges) ? 1u : 0u});
    }
}

void sort_items_lpt(std::vector<WorkItem> &items) {
    std::stable_sort(items.begin(), items.end(), [](const WorkItem &x, const WorkItem &y) {
        return (x.tile1 - x.tile0) > (y.tile1 - y.tile0);
    });
}

std::vector<uint32_t> build_groups(const std::vector<WorkItem> &items, uint32_t waves, uint32_t cost_limit) {
    const uint64_t spread = waves ? (items.size() + waves - 1) / waves : (uint64_t)kGroupMax;  // 0: no cap
    const uint32_t max_items = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(kGroupMax, spread));
    std::vector<uint32_t> starts;
    starts.reserve(items.size() / max_items + 2);
    uint32_t cost = 0, count = 0;
    for (uint32_t i = 0; i < (uint32_t)items.size(); ++i) {
        if (count == 0) starts.push_back(i);
        cost += (items[i].tile1 - items[i].tile0) + 1u;
        ++count;
        if (cost >= cost_limit || count >= max_items) {
            cost = 0;
            count = 0;
        }
    }
    starts.push_back((uint32_t)items.size());
    return starts;
}

hipError_t launch_batched(const ArrayInfo *arrays_dev, const WorkItem *items_dev, const uint32_t *groups_dev,
                          uint32_t n_groups, uint32_t *cursor_dev, uint32_t waves, hipStream_t st) {
    constexpr int kWpb = 4;
    const uint32_t w = std::max<uint32_t>(kWpb, std::min<uint32_t>(waves, n_groups + kWpb - 1));
    const uint32_t blocks = (w + kWpb - 1) / kWpb;
    // the grid's waves are blocks * kWpb (run_groups' nw): with no more groups
    // than that, no wave reads the cursor and the reset is left out (an
    // empty batch keeps it, so that a captured graph is never empty)
    if (n_groups == 0 || n_groups > blocks * (uint32_t)kWpb)
        hipLaunchKernelGGL(prologue_kernel, dim3(1), dim3(64), 0, st, cursor_dev);
    if (n_groups == 0) return hipGetLastError();
    hipLaunchKernelGGL(batched_kernel<kWpb>, dim3(blocks), dim3(kWpb * kWave), 0, st, arrays_dev, items_dev,
                       groups_dev, n_groups, cursor_dev);
    return hipGetLastError();
}

// ---- autotuner cache ------------------------------------------------------
static std::mutex g_tune_mu;

static std::string tune_cache_path() {
    if (const char *p = std::getenv("PPC_TUNE_CACHE")) return p;
    const char *home = std::getenv("HOME");
    std::string dir = std::string(home && *home ? home : "/tmp") + "/.cache";
    ::mkdir(dir.c_str(), 0755);
    return dir + "/ppc_tune.txt";
}

static int log2_bucket(uint64_t v) {
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

static bool tune_lookup(const std::string &key, uint32_t &p, uint32_t &waves) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = std::fopen(tune_cache_path().c_str(), "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[400];
        unsigned a = 0, b = 0;
        if (std::sscanf(line, "%399s %u %u", k, &a, &b) == 3 && key == k && a > 0 && b > 0) {
            p = a;
            waves = b;
            found = true;  // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

static void tune_store(const std::string &key, uint32_t p, uint32_t waves) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = std::fopen(tune_cache_path().c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %u %u\n", key.c_str(), p, waves);
    std::fclose(f);
}

}  // namespace ppc

using namespace ppc;

struct ppc_plan {
    int device = 0;
    std::vector<ArrayInfo> arrays;
    ArrayInfo *arrays_dev = nullptr;
    WorkItem *items_dev = nullptr;
    uint32_t *groups_dev = nullptr;
    uint32_t *cursor_dev = nullptr;
    uint32_t *small_dev = nullptr;  // indices of the arrays run by the small-array kernel
    uint32_t n_items = 0, n_groups = 0;
    uint32_t n_small = 0, small_k = 0;  // small arrays and their most chunks per lane
    uint32_t tiles_per_item = 0;
    uint32_t waves = 0;
    uint64_t total_bytes = 0;
    uint32_t tuned = 0;  // 0 = given/heuristic, 1 = measured now, 2 = from cache
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void plan_free(ppc_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->arrays_dev) (void)hipFree(p->arrays_dev);
    if (p->items_dev) (void)hipFree(p->items_dev);
    if (p->groups_dev) (void)hipFree(p->groups_dev);
    if (p->cursor_dev) (void)hipFree(p->cursor_dev);
    if (p->small_dev) (void)hipFree(p->small_dev);
    delete p;
}

// Work items of every array that the small-array kernel does not take.
std::vector<WorkItem> build_items(const std::vector<ArrayInfo> &arrays, uint32_t tiles_per_item) {
    std::vector<WorkItem> items;
    items.reserve(arrays.size() * 2);
    for (uint32_t i = 0; i < (uint32_t)arrays.size(); ++i)
        if (!is_small_array(arrays[i])) append_items(items, arrays[i], i, tiles_per_item);
    sort_items_lpt(items);
    return items;
}

// The small arrays with anything to count, in table order; k_max = their
// most chunks per lane.
std::vector<uint32_t> small_arrays(const std::vector<ArrayInfo> &arrays, uint32_t &k_max) {
    std::vector<uint32_t> idx;
    k_max = 0;
    for (uint32_t i = 0; i < (uint32_t)arrays.size(); ++i) {
        const ArrayInfo &a = arrays[i];
        if (!is_small_array(a) || a.n_chunks + a.edge0_len + a.edge1_len == 0) continue;
        idx.push_back(i);
        k_max = std::max(k_max, small_chunks_per_lane(a));
    }
    return idx;
}

// One run of the plan on `st`: the persistent kernel over the work items
// (or, for an empty plan, its cursor reset alone, so that a captured graph
// is never empty), then the small-array kernel.
hipError_t plan_enqueue(const ppc_plan *p, hipStream_t st) {
    if (p->n_groups > 0 || p->n_small == 0) {
        const hipError_t e =
            launch_batched(p->arrays_dev, p->items_dev, p->groups_dev, p->n_groups, p->cursor_dev, p->waves, st);
        if (e != hipSuccess) return e;
    }
    return launch_small_arrays(p->arrays_dev, p->small_dev, p->n_small, p->small_k, device_cus(p->device), st);
}

// Times one (tiles_per_item, waves) candidate on the plan's arrays with the
// counters redirected to scratch; returns the median of `reps` runs in ms.
ppc_status time_candidate(const ArrayInfo *tune_arrays_dev, const std::vector<ArrayInfo> &arrays, uint32_t p,
                          uint32_t waves, uint32_t *cursor_dev, hipStream_t st, int reps, float &ms_out) {
    std::vector<WorkItem> items = build_items(arrays, p);
    std::vector<uint32_t> groups = build_groups(items, waves, kPlanGroupCost);
    WorkItem *items_dev = nullptr;
    uint32_t *groups_dev = nullptr;
    if (!items.empty() && hipMalloc(&items_dev, items.size() * sizeof(WorkItem)) != hipSuccess) return PPC_ENOMEM;
    if (hipMalloc(&groups_dev, groups.size() * sizeof(uint32_t)) != hipSuccess) {
        if (items_dev) (void)hipFree(items_dev);
        return PPC_ENOMEM;
    }
    ppc_status rc = PPC_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<float> t;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = PPC_EDEVICE;
    if (rc == PPC_OK && !items.empty() &&
        hipMemcpyAsync(items_dev, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, st) !=
            hipSuccess)
        rc = PPC_EDEVICE;
    if (rc == PPC_OK &&
        hipMemcpyAsync(groups_dev, groups.data(), groups.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st) !=
            hipSuccess)
        rc = PPC_EDEVICE;
    const uint32_t n_groups = (uint32_t)groups.size() - 1u;
    for (int r = 0; rc == PPC_OK && r <= reps; ++r) {  // run 0 warms up
        if (hipEventRecord(e0, st) != hipSuccess ||
            launch_batched(tune_arrays_dev, items_dev, groups_dev, n_groups, cursor_dev, waves, st) != hipSuccess ||
            hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = PPC_EDEVICE;
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r > 0) t.push_back(ms);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    if (items_dev) (void)hipFree(items_dev);
    (void)hipFree(groups_dev);
    if (rc == PPC_OK) {
        std::sort(t.begin(), t.end());
        ms_out = t[t.size() / 2];
    }
    return rc;
}

ppc_status autotune(ppc_plan *p, hipStream_t st, uint32_t &best_p, uint32_t &best_w) {
    const int cus = device_cus(p->device);
    const size_t n = p->arrays.size();
    // redirect every array's counters into scratch so tuning runs leave the
    // caller's counters untouched
    std::vector<ArrayInfo> tune = p->arrays;
    unsigned long long *scratch = nullptr;
    ArrayInfo *tune_dev = nullptr;
    if (hipMalloc(&scratch, n * 64 * sizeof(unsigned long long)) != hipSuccess) return PPC_ENOMEM;
    for (size_t i = 0; i < n; ++i) tune[i].counts = scratch + i * 64;
    ppc_status rc = PPC_OK;
    if (hipMalloc(&tune_dev, n * sizeof(ArrayInfo)) != hipSuccess) rc = PPC_ENOMEM;
    if (rc == PPC_OK &&
        hipMemcpyAsync(tune_dev, tune.data(), n * sizeof(ArrayInfo), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = PPC_EDEVICE;
    const uint32_t cand_p[] = {4, 16, 64, 256, 1024};
    const uint32_t cand_w[] = {4, 8, 16};
    float best = 1e30f;
    for (uint32_t cp : cand_p)
        for (uint32_t cw : cand_w) {
            if (rc != PPC_OK) break;
            float ms = 0;
            rc = time_candidate(tune_dev, tune, cp, cw * (uint32_t)cus, p->cursor_dev, st, 3, ms);
            if (rc == PPC_OK && ms < best) {
                best = ms;
                best_p = cp;
                best_w = cw * (uint32_t)cus;
            }
        }
    (void)hipStreamSynchronize(st);
    if (tune_dev) (void)hipFree(tune_dev);
    (void)hipFree(scratch);
    return rc;
}

std::string tune_key(const ppc_plan *p) {
    std::vector<uint64_t> len;
    len.reserve(p->arrays.size());
    uint64_t mx = 0;
    for (const auto &a : p->arrays) {
        const uint64_t b = a.n_chunks * 16u + a.edge0_len + a.edge1_len;
        len.push_back(b);
        mx = std::max(mx, b);
    }
    uint64_t med = 0;
    if (!len.empty()) {
        std::nth_element(len.begin(), len.begin() + len.size() / 2, len.end());
        med = len[len.size() / 2];
    }
    hipDeviceProp_t prop;
    std::string name = "gpu";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) name = prop.gcnArchName;
    for (auto &ch : name)
        if (ch == ' ' || ch == ':') ch = '_';
    char buf[384];
    std::snprintf(buf, sizeof buf, "batched/%s/cu%d/n%d/bytes%d/med%d/max%d", name.c_str(), device_cus(p->device),
                  log2_bucket(p->arrays.size()), log2_bucket(p->total_bytes), log2_bucket(med), log2_bucket(mx));
    return buf;
}

}  // namespace

extern "C" {

ppc_status ppc_plan_create(ppc_plan **out, const ppc_desc *descs, size_t n, const ppc_plan_opts *opts,
                           void *stream) {
    if (out == nullptr) return PPC_EINVAL;
    *out = nullptr;
    if (n > 0 && descs == nullptr) return PPC_EINVAL;
    if (n >= (1ull << 31)) return PPC_EINVAL;
    if (opts && opts->reserved != 0) return PPC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    auto *p = new (std::nothrow) ppc_plan();
    if (!p) return PPC_ENOMEM;
    p->arrays.resize(n);
    for (size_t i = 0; i < n; ++i) {  // all argument checks come before any HIP call
        if (descs[i].reserved != 0 ||
            !make_array_info(p->arrays[i], descs[i].buf, descs[i].nbytes, descs[i].counts, descs[i].width)) {
            plan_free(p);
            return PPC_EINVAL;
        }
        p->total_bytes += descs[i].nbytes;
    }
    if (hipGetDevice(&p->device) != hipSuccess) {
        plan_free(p);
        return PPC_EDEVICE;
    }
    if (hipMalloc(&p->cursor_dev, sizeof(uint32_t)) != hipSuccess) {
        plan_free(p);
        return PPC_ENOMEM;
    }
    const int cus = device_cus(p->device);
    uint32_t tp = opts ? opts->tiles_per_item : 0u;
    uint32_t wv = opts ? opts->waves : 0u;
    const bool want_tune = opts ? opts->autotune != 0 : true;
    if (tp == 0 || wv == 0) {
        uint32_t bp = 16, bw = 8u * (uint32_t)cus;  // heuristic default
        const std::string key = tune_key(p);
        if (want_tune && tune_lookup(key, bp, bw)) {
            p->tuned = 2;
        } else if (want_tune && n > 0 && p->total_bytes >= ((uint64_t)64 << 20) &&
                   std::any_of(p->arrays.begin(), p->arrays.end(),
                               [](const ArrayInfo &a) { return !is_small_array(a); })) {
            ppc_status rc = autotune(p, st, bp, bw);
            if (rc != PPC_OK) {
                plan_free(p);
                return rc;
            }
            tune_store(key, bp, bw);
            p->tuned = 1;
        }
        if (tp == 0) tp = bp;
        if (wv == 0) wv = bw;
    }
    p->tiles_per_item = std::min(tp, kMaxItemTiles);
    p->waves = wv;
    std::vector<WorkItem> items = build_items(p->arrays, p->tiles_per_item);
    std::vector<uint32_t> groups = build_groups(items, p->waves, kPlanGroupCost);
    const std::vector<uint32_t> small = small_arrays(p->arrays, p->small_k);
    p->n_items = (uint32_t)items.size();
    p->n_groups = (uint32_t)groups.size() - 1u;
    p->n_small = (uint32_t)small.size();
    if ((n > 0 && hipMalloc(&p->arrays_dev, n * sizeof(ArrayInfo)) != hipSuccess) ||
        (!items.empty() && hipMalloc(&p->items_dev, items.size() * sizeof(WorkItem)) != hipSuccess) ||
        (!small.empty() && hipMalloc(&p->small_dev, small.size() * sizeof(uint32_t)) != hipSuccess) ||
        hipMalloc(&p->groups_dev, groups.size() * sizeof(uint32_t)) != hipSuccess) {
        plan_free(p);
        return PPC_ENOMEM;
    }
    if ((n > 0 && hipMemcpyAsync(p->arrays_dev, p->arrays.data(), n * sizeof(ArrayInfo), hipMemcpyHostToDevice,
                                 st) != hipSuccess) ||
        (!items.empty() && hipMemcpyAsync(p->items_dev, items.data(), items.size() * sizeof(WorkItem),
                                          hipMemcpyHostToDevice, st) != hipSuccess) ||
        (!small.empty() && hipMemcpyAsync(p->small_dev, small.data(), small.size() * sizeof(uint32_t),
                                          hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipMemcpyAsync(p->groups_dev, groups.data(), groups.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        plan_free(p);
        return PPC_EDEVICE;
    }
    p->use_graph = opts ? opts->use_graph != 0 : true;
    if (p->use_graph) {
        hipStream_t cap = nullptr;
        bool ok = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            const bool launched = plan_enqueue(p, cap) == hipSuccess;
            ok = hipStreamEndCapture(cap, &p->graph) == hipSuccess && launched;
        }
        ok = ok && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
        if (cap) (void)hipStreamDestroy(cap);
        if (!ok) {
            plan_free(p);
            return PPC_EDEVICE;
        }
    }
    *out = p;
    return PPC_OK;
}

ppc_status ppc_plan_run(ppc_plan *p, void *stream) {
    if (!p) return PPC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (p->use_graph) return hipGraphLaunch(p->exec, st) == hipSuccess ? PPC_OK : PPC_EDEVICE;
    return plan_enqueue(p, st) == hipSuccess ? PPC_OK : PPC_EDEVICE;
}

ppc_status ppc_plan_get_info(const ppc_plan *p, ppc_plan_info *info) {
    if (!p || !info) return PPC_EINVAL;
    info->n_arrays = p->arrays.size();
    info->n_items = p->n_items + p->n_small;  // a small array is one item
    info->total_bytes = p->total_bytes;
    info->tiles_per_item = p->tiles_per_item;
    info->waves = p->waves;
    info->tuned = p->tuned;
    info->graph = p->use_graph ? 1u : 0u;
    return PPC_OK;
}

ppc_status ppc_plan_destroy(ppc_plan *p) {
    if (!p) return PPC_EINVAL;
    (void)hipDeviceSynchronize();
    plan_free(p);
    return PPC_OK;
}

}  // extern "C"
