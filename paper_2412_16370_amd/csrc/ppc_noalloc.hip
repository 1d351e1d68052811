// ppc_noalloc.hip -- the batched count for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// Same arithmetic as the batched plan (the per-wave tile walk of the plain
// call over work items, f_w per item, 64-bit atomics into each array's
// counters), but the descriptor table is the caller's, in device memory, and
// every table the kernels need lives in one file-scope device array,
// `scratch`, of fixed size:
//   [0, 256)                      header: work cursor and item counts
//   [256, 256 + 64 * 2^16)        one ArrayInfo per array (at most 2^16)
//   [.., + 16 * 2^18)             work items (at most 2^18), largest first
// Two launches per call: a one-block setup kernel validates the
// descriptors, builds the array table, picks the tiles per item and writes
// the items; the persistent kernel then walks them.  Nothing is allocated
// and nothing is copied from the host, so the call can be captured.
//
// Each GPU holds one copy of `scratch` for as long as the process runs;
// calls that overlap on one GPU (different streams, or several host
// threads) share it and race.  Calls ordered on one stream do not.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "ppc.h"
#include "ppc_batch.hpp"
#include "ppc_device.hpp"
#include "ppc_host.hpp"

namespace ppc {

constexpr uint32_t kNaMaxArrays = PPC_NOALLOC_MAX_ARRAYS;
constexpr uint32_t kNaMaxItems = 1u << 18;
// Tiles per whole item: 256 tiles = 4 MiB, the setting the plan's autotuner
// picks for mixed batches.  Raised only when the total would need more than
// kNaMaxItems items, which takes more than 768 GiB of input in one call.
constexpr uint32_t kNaItemTiles = 256;
// Shorter items (one per array at most: its tiles past the last whole item,
// or only its head/tail bytes) go into buckets by the bit length of their
// tile count, clamped to kNaBuckets - 1, and are laid out largest bucket
// first: the largest-first order of the plan, without a sort.  Items of at
// most kNaGroupTiles tiles (buckets below kNaFirstSingle) are handed out
// kNaGroup per ticket; the rest one per ticket.
constexpr int kNaBuckets = 10;
constexpr int kNaFirstSingle = 3;  // bit length 3: 4 tiles or more
constexpr uint32_t kNaGroup = 16;
constexpr int kNaSetupThreads = 1024;
constexpr int kNaWpb = 4;

struct NaHeader {
    uint32_t cursor;     // tickets handed out after each wave's first
    uint32_t n_single;   // whole items, then shorter ones of >= 4 tiles: one per ticket
    uint32_t n_items;    // all items; those past n_single go kNaGroup per ticket
    uint32_t n_tickets;  // n_single + ceil((n_items - n_single) / kNaGroup)
    uint32_t tiles_per_item;
    uint32_t reserved[59];
};
static_assert(sizeof(NaHeader) == 256, "header size");

constexpr size_t kNaArraysOff = sizeof(NaHeader);
constexpr size_t kNaItemsOff = kNaArraysOff + (size_t)kNaMaxArrays * sizeof(ArrayInfo);
constexpr size_t kNaScratchBytes = kNaItemsOff + (size_t)kNaMaxItems * sizeof(WorkItem);
static_assert(kNaScratchBytes == PPC_NOALLOC_SCRATCH_BYTES, "scratch size in the header");

static __device__ __align__(256) uint8_t scratch[kNaScratchBytes];

// Exclusive prefix sums over the block's threads of K values at once
// (Hillis-Steele in LDS, one pair of barriers per step for all K); total[k]
// receives the sum of value k.
template <typename T, int K>
__device__ __forceinline__ void block_exclusive_scan(T (&v)[K], T (*lds)[kNaSetupThreads], T (&total)[K]) {
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k][tid] = v[k];
    __syncthreads();
    for (uint32_t d = 1; d < (uint32_t)kNaSetupThreads; d <<= 1) {
        T add[K];
#pragma unroll
        for (int k = 0; k < K; ++k) add[k] = tid >= d ? lds[k][tid - d] : T(0);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) lds[k][tid] += add[k];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        total[k] = lds[k][kNaSetupThreads - 1];
        v[k] = lds[k][tid] - v[k];
    }
    __syncthreads();
}

// Bucket of a shorter item of t tiles (t < tiles per item).
__device__ __forceinline__ int na_bucket(uint32_t t) { return (int)min(bit_length(t), (uint32_t)(kNaBuckets - 1)); }

// One block.  Thread t handles arrays [t*per, (t+1)*per).  If any
// descriptor is invalid, no item is written and the batch counts nothing.
__global__ __launch_bounds__(kNaSetupThreads) void noalloc_setup_kernel(const ppc_desc *__restrict__ descs,
                                                                        uint32_t n, uint32_t *n_invalid_out,
                                                                        uint8_t *scr) {
    NaHeader *h = reinterpret_cast<NaHeader *>(scr);
    ArrayInfo *arrays = reinterpret_cast<ArrayInfo *>(scr + kNaArraysOff);
    WorkItem *items = reinterpret_cast<WorkItem *>(scr + kNaItemsOff);
    __shared__ uint64_t lds64[1][kNaSetupThreads];
    __shared__ uint32_t lds32[kNaBuckets + 2][kNaSetupThreads];

    const uint32_t tid = threadIdx.x;
    const uint32_t per = (n + kNaSetupThreads - 1) / kNaSetupThreads;
    const uint32_t a0 = min(n, tid * per), a1 = min(n, a0 + per);

    // pass 1: the array table, invalid descriptors, total tiles
    uint32_t bad[1] = {0};
    uint64_t tiles[1] = {0};
    for (uint32_t i = a0; i < a1; ++i) {
        const ppc_desc d = descs[i];
        ArrayInfo ai;
        if (d.reserved != 0u || !make_array_info(ai, d.buf, d.nbytes, d.counts, d.width)) {
            ++bad[0];
            ai = ArrayInfo{};
        }
        arrays[i] = ai;
        tiles[0] += ai.n_tiles;
    }
    uint32_t n_bad[1];
    uint64_t n_tiles[1];
    block_exclusive_scan<uint32_t, 1>(bad, lds32, n_bad);
    block_exclusive_scan<uint64_t, 1>(tiles, lds64, n_tiles);

    // tiles per whole item: every array gives at most n_tiles/P + 1 items,
    // so P >= n_tiles / (kNaMaxItems - n) keeps the total within the table
    const uint64_t room = (uint64_t)kNaMaxItems - n;
    const uint64_t p64 = max((uint64_t)kNaItemTiles, (n_tiles[0] + room - 1) / room);
    const bool ok = n_bad[0] == 0u && p64 <= (uint64_t)kMaxItemTiles;
    const uint32_t P = (uint32_t)min(p64, (uint64_t)kMaxItemTiles);

    // pass 2: items per thread: whole ones, and per bucket the shorter ones
    // (one at most per array)
    uint32_t cnt[kNaBuckets + 1] = {0};  // [0, kNaBuckets): buckets, [kNaBuckets]: whole items
    if (ok) {
        for (uint32_t i = a0; i < a1; ++i) {
            const ArrayInfo &ai = arrays[i];
            const bool edges = ai.edge0_len + ai.edge1_len > 0u;
            const uint32_t rest = ai.n_tiles % P;
            cnt[kNaBuckets] += ai.n_tiles / P;
            if (rest != 0u || (ai.n_tiles == 0u && edges)) ++cnt[na_bucket(rest)];
        }
    }
    uint32_t tot[kNaBuckets + 1];
    block_exclusive_scan<uint32_t, kNaBuckets + 1>(cnt, lds32, tot);

    // layout: whole items, then buckets from the largest down
    uint32_t base[kNaBuckets];
    uint32_t next = tot[kNaBuckets];
    for (int k = kNaBuckets - 1; k >= 0; --k) {
        base[k] = next;
        next += tot[k];
    }
    const uint32_t n_items = next;
    const uint32_t n_single = base[kNaFirstSingle] + tot[kNaFirstSingle];

    // pass 3: write the items; an array's first item carries its edges
    if (ok) {
        uint32_t f = cnt[kNaBuckets];
        for (uint32_t i = a0; i < a1; ++i) {
            const ArrayInfo &ai = arrays[i];
            const uint32_t edges = ai.edge0_len + ai.edge1_len > 0u ? 1u : 0u;
            const uint32_t whole = ai.n_tiles / P, rest = ai.n_tiles % P;
            for (uint32_t k = 0; k < whole; ++k) items[f++] = WorkItem{i, k * P, (k + 1u) * P, k == 0u ? edges : 0u};
            if (rest != 0u || (ai.n_tiles == 0u && edges)) {
                const int b = na_bucket(rest);
                items[base[b] + cnt[b]++] = WorkItem{i, whole * P, ai.n_tiles, whole == 0u ? edges : 0u};
            }
        }
    }
    if (tid == 0) {
        h->cursor = 0u;
        h->n_single = ok ? n_single : 0u;
        h->n_items = ok ? n_items : 0u;
        h->n_tickets = ok ? n_single + (n_items - n_single + kNaGroup - 1u) / kNaGroup : 0u;
        h->tiles_per_item = P;
        if (n_invalid_out) *n_invalid_out = ok ? 0u : (n_bad[0] ? n_bad[0] : n);
    }
}

// Persistent walk: wave g starts with ticket g, then takes tickets from the
// cursor once its current one is done.  Ticket t < n_single is item t;
// later tickets are runs of kNaGroup items.
template <int WPB>
__global__ __launch_bounds__(WPB *kWave) void noalloc_batched_kernel(uint8_t *scr) {
    NaHeader *h = reinterpret_cast<NaHeader *>(scr);
    const ArrayInfo *arrays = reinterpret_cast<const ArrayInfo *>(scr + kNaArraysOff);
    const WorkItem *items = reinterpret_cast<const WorkItem *>(scr + kNaItemsOff);
    const uint32_t n_tickets = (uint32_t)__builtin_amdgcn_readfirstlane((int)h->n_tickets);
    const uint32_t n_single = (uint32_t)__builtin_amdgcn_readfirstlane((int)h->n_single);
    const uint32_t n_items = (uint32_t)__builtin_amdgcn_readfirstlane((int)h->n_items);
    const uint32_t nw = gridDim.x * WPB;
    uint32_t t = blockIdx.x * WPB + wave_in_block();
    while (t < n_tickets) {
        if (t < n_single) {
            run_item(arrays, items[t]);
        } else {
            const uint32_t i0 = n_single + (t - n_single) * kNaGroup;
            const uint32_t i1 = min(i0 + kNaGroup, n_items);
            for (uint32_t i = i0; i < i1; ++i) run_item(arrays, items[i]);
        }
        uint32_t ticket = 0;
        if (__lane_id() == 0u) ticket = atomicAdd(&h->cursor, 1u);
        t = nw + (uint32_t)__builtin_amdgcn_readfirstlane((int)ticket);
    }
}

// Device address of `scratch` per device, taken once with that device
// current (each device has its own copy of the array).
static std::mutex g_na_mu;
static uint8_t *g_na_ptr[64] = {nullptr};

static uint8_t *noalloc_scratch(int device) {
    if (device < 0 || device >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (g_na_ptr[device] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return nullptr;
        g_na_ptr[device] = static_cast<uint8_t *>(p);
    }
    return g_na_ptr[device];
}

}  // namespace ppc

using namespace ppc;

extern "C" {

ppc_status ppc_batch_noalloc(const ppc_desc *descs, uint32_t n, uint32_t *n_invalid, void *stream) {
    if (n > kNaMaxArrays) return PPC_EINVAL;
    if (n > 0 && descs == nullptr) return PPC_EINVAL;
    if (((uintptr_t)descs & 7u) != 0 || ((uintptr_t)n_invalid & 3u) != 0) return PPC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PPC_EDEVICE;
    uint8_t *scr = noalloc_scratch(dev);
    if (scr == nullptr) return PPC_EDEVICE;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(kNaSetupThreads), 0, st, descs, n, n_invalid, scr);
    if (n > 0) {
        const uint32_t waves = 4u * (uint32_t)device_cus(dev);
        hipLaunchKernelGGL(noalloc_batched_kernel<kNaWpb>, dim3((waves + kNaWpb - 1) / kNaWpb), dim3(kNaWpb * kWave),
                           0, st, scr);
    }
    return hipGetLastError() == hipSuccess ? PPC_OK : PPC_EDEVICE;
}

}  // extern "C"
