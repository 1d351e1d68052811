// ppc_batch.hpp -- work-item tables shared by the batched plan and the server.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "ppc.h"
#include "ppc_device.hpp"

namespace ppc {

// One array of a batch, as the persistent kernel sees it (64 bytes).
struct ArrayInfo {
    const uint4 *body;          // first full 16-byte chunk (nullptr if none)
    uint64_t n_chunks;          // full chunks
    const uint8_t *edge0;       // head bytes
    const uint8_t *edge1;       // tail bytes
    unsigned long long *counts; // w counters
    uint32_t n_full;            // whole tiles
    uint32_t n_tiles;           // whole tiles + partial tile
    uint32_t edge0_len, edge1_len;
    uint32_t width, m;          // width and buf mod (w/8)
};
static_assert(sizeof(ArrayInfo) == 64, "ArrayInfo layout");

// One unit of work: tiles [tile0, tile1) of array `array`; flag bit 0 = this
// item also counts the array's head/tail bytes.
struct WorkItem {
    uint32_t array;
    uint32_t tile0, tile1;
    uint32_t flags;
};
static_assert(sizeof(WorkItem) == 16, "WorkItem layout");

// Header of a server batch in its staging buffer (64 bytes): the
// ArrayInfo table follows at byte 64, the WorkItem table at a fixed offset.
struct BatchHeader {
    uint32_t n_arrays, n_items, n_groups;
    uint32_t reserved[13];
};
static_assert(sizeof(BatchHeader) == 64, "BatchHeader layout");

// Per-item tile cap: keeps every per-wave 32-bit count below 2^31.
constexpr uint32_t kMaxItemTiles = 1u << 20;

// Fills `ai` for one array (host or device code).  Returns false for an
// invalid array (same rules as the plain call); `ai` then describes an
// empty array.
__host__ __device__ inline bool make_array_info(ArrayInfo &ai, const void *buf, uint64_t nbytes, uint64_t *counts,
                                                uint32_t width) {
    ai = ArrayInfo{};
    if (!(width == 8 || width == 16 || width == 32 || width == 64)) return false;
    if (counts == nullptr || ((uintptr_t)counts & 7u) != 0) return false;
    if (nbytes > 0 && buf == nullptr) return false;
    if (nbytes == 0) {
        ai.counts = reinterpret_cast<unsigned long long *>(counts);
        ai.width = width;
        return true;
    }
    const uintptr_t b0 = (uintptr_t)buf, b1 = b0 + nbytes;
    const uintptr_t f = (b0 + 15u) & ~(uintptr_t)15u, e = b1 & ~(uintptr_t)15u;
    if (f < e) {
        const uint64_t n_chunks = (uint64_t)(e - f) / 16u;
        const uint64_t n_tiles = (n_chunks + kTileChunks - 1) / kTileChunks;
        if (n_tiles >= (1ull << 32)) return false;  // > 64 TiB in one array
        ai.body = reinterpret_cast<const uint4 *>(f);
        ai.n_chunks = n_chunks;
        ai.n_full = (uint32_t)(n_chunks / kTileChunks);
        ai.n_tiles = (uint32_t)n_tiles;
        ai.edge0 = static_cast<const uint8_t *>(buf);
        ai.edge0_len = (uint32_t)(f - b0);
        ai.edge1 = reinterpret_cast<const uint8_t *>(e);
        ai.edge1_len = (uint32_t)(b1 - e);
    } else {
        ai.edge0 = static_cast<const uint8_t *>(buf);
        ai.edge0_len = (uint32_t)nbytes;  // <= 30
    }
    ai.counts = reinterpret_cast<unsigned long long *>(counts);
    ai.width = width;
    ai.m = (uint32_t)((uintptr_t)buf % (width / 8u));
    return true;
}

// One work item on one wave, with its array's entry: the item's tiles (and
// the array's head/tail bytes if flagged) are counted and folded into the
// array's counters.
__device__ __forceinline__ void run_item_of(const ArrayInfo &ai, const WorkItem &it) {
    const uint32_t lane = __lane_id();
    const bool has_edge = (it.flags & 1u) != 0u;
    uint4 edge = zero4();
    if (has_edge) {
        if (lane < 32) {
            if (lane < ai.edge0_len) edge = byte_as_chunk((uint64_t)(ai.edge0 + lane), ai.edge0[lane]);
        } else if (lane - 32 < ai.edge1_len) {
            edge = byte_as_chunk((uint64_t)(ai.edge1 + (lane - 32)), ai.edge1[lane - 32]);
        }
    }
    const uint32_t acc =
        wave_count_tiles(ai.body, ai.n_chunks, ai.n_full, it.tile0, it.tile1, 1u, edge, has_edge);
    fold_add(acc, ai.width, ai.m, ai.counts);
}

// Items [i0, i1) one after another on one wave.  The next item's array
// entry and the work item after it are loaded while the current item runs,
// so a short item does not wait for its two descriptor loads (work item,
// then array entry) after the previous one.
__device__ __forceinline__ void run_items(const ArrayInfo *__restrict__ arrays, const WorkItem *__restrict__ items,
                                          uint32_t i0, uint32_t i1) {
    if (i0 >= i1) return;
    const uint32_t last = i1 - 1u;
    WorkItem it = items[i0];
    ArrayInfo ai = arrays[it.array];
    WorkItem nit = items[min(i0 + 1u, last)];
    for (uint32_t i = i0; i < i1; ++i) {
        // loads of valid entries only: past the last item they repeat it
        const ArrayInfo nai = arrays[nit.array];
        const WorkItem nnit = items[min(i + 2u, last)];
        run_item_of(ai, it);
        it = nit;
        ai = nai;
        nit = nnit;
    }
}

// ---- arrays shorter than one tile: a kernel of their own -------------------
// Such an array is a single work item on which a wave holds at most
// kSmallMaxK chunks per lane, so the tile walk only ever takes one of its
// two short paths.  Those need a fraction of the registers of the whole
// walk (63-108 VGPRs against 223), so a kernel built for them alone runs
// 4 or 8 waves per SIMD instead of 2: two to four times as many of these
// short, latency-bound items keep their loads in flight.  Plans give such
// arrays to this kernel; the allocation-free call does in batches of short
// arrays.
constexpr uint32_t kSmallMaxK = 14;
constexpr int kSmallWpb = 4;

__host__ __device__ inline bool is_small_array(const ArrayInfo &ai) {
    return ai.n_full == 0 && ai.n_chunks <= (uint64_t)kSmallMaxK * kWave;
}

// Chunks per lane of a small array's body (0 if it has none).
__host__ __device__ inline uint32_t small_chunks_per_lane(const ArrayInfo &ai) {
    return (uint32_t)((ai.n_chunks + kWave - 1u) / kWave);
}

// The chunks-per-lane bound a small-array launch is built for: 1, 2, 4, 8
// or kSmallMaxK.
inline uint32_t small_k_class(uint32_t k) { return k <= 1u ? 1u : k <= 2u ? 2u : k <= 4u ? 4u : k <= 8u ? 8u : kSmallMaxK; }

// The tile walk's two short paths for a small array (body of k <= K chunks
// per lane, no whole tile): at most one chunk per lane goes with the edge
// chunk through one half adder; more go through the carry-save network,
// which leaves the count in binary in bit_length(k + 1) planes.  Returns
// lane L = count at address position L.
template <int K>
__device__ __forceinline__ uint32_t wave_count_small(const uint4 *body, uint64_t n_chunks, uint4 edge,
                                                     bool has_edge) {
    const uint32_t lane = __lane_id();
    uint4 p[kPlanes];
#pragma unroll
    for (int e = 0; e < kPlanes; ++e) p[e] = zero4();
    if (n_chunks <= (uint64_t)kWave) {
        uint4 v = zero4();
        if (lane < n_chunks) v = body[lane];
        p[0] = make_uint4(v.x ^ edge.x, v.y ^ edge.y, v.z ^ edge.z, v.w ^ edge.w);
        p[1] = make_uint4(v.x & edge.x, v.y & edge.y, v.z & edge.z, v.w & edge.w);
        return reduce_planes<4>(p);
    }
    const uint32_t k = (uint32_t)((n_chunks + kWave - 1u) / kWave);
    uint4 v[kLoadsPerTile];
#pragma unroll
    for (int j = 0; j < kLoadsPerTile; ++j) {
        const uint64_t idx = (uint64_t)j * kWave + lane;
        v[j] = (j < K && idx < n_chunks) ? body[idx] : zero4();
    }
    Planes pl;
    pl.a1 = edge;
    pl.a2 = pl.a4 = pl.a8 = zero4();
    (void)pl.csa16(v);
    p[0] = pl.a1;
    p[1] = pl.a2;
    p[2] = pl.a4;
    p[3] = pl.a8;
    // k <= 14 and the edge chunk: at most 15 inputs per bit, four planes
    return bit_length(k + (has_edge ? 1u : 0u)) <= 2u ? reduce_planes<4>(p) : reduce_planes<6>(p);
}

// One small array on one wave: its head/tail bytes and body are counted
// and folded into its counters (what run_item_of does for its one item).
template <int K>
__device__ __forceinline__ void run_small_array(const ArrayInfo &ai) {
    const uint32_t lane = __lane_id();
    const bool has_edge = ai.edge0_len + ai.edge1_len > 0u;
    uint4 edge = zero4();
    if (lane < 32) {
        if (lane < ai.edge0_len) edge = byte_as_chunk((uint64_t)(ai.edge0 + lane), ai.edge0[lane]);
    } else if (lane - 32 < ai.edge1_len) {
        edge = byte_as_chunk((uint64_t)(ai.edge1 + (lane - 32)), ai.edge1[lane - 32]);
    }
    const uint32_t acc = wave_count_small<K>(ai.body, ai.n_chunks, edge, has_edge);
    fold_add(acc, ai.width, ai.m, ai.counts);
}

// Enqueues the small-array kernel over the `n` array indices at idx_dev,
// every one a small array with at most k_max chunks per lane.
hipError_t launch_small_arrays(const ArrayInfo *arrays_dev, const uint32_t *idx_dev, uint32_t n, uint32_t k_max,
                               int cus, hipStream_t st);

// Appends the work items of array `idx` (tiles split into pieces of at most
// `tiles_per_item`).
void append_items(std::vector<WorkItem> &items, const ArrayInfo &ai, uint32_t idx, uint32_t tiles_per_item);

// Sorts items largest first (longest-processing-time order).
void sort_items_lpt(std::vector<WorkItem> &items);

// Groups consecutive items (in LPT order) into units of work handed out by
// one ticket: a group closes when its cost (tiles + 1 per item for the
// per-item reduction) reaches `cost`, or when it holds kGroupMax items or,
// if `waves` is not 0, ceil(items / waves) items, whichever is fewer.  So a
// large item is a group of its own and tiny ones travel together, and a
// batch of few items spreads over every wave, each with one group and no
// ticket.  The server uses kServedGroupCost (p99 at half load 190-200 us
// spread over its grid, instead of 220-320 us); plans kPlanGroupCost
// (65,536 arrays of 1 KiB: 55 against 121 us per run with cost 16; arrays
// of 64 KiB or more: the same).  Returns the n_groups + 1 start indices.
constexpr uint32_t kServedGroupCost = 16;
constexpr uint32_t kPlanGroupCost = 32;
constexpr uint32_t kGroupMax = 64;
std::vector<uint32_t> build_groups(const std::vector<WorkItem> &items, uint32_t waves, uint32_t cost);

// Enqueues the persistent kernel on `st`, preceded by a cursor reset when
// the cursor is used.  Wave g of the grid starts with group g; further
// groups come from the cursor, which the kernel touches only when there
// are more groups than the grid's waves.
hipError_t launch_batched(const ArrayInfo *arrays_dev, const WorkItem *items_dev, const uint32_t *groups_dev,
                          uint32_t n_groups, uint32_t *cursor_dev, uint32_t waves, hipStream_t st);

// Captures the fixed launch sequence of one server stream into a graph:
// copy the batch tables (sizes read from the header) from pinned host
// memory to the device, run the persistent kernel over them, then copy the
// first n_arrays * 64 counters to pinned host memory, clear them and reset
// the cursor for the next batch.  Per batch the host only fills the staging
// buffer and launches the graph.
hipError_t capture_served_graph(hipGraph_t *graph, hipGraphExec_t *exec, const uint8_t *stage_host,
                                uint8_t *stage_dev, size_t items_off, size_t groups_off,
                                unsigned long long *counts_dev, uint64_t *results_host, uint32_t *cursor_dev,
                                uint32_t waves);

// The same three kernels launched directly on `st` (no graph).
hipError_t enqueue_served_batch(hipStream_t st, const uint8_t *stage_host, uint8_t *stage_dev, size_t items_off,
                                size_t groups_off, unsigned long long *counts_dev, uint64_t *results_host,
                                uint32_t *cursor_dev, uint32_t waves);

}  // namespace ppc
