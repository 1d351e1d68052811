// ppc_noalloc.hip -- the batched count for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// Same arithmetic as the batched plan (the per-wave tile walk of the plain
// call over work items, f_w per item, 64-bit atomics into each array's
// counters), but the descriptor table is the caller's, in device memory, and
// every table the kernels need lives in one file-scope device array,
// `scratch`, of fixed size:
//   [0, 512)                      header: work cursor, walk grid, item size,
//                                 the item table's segments
//   [512, 512 + 64 * 2^16)        one ArrayInfo per array (at most 2^16)
//   [.., + 128 * 256)             per-block partial sums of the setup kernels
//   [.., + 16 * 2^18)             work items (at most 2^18), largest first
// Setup on the device, one thread per array: for at most 256 arrays one
// kernel, else three (array table and block sums; walk grid, item size and
// per-block item counts; item offsets and the items themselves), then the
// persistent kernel that walks the items, then, for a batch of short
// arrays, the plan's small-array kernel pattern over the arrays shorter
// than one tile (they then get no work items; see is_small_array).  Nothing is allocated and nothing is copied
// from the host, so the call can be captured.
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
// Tiles per whole item P: about kNaItemsPerWave items per wave of the walk
// (total tiles / (kNaItemsPerWave * waves)), kept within
// [kNaMinItemTiles, kNaMaxItemTilesBal].  Each item ends in a drain of the
// wave's loads, a plane reduction and w atomics, so few large items per wave
// run fastest as long as every wave has one; 256 tiles (4 MiB) is the
// plan's tuned size for large mixed batches.  P is raised above that only
// when the table would need more than kNaMaxItems items, which takes more
// than 768 GiB of input in one call.
constexpr uint32_t kNaItemsPerWave = 1;
constexpr uint32_t kNaMinItemTiles = 4;
constexpr uint32_t kNaMaxItemTilesBal = 256;
// Shorter items (one per array at most: its tiles past the last whole item,
// or only its head/tail bytes) go into buckets by their tile count (two
// per bit length, see na_bucket), and are laid out largest bucket
// first: the largest-first order of the plan, without a sort.  The whole
// items and each bucket form one segment of the table.  A ticket hands out
// a run of items of one segment, a power of two of them: as many as make
// about kNaGroupTiles tiles at the segment's smallest item size (32 items
// of at most one tile, 8 of 4-7 tiles, one of 32 or more), so that short
// items do not queue one by one on the cursor; but at most items / walking
// waves, so that a small batch still spreads over every wave, and halved
// while the segment would make between one and two tickets per wave (the
// second round would leave most waves idle).
constexpr int kNaBuckets = 16;
constexpr int kNaSegments = kNaBuckets + 1;  // [0]: whole items, [1 + (kNaBuckets - 1 - b)]: bucket b
constexpr uint32_t kNaGroupTiles = 32;
constexpr int kNaSetupThreads = 256;
constexpr int kNaSetupWaves = kNaSetupThreads / kWave;
constexpr uint32_t kNaMaxBlocks = kNaMaxArrays / kNaSetupThreads;
static_assert(kNaMaxBlocks <= (uint32_t)kNaSetupThreads, "one thread per setup block in the block scans");
constexpr int kNaWpb = 4;
// The walk launches kNaWavesPerCuSmall waves per CU.  All of them walk when
// the arrays are short (fewer than kNaShortMeanTiles tiles per array on
// average), where each item is a chain of dependent memory accesses and
// more waves hide more of that latency; otherwise only the first
// kNaWavesPerCu per CU do and the rest exit at once, so each SIMD streams
// with one wave, which is faster for long items.
constexpr uint32_t kNaWavesPerCu = 4;
constexpr uint32_t kNaWavesPerCuSmall = 8;
constexpr uint64_t kNaShortMeanTiles = 4;

// One segment of the item table: items [item0, item0 + count), handed out
// `group` per ticket from ticket ticket0 on.
struct NaSegment {
    uint32_t ticket0, item0, count, group;
};

struct NaHeader {
    uint32_t cursor;     // tickets handed out after each wave's first
    uint32_t n_items;    // all items
    uint32_t n_tickets;  // sum over segments of ceil(count / group)
    uint32_t tiles_per_item;
    uint32_t ok;         // 1: every descriptor valid and the items fit the table
    uint32_t n_bad;      // invalid descriptors
    uint32_t waves;      // waves of the walk that take tickets
    uint32_t small_apart;  // 1: arrays shorter than one tile get no items; noalloc_small_kernel counts them
    NaSegment seg[kNaSegments];
    uint32_t reserved[52];
};
static_assert(sizeof(NaHeader) == 512, "header size");

// Sums of one setup block: its invalid descriptors and tiles (first setup
// kernel), its item counts per bucket and its whole items (second).
struct NaPartial {
    uint64_t tiles;
    uint32_t bad;
    uint32_t cnt[kNaBuckets + 1];  // [0, kNaBuckets): buckets, [kNaBuckets]: whole items
    uint32_t pad[12];
};
static_assert(sizeof(NaPartial) == 128, "partial size");

constexpr size_t kNaArraysOff = sizeof(NaHeader);
constexpr size_t kNaPartOff = kNaArraysOff + (size_t)kNaMaxArrays * sizeof(ArrayInfo);
constexpr size_t kNaItemsOff = kNaPartOff + (size_t)kNaMaxBlocks * sizeof(NaPartial);
constexpr size_t kNaScratchBytes = kNaItemsOff + (size_t)kNaMaxItems * sizeof(WorkItem);
static_assert(kNaScratchBytes == PPC_NOALLOC_SCRATCH_BYTES, "scratch size in the header");

static __device__ __align__(256) uint8_t scratch[kNaScratchBytes];

// Exclusive prefix sums over the block's threads of K values at once:
// within each wave by lane shuffles (six steps, no barrier), then the four
// wave totals through LDS.  total[k] receives the sum of value k over the
// block.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const T y = __shfl_up(x, (unsigned)d, kWave);
        if (lane >= (uint32_t)d) x += y;
    }
    return x;
}

template <typename T, int K>
__device__ __forceinline__ void block_exclusive_scan(T (&v)[K], T (*lds)[kNaSetupWaves], T (&total)[K]) {
    constexpr int kWaves = kNaSetupWaves;
    const uint32_t lane = __lane_id(), wave = threadIdx.x / kWave;
    T incl[K];
#pragma unroll
    for (int k = 0; k < K; ++k) incl[k] = wave_inclusive_scan(v[k]);
    if (lane == kWave - 1)
#pragma unroll
        for (int k = 0; k < K; ++k) lds[k][wave] = incl[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        T before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const T s = lds[k][w];
            before += (uint32_t)w < wave ? s : T(0);
            all += s;
        }
        total[k] = all;
        v[k] = before + incl[k] - v[k];
    }
    __syncthreads();
}

// 0..3 tiles: buckets 0..3; above, two buckets per bit length L >= 3, split
// by the bit below the top one (4-5, 6-7, 8-11, 12-15, ...), so that
// bucket order is within a factor 1.5 of size order.
__device__ __forceinline__ int na_bucket(uint32_t t) {
    if (t < 4u) return (int)t;
    const uint32_t L = bit_length(t);
    return (int)min(4u + 2u * (L - 3u) + ((t >> (L - 2u)) & 1u), (uint32_t)(kNaBuckets - 1));
}

// log2 of the smallest item size in bucket b < kNaBuckets, rounded down.
__device__ __forceinline__ uint32_t na_bucket_lg_min(int b) {
    return b < 4 ? (b >= 2 ? 1u : 0u) : (uint32_t)(b - 4) / 2u + 2u;
}

// Slots of one array's items within its setup block's share of the table:
// its whole items take `whole` consecutive slots of the block's whole items
// from f_whole on, its shorter item (if any; b >= 0) slot f_rest of the
// block's bucket b.  The slots are claimed with atomics on the block's
// per-bucket counters in LDS, so their order within a block and bucket is
// arbitrary (counts do not depend on the order of items).
struct NaSlots {
    uint32_t whole, f_whole;
    int b;
    uint32_t f_rest;
};

__device__ __forceinline__ NaSlots na_claim(const ArrayInfo &ai, uint32_t P, bool small_apart, uint32_t *bucket_cnt) {
    if (small_apart && is_small_array(ai)) return NaSlots{0u, 0u, -1, 0u};  // noalloc_small_kernel counts it
    const bool edges = ai.edge0_len + ai.edge1_len > 0u;
    const uint32_t rest = ai.n_tiles % P;
    NaSlots sl{ai.n_tiles / P, 0u, -1, 0u};
    if (sl.whole != 0u) sl.f_whole = atomicAdd(&bucket_cnt[kNaBuckets], sl.whole);
    if (rest != 0u || (ai.n_tiles == 0u && edges)) {
        sl.b = na_bucket(rest);
        sl.f_rest = atomicAdd(&bucket_cnt[sl.b], 1u);
    }
    return sl;
}

// Thread i <-> array i: validates descriptor i and writes its table entry
// (an invalid one gets an empty entry).  Returns the entry; *bad and *tiles
// receive whether it was invalid and its tile count.
__device__ __forceinline__ ArrayInfo na_array_entry(const ppc_desc *__restrict__ descs, uint32_t n, uint32_t i,
                                                    ArrayInfo *arrays, uint32_t &bad, uint64_t &tiles) {
    ArrayInfo ai{};
    bad = 0u;
    tiles = 0u;
    if (i < n) {
        const ppc_desc d = descs[i];
        if (d.reserved != 0u || !make_array_info(ai, d.buf, d.nbytes, d.counts, d.width)) {
            bad = 1u;
            ai = ArrayInfo{};
        }
        arrays[i] = ai;
        tiles = ai.n_tiles;
    }
    return ai;
}

struct NaChoice {
    uint32_t waves;    // walking waves
    uint32_t P;        // tiles per whole item
    bool ok;           // every descriptor valid and the items fit the table
    bool small_apart;  // short batch: its arrays shorter than one tile go to noalloc_small_kernel
};

// Walking waves and item size for T tiles over n arrays on `cus` CUs.
__device__ __forceinline__ NaChoice na_choose(uint64_t T, uint32_t n_bad, uint32_t n, uint32_t cus) {
    // every array gives at most n_tiles/P + 1 items, so P >= T / (kNaMaxItems
    // - n) keeps the total within the table
    const uint64_t room = (uint64_t)kNaMaxItems - n;
    const bool short_batch = T < kNaShortMeanTiles * n;
    const uint32_t waves = (short_batch ? kNaWavesPerCuSmall : kNaWavesPerCu) * max(cus, 1u);
    const uint64_t per_wave = (uint64_t)kNaItemsPerWave * waves;
    const uint64_t bal =
        min(max((T + per_wave - 1) / per_wave, (uint64_t)kNaMinItemTiles), (uint64_t)kNaMaxItemTilesBal);
    const uint64_t p64 = max(bal, (T + room - 1) / room);
    return NaChoice{waves, (uint32_t)min(p64, (uint64_t)kMaxItemTiles), n_bad == 0u && p64 <= (uint64_t)kMaxItemTiles,
                    short_batch};
}

// Start of each bucket's items in the table (whole items first, then the
// buckets from the largest down) from the totals; returns the item count.
__device__ __forceinline__ uint32_t na_layout(const uint32_t (&tot)[kNaBuckets + 1], uint32_t (&base)[kNaBuckets + 1]) {
    base[kNaBuckets] = 0u;
    uint32_t next = tot[kNaBuckets];
    for (int k = kNaBuckets - 1; k >= 0; --k) {
        base[k] = next;
        next += tot[k];
    }
    return next;
}

// Writes array i's items: its whole items from slot f_whole on, its
// shorter item (if sl.b >= 0) at slot f_rest; the array's first item
// carries its head/tail bytes.
__device__ __forceinline__ void na_write_items(const ArrayInfo &ai, uint32_t i, uint32_t P, const NaSlots &sl,
                                               uint32_t f_whole, uint32_t f_rest, WorkItem *items) {
    const uint32_t edges = ai.edge0_len + ai.edge1_len > 0u ? 1u : 0u;
    for (uint32_t k = 0; k < sl.whole; ++k) items[f_whole + k] = WorkItem{i, k * P, (k + 1u) * P, k == 0u ? edges : 0u};
    if (sl.b >= 0) items[f_rest] = WorkItem{i, sl.whole * P, ai.n_tiles, sl.whole == 0u ? edges : 0u};
}

// The header for the walk, by the 64 lanes of a block's first wave: lane j
// builds segment j (whole items for j = 0, then the buckets from the
// largest down) from the item totals per bucket in LDS, with its group size,
// and wave prefix sums give each segment's first item and first ticket.
// If `base_out` is given, the first item of each bucket goes there (LDS).
// Also reports invalid descriptors.
__device__ void na_write_header(NaHeader *h, const uint32_t *tot, const NaChoice &c, uint32_t n_bad, uint32_t n,
                                uint32_t *n_invalid_out, uint32_t *base_out) {
    const uint32_t j = __lane_id();
    const bool seg = j < (uint32_t)kNaSegments;
    const int b = seg ? kNaBuckets - (int)j : 0;  // this lane's bucket (kNaBuckets: whole items)
    const uint32_t count = seg && c.ok ? tot[b] : 0u;
    const uint32_t incl = wave_inclusive_scan(count);
    const uint32_t base = incl - count;
    const uint32_t n_items = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    if (seg && base_out) base_out[b] = base;
    // group sizes are powers of two (log2 below), so this needs no division
    // past the one for the cap
    const uint32_t nw = max(c.waves, 1u);
    const uint32_t cap = n_items / nw;
    const uint32_t lg_cap = cap == 0u ? 0u : bit_length(cap) - 1u;
    const uint32_t lg_target = bit_length(kNaGroupTiles) - 1u;
    // log2 of the segment's smallest item size, rounded down (P is at least 4)
    const uint32_t lg_min = b == kNaBuckets ? bit_length(c.P) - 1u : na_bucket_lg_min(b);
    uint32_t lg_g = min(lg_target > lg_min ? lg_target - lg_min : 0u, lg_cap);
    while (lg_g > 0u) {
        const uint32_t k = (count + (1u << lg_g) - 1u) >> lg_g;
        if (k <= nw || k >= 2u * nw) break;
        --lg_g;
    }
    const uint32_t tickets = (count + (1u << lg_g) - 1u) >> lg_g;
    const uint32_t t_incl = wave_inclusive_scan(tickets);
    if (seg) h->seg[j] = NaSegment{t_incl - tickets, base, count, 1u << lg_g};
    if (j == 0) {
        h->cursor = 0u;
        h->n_items = n_items;
        h->n_tickets = (uint32_t)__builtin_amdgcn_readlane((int)t_incl, kWave - 1);
        h->tiles_per_item = c.P;
        h->ok = c.ok ? 1u : 0u;
        h->n_bad = n_bad;
        h->waves = c.waves;
        h->small_apart = c.small_apart ? 1u : 0u;
        if (n_invalid_out) *n_invalid_out = c.ok ? 0u : (n_bad ? n_bad : n);
    }
}

// ---- setup kernels ---------------------------------------------------------

// Batches of at most kNaSetupThreads arrays: one block does every step.
__global__ __launch_bounds__(kNaSetupThreads) void noalloc_setup_one_block_kernel(const ppc_desc *__restrict__ descs,
                                                                                  uint32_t n, uint32_t cus,
                                                                                  uint32_t *n_invalid_out,
                                                                                  uint8_t *scr) {
    NaHeader *h = reinterpret_cast<NaHeader *>(scr);
    ArrayInfo *arrays = reinterpret_cast<ArrayInfo *>(scr + kNaArraysOff);
    WorkItem *items = reinterpret_cast<WorkItem *>(scr + kNaItemsOff);
    __shared__ uint64_t lds64[1][kNaSetupWaves];
    __shared__ uint32_t lds32[1][kNaSetupWaves];
    __shared__ uint32_t bucket_cnt[kNaBuckets + 1], lbase[kNaBuckets + 1];
    const uint32_t i = threadIdx.x;
    if (i <= (uint32_t)kNaBuckets) bucket_cnt[i] = 0u;
    uint32_t bad[1];
    uint64_t tiles[1];
    const ArrayInfo ai = na_array_entry(descs, n, i, arrays, bad[0], tiles[0]);
    uint32_t n_bad[1];
    uint64_t T[1];
    block_exclusive_scan<uint32_t, 1>(bad, lds32, n_bad);  // its barriers also order the zeroing
    block_exclusive_scan<uint64_t, 1>(tiles, lds64, T);
    const NaChoice c = na_choose(T[0], n_bad[0], n, cus);
    NaSlots sl{0u, 0u, -1, 0u};
    if (c.ok && i < n) sl = na_claim(ai, c.P, c.small_apart, bucket_cnt);
    __syncthreads();
    if (i < (uint32_t)kWave) na_write_header(h, bucket_cnt, c, n_bad[0], n, n_invalid_out, lbase);
    __syncthreads();
    if (c.ok && i < n)
        na_write_items(ai, i, c.P, sl, lbase[kNaBuckets] + sl.f_whole, sl.b >= 0 ? lbase[sl.b] + sl.f_rest : 0u, items);
}

// Larger batches, three kernels.  Setup 1, thread i <-> array i: the array
// table entry, and the block's sums of invalid descriptors and tiles.
__global__ __launch_bounds__(kNaSetupThreads) void noalloc_arrays_kernel(const ppc_desc *__restrict__ descs,
                                                                         uint32_t n, uint8_t *scr) {
    ArrayInfo *arrays = reinterpret_cast<ArrayInfo *>(scr + kNaArraysOff);
    NaPartial *part = reinterpret_cast<NaPartial *>(scr + kNaPartOff);
    __shared__ uint64_t lds64[1][kNaSetupWaves];
    __shared__ uint32_t lds32[1][kNaSetupWaves];
    uint32_t bad[1];
    uint64_t tiles[1];
    (void)na_array_entry(descs, n, blockIdx.x * kNaSetupThreads + threadIdx.x, arrays, bad[0], tiles[0]);
    uint32_t sb[1];
    uint64_t st[1];
    block_exclusive_scan<uint32_t, 1>(bad, lds32, sb);
    block_exclusive_scan<uint64_t, 1>(tiles, lds64, st);
    if (threadIdx.x == 0) {
        part[blockIdx.x].bad = sb[0];
        part[blockIdx.x].tiles = st[0];
    }
}

// Setup 2: every block sums the first kernel's block sums (the same totals
// in every block), makes the same choice of walking waves and item size,
// and writes its own item counts per bucket; block 0 records the choice in
// the header.
__global__ __launch_bounds__(kNaSetupThreads) void noalloc_count_kernel(uint32_t n, uint32_t cus, uint8_t *scr) {
    NaHeader *h = reinterpret_cast<NaHeader *>(scr);
    const ArrayInfo *arrays = reinterpret_cast<const ArrayInfo *>(scr + kNaArraysOff);
    NaPartial *part = reinterpret_cast<NaPartial *>(scr + kNaPartOff);
    __shared__ uint64_t lds64[1][kNaSetupWaves];
    __shared__ uint32_t lds32[1][kNaSetupWaves];
    __shared__ uint32_t bucket_cnt[kNaBuckets + 1];
    const uint32_t tid = threadIdx.x, nb = gridDim.x;
    if (tid <= (uint32_t)kNaBuckets) bucket_cnt[tid] = 0u;
    uint32_t bad[1] = {tid < nb ? part[tid].bad : 0u};
    uint64_t tiles[1] = {tid < nb ? part[tid].tiles : 0ull};
    uint32_t n_bad[1];
    uint64_t T[1];
    block_exclusive_scan<uint32_t, 1>(bad, lds32, n_bad);
    block_exclusive_scan<uint64_t, 1>(tiles, lds64, T);
    const NaChoice c = na_choose(T[0], n_bad[0], n, cus);
    const uint32_t i = blockIdx.x * kNaSetupThreads + tid;
    if (c.ok && i < n) (void)na_claim(arrays[i], c.P, c.small_apart, bucket_cnt);
    __syncthreads();
    if (tid <= (uint32_t)kNaBuckets) part[blockIdx.x].cnt[tid] = bucket_cnt[tid];
    if (blockIdx.x == 0 && tid == 0) {
        h->tiles_per_item = c.P;
        h->ok = c.ok ? 1u : 0u;
        h->n_bad = n_bad[0];
        h->waves = c.waves;
        h->small_apart = c.small_apart ? 1u : 0u;
    }
}

// Setup 3: every block scans the blocks' item counts (the same layout in
// every block; within each bucket, blocks in order), then thread i claims
// slots in its block's share again and writes array i's items.  Block 0
// completes the header.
__global__ __launch_bounds__(kNaSetupThreads) void noalloc_items_kernel(uint32_t n, uint32_t *n_invalid_out,
                                                                        uint8_t *scr) {
    NaHeader *h = reinterpret_cast<NaHeader *>(scr);
    const ArrayInfo *arrays = reinterpret_cast<const ArrayInfo *>(scr + kNaArraysOff);
    const NaPartial *part = reinterpret_cast<const NaPartial *>(scr + kNaPartOff);
    WorkItem *items = reinterpret_cast<WorkItem *>(scr + kNaItemsOff);
    __shared__ uint32_t lds32[kNaBuckets + 1][kNaSetupWaves];
    __shared__ uint32_t bucket_cnt[kNaBuckets + 1], start[kNaBuckets + 1], ltot[kNaBuckets + 1];
    const uint32_t tid = threadIdx.x, nb = gridDim.x;
    const NaChoice c{h->waves, h->tiles_per_item, h->ok != 0u, h->small_apart != 0u};
    const uint32_t n_bad = h->n_bad;
    if (tid <= (uint32_t)kNaBuckets) bucket_cnt[tid] = 0u;

    uint32_t blk[kNaBuckets + 1], tot[kNaBuckets + 1], base[kNaBuckets + 1];
#pragma unroll
    for (int k = 0; k <= kNaBuckets; ++k) blk[k] = tid < nb ? part[tid].cnt[k] : 0u;
    block_exclusive_scan<uint32_t, kNaBuckets + 1>(blk, lds32, tot);
    (void)na_layout(tot, base);
    if (tid == blockIdx.x)  // this block's share of each bucket starts here
#pragma unroll
        for (int k = 0; k <= kNaBuckets; ++k) start[k] = base[k] + blk[k];
    if (tid == 0)
#pragma unroll
        for (int k = 0; k <= kNaBuckets; ++k) ltot[k] = tot[k];
    __syncthreads();
    const uint32_t i = blockIdx.x * kNaSetupThreads + tid;
    if (c.ok && i < n) {
        const ArrayInfo ai = arrays[i];
        const NaSlots sl = na_claim(ai, c.P, c.small_apart, bucket_cnt);
        na_write_items(ai, i, c.P, sl, start[kNaBuckets] + sl.f_whole, sl.b >= 0 ? start[sl.b] + sl.f_rest : 0u,
                       items);
    }
    if (blockIdx.x == 0 && tid < (uint32_t)kWave) na_write_header(h, ltot, c, n_bad, n, n_invalid_out, nullptr);
}

// Persistent walk: of the launched waves, the first `waves` (from the
// header) walk and the rest exit.  Wave g starts with ticket g, then takes
// tickets from the cursor once its current one is done; if there are no
// more tickets than walking waves, the first is the only one and the
// cursor is not touched (otherwise every wave's last atomic, which finds
// nothing, queues on the one address at the same moment).  Ticket t
// belongs to the last segment whose first ticket is at most t, and stands
// for the run of that segment's items it numbers.
template <int WPB>
__global__ __launch_bounds__(WPB *kWave) void noalloc_batched_kernel(uint8_t *scr) {
    NaHeader *h = reinterpret_cast<NaHeader *>(scr);
    const ArrayInfo *arrays = reinterpret_cast<const ArrayInfo *>(scr + kNaArraysOff);
    const WorkItem *items = reinterpret_cast<const WorkItem *>(scr + kNaItemsOff);
    const uint32_t n_tickets = (uint32_t)__builtin_amdgcn_readfirstlane((int)h->n_tickets);
    const uint32_t nw = min((uint32_t)__builtin_amdgcn_readfirstlane((int)h->waves), gridDim.x * WPB);
    uint32_t t = blockIdx.x * WPB + wave_in_block();
    if (t >= nw) return;
    // the segment table, read once (the loop's atomics would otherwise make
    // the compiler reload it for every ticket): lane j holds segment j
    const uint32_t lane = __lane_id();
    NaSegment sg{0xffffffffu, 0u, 0u, 1u};
    if (lane < (uint32_t)kNaSegments) sg = h->seg[lane];
    while (t < n_tickets) {
        // the last segment whose first ticket is at most t (segment 0 starts at 0)
        const uint64_t m = __ballot(sg.ticket0 <= t);
        const int j = 63 - __builtin_clzll(m);
        const uint32_t tk0 = (uint32_t)__builtin_amdgcn_readlane((int)sg.ticket0, j);
        const uint32_t it0 = (uint32_t)__builtin_amdgcn_readlane((int)sg.item0, j);
        const uint32_t end = it0 + (uint32_t)__builtin_amdgcn_readlane((int)sg.count, j);
        const uint32_t g = (uint32_t)__builtin_amdgcn_readlane((int)sg.group, j);
        const uint32_t i0 = it0 + (t - tk0) * g;
        const uint32_t i1 = min(i0 + g, end);
        run_items(arrays, items, i0, i1);
        if (n_tickets <= nw) break;
        uint32_t ticket = 0;
        if (__lane_id() == 0u) ticket = atomicAdd(&h->cursor, 1u);
        t = nw + (uint32_t)__builtin_amdgcn_readfirstlane((int)ticket);
    }
}

// The arrays shorter than one tile of a short batch (fewer than
// kNaShortMeanTiles tiles per array on average), which the walk then has
// no items for.  In other batches they stay in the walk, where they fill
// its tail, and this kernel returns at once; so it does if the setup found
// an invalid descriptor.  Wave g of nw owns array entries g, g + nw,
// g + 2 nw, ... (at most 64: the host sizes the grid for it), so that the
// waves work through the table side by side.  Lane l reads entry g + l * nw,
// a ballot marks the small ones with anything to count, and the wave
// counts those in order (the next one's entry is loaded while the current
// array runs).  Built for the largest such array, 14 chunks per lane, at 4
// waves per SIMD.
__global__ __launch_bounds__(kSmallWpb *kWave) __attribute__((amdgpu_waves_per_eu(4, 4))) void
noalloc_small_kernel(const uint8_t *scr, uint32_t n) {
    const NaHeader *h = reinterpret_cast<const NaHeader *>(scr);
    const ArrayInfo *arrays = reinterpret_cast<const ArrayInfo *>(scr + kNaArraysOff);
    const uint32_t nw = gridDim.x * kSmallWpb;
    const uint32_t g = blockIdx.x * kSmallWpb + wave_in_block();
    if (g >= n || __builtin_amdgcn_readfirstlane((int)(h->ok & h->small_apart)) == 0) return;
    const uint64_t mine_idx = (uint64_t)g + (uint64_t)__lane_id() * nw;
    bool mine = false;
    if (mine_idx < n) {
        const ArrayInfo &a = arrays[mine_idx];
        mine = is_small_array(a) && a.n_chunks + a.edge0_len + a.edge1_len > 0u;
    }
    uint64_t m = __ballot(mine);
    if (m == 0u) return;
    uint32_t j = (uint32_t)__builtin_ctzll(m);
    m &= m - 1u;
    ArrayInfo ai = arrays[g + j * nw];
    for (;;) {
        const uint32_t nj = m != 0u ? (uint32_t)__builtin_ctzll(m) : j;
        const ArrayInfo nai = arrays[g + nj * nw];  // the current entry again after the last
        run_small_array<kSmallMaxK>(ai);
        if (m == 0u) break;
        m &= m - 1u;
        j = nj;
        ai = nai;
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
    const uint32_t nb = (n + kNaSetupThreads - 1) / kNaSetupThreads;
    const uint32_t cus = (uint32_t)device_cus(dev);
    const uint32_t waves = kNaWavesPerCuSmall * cus;
    if (nb <= 1) {
        hipLaunchKernelGGL(noalloc_setup_one_block_kernel, dim3(1), dim3(kNaSetupThreads), 0, st, descs, n, cus,
                           n_invalid, scr);
    } else {
        hipLaunchKernelGGL(noalloc_arrays_kernel, dim3(nb), dim3(kNaSetupThreads), 0, st, descs, n, scr);
        hipLaunchKernelGGL(noalloc_count_kernel, dim3(nb), dim3(kNaSetupThreads), 0, st, n, cus, scr);
        hipLaunchKernelGGL(noalloc_items_kernel, dim3(nb), dim3(kNaSetupThreads), 0, st, n, n_invalid, scr);
    }
    if (n > 0) {
        hipLaunchKernelGGL(noalloc_batched_kernel<kNaWpb>, dim3((waves + kNaWpb - 1) / kNaWpb), dim3(kNaWpb * kWave),
                           0, st, scr);
        // one round of resident blocks (4 waves per SIMD) unless that leaves
        // a wave more than 64 array entries, and no wave without one
        const uint32_t per_wave_max = 64u * kSmallWpb;
        const uint32_t sb = std::max<uint32_t>(std::min<uint32_t>(4u * cus, (n + kSmallWpb - 1) / kSmallWpb),
                                               (n + per_wave_max - 1) / per_wave_max);
        hipLaunchKernelGGL(noalloc_small_kernel, dim3(sb), dim3(kSmallWpb * kWave), 0, st, scr, n);
    }
    return hipGetLastError() == hipSuccess ? PPC_OK : PPC_EDEVICE;
}

}  // extern "C"
