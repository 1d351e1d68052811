// ppc_plain.hip -- the plain single-array pospopcnt call and the read
// roofline kernel for gfx950.
//
// Algorithm (Section 4 of the paper, re-laid out for a GPU):
//   head/tail  : bytes before the first and after the last 16-byte aligned
//                chunk are loaded one per lane by wave 0 and entered as
//                single-byte chunks (head processing, Section 4.1; tail,
//                Section 4.6).  Nothing outside [buf, buf+nbytes) is read.
//   main loop  : each wave walks tiles of 64 lanes x 16 chunks (16 KiB); per
//                tile every lane runs the CSA_{16+4} network (Section 4.2)
//                and adds the weight-16 plane to a bit-sliced counter
//                (the role of the intermediate accumulation, Section 4.3).
//   overflow   : a segment holds at most 63 tiles so the 6-plane bit-sliced
//                counter cannot overflow (Section 4.4's flush rule, with the
//                bound fixed at compile time instead of tracked at run time).
//   final acc. : planes -> 64 integer counts per wave by cross-lane
//                transposes and popcounts (Section 4.5).
//   f_w        : per-block LDS partials are folded to w positions relative
//                to `buf` and added to `counts` with 64-bit atomics.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

#include "ppc.h"
#include "ppc_device.hpp"
#include "ppc_host.hpp"

namespace ppc {

struct PlainArgs {
    const uint4 *body;          // first full 16-byte chunk
    uint64_t n_chunks;          // full chunks in the body
    uint32_t n_full_tiles;      // tiles whose 1024 chunks are all in the body
    uint32_t n_tiles;           // n_full_tiles, + 1 if a partial tile remains
    const uint8_t *edge0;       // head bytes (lanes 0..31 of wave 0)
    const uint8_t *edge1;       // tail bytes (lanes 32..63 of wave 0)
    uint32_t edge0_len, edge1_len;
    unsigned long long *counts; // w uint64 counters (one for the total popcount)
    uint32_t width;             // 8, 16, 32, 64; 0 = total popcount
    uint32_t m;                 // slot of buf's first byte subtracted from address slots (mod w/8)
};

// WPB: waves per block.  Loads are streaming (non-temporal): each byte is
// read once, and against inputs in DRAM the streaming hint is never slower
// (up to 20 % faster on inputs of a few MiB, ~10 % on long streams) than the
// cached policies.  Each wave walks tiles gw, gw + nw, ... (nw = waves in
// the grid), so one load instruction of a wave reads 1 KiB and the 16 loads
// of a tile 16 KiB, all contiguous; at any moment the grid works on one
// contiguous window.
// kTotal: the total popcount (width 0); each lane returns its share of the
// total rather than a position's count, and the fold sums the lanes.
template <int WPB, bool kTotal = false>
__global__ __launch_bounds__(WPB *kWave) void pospop_plain_kernel(PlainArgs a) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wib = wave_in_block();
    const uint32_t gw = blockIdx.x * WPB + wib;
    const uint32_t nw = gridDim.x * WPB;

    uint4 edge = zero4();
    if (gw == 0) {  // head and tail bytes, one per lane, read bytewise
        if (lane < 32) {
            if (lane < a.edge0_len) edge = byte_as_chunk((uint64_t)(a.edge0 + lane), a.edge0[lane]);
        } else if (lane - 32 < a.edge1_len) {
            edge = byte_as_chunk((uint64_t)(a.edge1 + (lane - 32)), a.edge1[lane - 32]);
        }
    }
    const uint32_t acc =
        wave_count_tiles<kTotal, true>(a.body, a.n_chunks, a.n_full_tiles, gw, a.n_tiles, nw, edge, gw == 0);

    __shared__ uint32_t part[WPB][kWave];
    part[wib][lane] = acc;
    __syncthreads();
    if (wib == 0) {  // block sum per address position, then f_w and the atomics
        uint64_t v = 0;
#pragma unroll
        for (int wv = 0; wv < WPB; ++wv) v += part[wv][lane];
        fold_add(v, a.width, a.m, a.counts);
    }
}

// Read roofline: same tiles, same streaming loads and the same next-tile
// prefetch as the pospopcnt kernel; sums the 64-bit words instead of
// counting bits.
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void load_tile_u64(u64x2 (&v)[kLoadsPerTile], const uint4 *p) {
#pragma unroll
    for (int j = 0; j < kLoadsPerTile; ++j) {
        v[j] = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(p + j * kWave));
        __builtin_amdgcn_sched_barrier(0);  // issue order = chunk order, as in load_tile
    }
}

template <int WPB>
__global__ __launch_bounds__(WPB *kWave) void read_roofline_kernel(const uint4 *body, uint32_t n_tiles,
                                                                   unsigned long long *sink) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t gw = blockIdx.x * WPB + wave_in_block();
    const uint32_t nw = gridDim.x * WPB;
    u64x2 acc = {0, 0};
    const uint32_t n_mine = gw < n_tiles ? (n_tiles - gw + nw - 1) / nw : 0u;
    auto tile_ptr = [&](uint32_t i) { return body + (uint64_t)(gw + i * nw) * kTileChunks + lane; };
    if (n_mine > 0) {
        u64x2 va[kLoadsPerTile], vb[kLoadsPerTile];
        load_tile_u64(va, tile_ptr(0));
        uint32_t i = 0;
        while (i + 2u < n_mine) {
            load_tile_u64(vb, tile_ptr(i + 1u));
            __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the math
#pragma unroll
            for (int j = 0; j < kLoadsPerTile; ++j) acc += va[j];
            load_tile_u64(va, tile_ptr(i + 2u));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < kLoadsPerTile; ++j) acc += vb[j];
            i += 2u;
        }
        if (i + 1u < n_mine) {
            load_tile_u64(vb, tile_ptr(i + 1u));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < kLoadsPerTile; ++j) acc += va[j] + vb[j];
        } else {
#pragma unroll
            for (int j = 0; j < kLoadsPerTile; ++j) acc += va[j];
        }
    }
    __shared__ uint64_t part[WPB][kWave];
    part[wave_in_block()][lane] = acc.x + acc.y;
    __syncthreads();
    if (wave_in_block() == 0) {
        uint64_t b = 0;
#pragma unroll
        for (int wv = 0; wv < WPB; ++wv) b += part[wv][lane];
        fold_add(b, 0u, 0u, sink);
    }
}

// ---- host side -----------------------------------------------------------
// Launch geometry set by ppc_set_plain_geometry, packed into one word so a
// call reads a consistent pair: low 32 bits = wave cap (0 = default), high
// 32 bits = waves per block.
static std::atomic<uint64_t> g_plain_geom{(uint64_t)8 << 32};

// Launch events: when given, the start/stop events are recorded by the
// kernel dispatch itself (hipExtLaunchKernel), so their interval is the
// kernel's own execution time.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

static hipError_t launch_plain(const PlainArgs &a, unsigned blocks, unsigned wpb, hipStream_t st, LaunchEvents ev) {
    if (a.width == 0u) {
        if (wpb == 2)
            hipExtLaunchKernelGGL((pospop_plain_kernel<2, true>), dim3(blocks), dim3(128), 0, st, ev.start, ev.stop, 0, a);
        else if (wpb == 4)
            hipExtLaunchKernelGGL((pospop_plain_kernel<4, true>), dim3(blocks), dim3(256), 0, st, ev.start, ev.stop, 0, a);
        else
            hipExtLaunchKernelGGL((pospop_plain_kernel<8, true>), dim3(blocks), dim3(512), 0, st, ev.start, ev.stop, 0, a);
        return hipGetLastError();
    }
    if (wpb == 2)
        hipExtLaunchKernelGGL((pospop_plain_kernel<2>), dim3(blocks), dim3(128), 0, st, ev.start, ev.stop, 0, a);
    else if (wpb == 4)
        hipExtLaunchKernelGGL((pospop_plain_kernel<4>), dim3(blocks), dim3(256), 0, st, ev.start, ev.stop, 0, a);
    else
        hipExtLaunchKernelGGL((pospop_plain_kernel<8>), dim3(blocks), dim3(512), 0, st, ev.start, ev.stop, 0, a);
    return hipGetLastError();
}

// Default grid: one 8-wave block on each of three quarters of the compute
// units (192 blocks on MI355X's 256 CUs).  Measured on DRAM-resident inputs
// of 32 MiB to 1 GiB, 192 blocks stream 2-4 % faster than 256 (1 GiB:
// ~7.2 TB/s against ~6.95), and the read-only kernel gains the same, so the
// gain is in the memory system, not in the counting.  The same number of
// waves spread over every CU (6 per CU in 2-wave blocks) is slower than
// either, so a streaming CU wants its two waves per SIMD, and the
// likeliest reading is that fewer requesting CUs contend less on the way
// to the HBM while still keeping it busy.
PlainGeometry plain_geometry(int device) {
    const uint64_t g = g_plain_geom.load(std::memory_order_relaxed);
    PlainGeometry geo{(unsigned)g, (unsigned)(g >> 32)};
    if (geo.waves == 0) geo.waves = std::max(1u, (unsigned)device_cus(device) * 3u / 4u) * 8u;
    return geo;
}

unsigned full_grid_wave_cap(int device) {
    const unsigned w = (unsigned)g_plain_geom.load(std::memory_order_relaxed);
    if (w) return w;
    return (unsigned)device_cus(device) * 8u;  // one 8-wave block per CU
}

// One launch over a range the caller has sized with kMaxTilesPerWave.
// `geo` is the geometry the caller sized the range with: the grid holds
// min(tiles, geo.waves) waves or more, so no wave gets more tiles than the
// caller allowed for.
static ppc_status plain_launch_range(unsigned width, uint64_t *counts, const uint8_t *buf, size_t nbytes,
                                     uint32_t m, PlainGeometry geo, hipStream_t st, LaunchEvents ev) {
    const uintptr_t b0 = (uintptr_t)buf;
    const uintptr_t b1 = b0 + nbytes;
    const uintptr_t f = (b0 + 15u) & ~(uintptr_t)15u;  // first full chunk
    const uintptr_t e = b1 & ~(uintptr_t)15u;           // end of full chunks
    PlainArgs a{};
    a.counts = reinterpret_cast<unsigned long long *>(counts);
    a.width = width;
    a.m = m;
    if (f < e) {
        a.body = reinterpret_cast<const uint4 *>(f);
        a.n_chunks = (uint64_t)(e - f) / 16u;
        a.edge0 = buf;
        a.edge0_len = (uint32_t)(f - b0);
        a.edge1 = reinterpret_cast<const uint8_t *>(e);
        a.edge1_len = (uint32_t)(b1 - e);
    } else {  // fewer than two chunk boundaries: every byte is an edge byte
        a.body = nullptr;
        a.n_chunks = 0;
        a.edge0 = buf;
        a.edge0_len = (uint32_t)nbytes;  // <= 30
        a.edge1 = nullptr;
        a.edge1_len = 0;
    }
    a.n_full_tiles = (uint32_t)(a.n_chunks / kTileChunks);
    a.n_tiles = (uint32_t)((a.n_chunks + kTileChunks - 1) / kTileChunks);
    const uint64_t waves = std::min<uint64_t>(std::max<uint32_t>(a.n_tiles, 1u), geo.waves);
    const unsigned blocks = (unsigned)((waves + geo.wpb - 1) / geo.wpb);
    return launch_plain(a, blocks, geo.wpb, st, ev) == hipSuccess ? PPC_OK : PPC_EDEVICE;
}

// Per-wave counts are 32-bit: a wave adds at most 64 lanes x 2 dwords x 16
// chunks = 2^11 per position per tile, so no wave may own more than 2^20
// tiles in one launch (2^31 < 2^32).  Launches are cut so that
// tiles <= waves x 2^20, and at 1 TiB to keep tile indices in 32 bits.
static constexpr uint64_t kMaxTilesPerWave = 1ull << 20;
static constexpr size_t kMaxLaunchBytes = (size_t)1 << 40;

// Positions are counted relative to a stream start `offset` bytes before
// buf: byte buf[b] feeds slot (offset + b) mod s.  Address slot a of byte
// buf[b] is (buf + b) mod 8, so the fold subtracts m = (buf - offset) mod s.
ppc_status plain_pospopcnt_at(unsigned width, uint64_t *counts, const void *buf, size_t nbytes, uint64_t offset,
                              hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop) {
    if (!(width == 0 || width == 8 || width == 16 || width == 32 || width == 64)) return PPC_EINVAL;
    if (counts == nullptr || ((uintptr_t)counts & 7u) != 0) return PPC_EINVAL;
    if (nbytes == 0) return PPC_OK;
    if (buf == nullptr) return PPC_EINVAL;
    const uint8_t *p = static_cast<const uint8_t *>(buf);
    const uint32_t s = width ? width / 8u : 1u;
    const uint32_t m = (uint32_t)(((uintptr_t)p - (uintptr_t)(offset % 8u) + 8u) % s);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PPC_EDEVICE;
    const PlainGeometry geo = plain_geometry(dev);  // one read: pieces and grids agree
    const size_t tile_bytes = (size_t)kTileChunks * 16u;
    const size_t piece = std::min<size_t>(kMaxLaunchBytes, (size_t)geo.waves * kMaxTilesPerWave * tile_bytes);
    size_t done = 0;
    while (done < nbytes) {  // pieces start at multiples of 8 from buf: same m
        const size_t len = std::min(piece, nbytes - done);
        LaunchEvents ev;  // start on the first launch, stop on the last
        if (done == 0) ev.start = ev_start;
        if (done + len == nbytes) ev.stop = ev_stop;
        ppc_status rc = plain_launch_range(width, counts, p + done, len, m, geo, st, ev);
        if (rc != PPC_OK) return rc;
        done += len;
    }
    return PPC_OK;
}

ppc_status plain_pospopcnt(unsigned width, uint64_t *counts, const void *buf, size_t nbytes, hipStream_t st) {
    if (width == 0) return PPC_EINVAL;
    return plain_pospopcnt_at(width, counts, buf, nbytes, 0, st, nullptr, nullptr);
}

}  // namespace ppc

using namespace ppc;

extern "C" {

ppc_status ppc_pospopcnt(unsigned width, uint64_t *counts, const void *buf, size_t nbytes, void *stream) {
    return plain_pospopcnt(width, counts, buf, nbytes, (hipStream_t)stream);
}
ppc_status ppc_pospopcnt8(uint64_t *counts, const void *buf, size_t nbytes, void *stream) {
    return plain_pospopcnt(8, counts, buf, nbytes, (hipStream_t)stream);
}
ppc_status ppc_pospopcnt16(uint64_t *counts, const void *buf, size_t nbytes, void *stream) {
    return plain_pospopcnt(16, counts, buf, nbytes, (hipStream_t)stream);
}
ppc_status ppc_pospopcnt32(uint64_t *counts, const void *buf, size_t nbytes, void *stream) {
    return plain_pospopcnt(32, counts, buf, nbytes, (hipStream_t)stream);
}
ppc_status ppc_pospopcnt64(uint64_t *counts, const void *buf, size_t nbytes, void *stream) {
    return plain_pospopcnt(64, counts, buf, nbytes, (hipStream_t)stream);
}

ppc_status ppc_pospopcnt_at(unsigned width, uint64_t *counts, const void *buf, size_t nbytes,
                            uint64_t stream_offset, void *stream) {
    if (width == 0) return PPC_EINVAL;
    return plain_pospopcnt_at(width, counts, buf, nbytes, stream_offset, (hipStream_t)stream, nullptr, nullptr);
}

ppc_status ppc_pospopcnt_timed(unsigned width, uint64_t *counts, const void *buf, size_t nbytes, void *stream,
                               void *start_event, void *stop_event) {
    if (width == 0) return PPC_EINVAL;
    return plain_pospopcnt_at(width, counts, buf, nbytes, 0, (hipStream_t)stream, (hipEvent_t)start_event,
                              (hipEvent_t)stop_event);
}

ppc_status ppc_popcount(uint64_t *total, const void *buf, size_t nbytes, void *stream) {
    return plain_pospopcnt_at(0, total, buf, nbytes, 0, (hipStream_t)stream, nullptr, nullptr);
}

ppc_status ppc_set_plain_geometry(unsigned waves, unsigned waves_per_block) {
    if (!(waves_per_block == 2 || waves_per_block == 4 || waves_per_block == 8)) return PPC_EINVAL;
    if (waves > (1u << 24)) return PPC_EINVAL;
    g_plain_geom.store((uint64_t)waves | ((uint64_t)waves_per_block << 32));
    return PPC_OK;
}

ppc_status ppc_get_plain_geometry(unsigned *waves, unsigned *waves_per_block) {
    if (!waves || !waves_per_block) return PPC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PPC_EDEVICE;
    const PlainGeometry geo = plain_geometry(dev);
    *waves = geo.waves;
    *waves_per_block = geo.wpb;
    return PPC_OK;
}

ppc_status ppc_read_roofline_timed(uint64_t *sink, const void *buf, size_t nbytes, void *stream,
                                   void *start_event, void *stop_event) {
    if (sink == nullptr || ((uintptr_t)sink & 7u) != 0) return PPC_EINVAL;
    if (nbytes == 0) return PPC_OK;
    if (buf == nullptr || ((uintptr_t)buf & 15u) != 0 || (nbytes & 15u) != 0) return PPC_EINVAL;
    if (nbytes % ((size_t)kTileChunks * 16u) != 0) return PPC_EINVAL;  // whole tiles only
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PPC_EDEVICE;
    const uint64_t n_tiles64 = nbytes / ((size_t)kTileChunks * 16u);
    if (n_tiles64 >= (1ull << 32)) return PPC_EINVAL;
    const uint32_t n_tiles = (uint32_t)n_tiles64;
    const PlainGeometry geo = plain_geometry(dev);
    const unsigned wpb = geo.wpb;
    const uint64_t waves = std::min<uint64_t>(n_tiles, geo.waves);
    const unsigned blocks = (unsigned)((waves + wpb - 1) / wpb);
    hipStream_t st = (hipStream_t)stream;
    const uint4 *body = static_cast<const uint4 *>(buf);
    auto *out = reinterpret_cast<unsigned long long *>(sink);
    hipEvent_t e0 = (hipEvent_t)start_event, e1 = (hipEvent_t)stop_event;
    if (wpb == 2)
        hipExtLaunchKernelGGL(read_roofline_kernel<2>, dim3(blocks), dim3(128), 0, st, e0, e1, 0, body, n_tiles, out);
    else if (wpb == 4)
        hipExtLaunchKernelGGL(read_roofline_kernel<4>, dim3(blocks), dim3(256), 0, st, e0, e1, 0, body, n_tiles, out);
    else
        hipExtLaunchKernelGGL(read_roofline_kernel<8>, dim3(blocks), dim3(512), 0, st, e0, e1, 0, body, n_tiles, out);
    return hipGetLastError() == hipSuccess ? PPC_OK : PPC_EDEVICE;
}

ppc_status ppc_read_roofline(uint64_t *sink, const void *buf, size_t nbytes, void *stream) {
    return ppc_read_roofline_timed(sink, buf, nbytes, stream, nullptr, nullptr);
}

}  // extern "C"
