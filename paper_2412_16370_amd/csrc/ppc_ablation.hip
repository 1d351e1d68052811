// ppc_ablation.hip -- accumulation-schedule variants of the plain call, for
// measuring what the paper's bit-parallel accumulation buys on a GPU.
//
//   variant 0: the library's path (carry-save front end, bit-parallel
//              accumulation of the weight-16 plane, Sections 4.2-4.5);
//   variant 1: carry-save front end, then every bit of the weight-16 plane
//              added to its own per-lane position counter -- the O(w)
//              accumulation of Klarqvist et al. (Algorithm 2), whose cost
//              grows with the number of positions;
//   variant 2: no carry-save front end: every loaded chunk's bits are added
//              to per-lane position counters (Fig. 2's loop, vectorised over
//              lanes).
// All three compute the same exact counts; only the instruction count per
// byte differs.  Counters of variants 1 and 2 are reduced across the wave by
// a halving butterfly (lane L ends with position L).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ppc.h"
#include "ppc_batch.hpp"
#include "ppc_device.hpp"
#include "ppc_host.hpp"

namespace ppc {

// Per-lane counters of the 64 address positions (dwords .x/.z hold
// positions 0..31, .y/.w positions 32..63).
struct PosCounters {
    uint32_t c[kWave];

    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int j = 0; j < kWave; ++j) c[j] = 0;
    }

    // c[position] += bit << SHIFT for every bit of one 16-byte vector.
    template <int SHIFT>
    __device__ __forceinline__ void add(uint4 v) {
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const uint32_t lo = ((v.x >> j) & 1u) + ((v.z >> j) & 1u);
            const uint32_t hi = ((v.y >> j) & 1u) + ((v.w >> j) & 1u);
            c[j] += lo << SHIFT;
            c[32 + j] += hi << SHIFT;
        }
    }

    // One halving step: the lane with bit S set keeps the upper half of the
    // live counters and receives its partner's upper half; the other lane
    // keeps and receives the lower half.
    template <int S>
    __device__ __forceinline__ void halve(uint32_t lane) {
        const bool up = (lane & (uint32_t)S) != 0;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const uint32_t keep = up ? c[i + S] : c[i];
            const uint32_t send = up ? c[i] : c[i + S];
            c[i] = keep + (uint32_t)__shfl_xor((int)send, S);
        }
    }

    // Sum over the wave's lanes: lane L ends with the total of position L.
    __device__ __forceinline__ uint32_t wave_sum() {
        const uint32_t lane = __lane_id();
        halve<32>(lane);
        halve<16>(lane);
        halve<8>(lane);
        halve<4>(lane);
        halve<2>(lane);
        halve<1>(lane);
        return c[0];
    }
};

template <int VARIANT>
__device__ __forceinline__ uint32_t wave_count_variant(const uint4 *body, uint64_t n_chunks, uint32_t n_full,
                                                       uint32_t t0, uint32_t t_end, uint32_t stride, uint4 edge,
                                                       bool has_edge) {
    const uint32_t lane = __lane_id();
    PosCounters pc;
    pc.clear();
    pc.add<0>(edge);
    uint4 a1 = zero4(), a2 = zero4(), a4 = zero4(), a8 = zero4();
    auto add_tile = [&](const uint4 (&v)[kLoadsPerTile]) {
        if constexpr (VARIANT == 1) {
            Planes pl;
            pl.a1 = a1;
            pl.a2 = a2;
            pl.a4 = a4;
            pl.a8 = a8;
            const uint4 s16 = pl.csa16(v);
            a1 = pl.a1;
            a2 = pl.a2;
            a4 = pl.a4;
            a8 = pl.a8;
            pc.add<4>(s16);
        } else {
            pc.add<0>(v[0]);
            pc.add<0>(v[1]);
            pc.add<0>(v[2]);
            pc.add<0>(v[3]);
            pc.add<0>(v[4]);
            pc.add<0>(v[5]);
            pc.add<0>(v[6]);
            pc.add<0>(v[7]);
            pc.add<0>(v[8]);
            pc.add<0>(v[9]);
            pc.add<0>(v[10]);
            pc.add<0>(v[11]);
            pc.add<0>(v[12]);
            pc.add<0>(v[13]);
            pc.add<0>(v[14]);
            pc.add<0>(v[15]);
        }
    };
    // one tile in registers at a time: these variants are ALU-heavy, so
    // latency is hidden by the other waves rather than by a second buffer
    const uint32_t full_end = t_end < n_full ? t_end : n_full;
    const uint32_t n_mine = t0 < full_end ? (full_end - t0 + stride - 1) / stride : 0u;
    for (uint32_t i = 0; i < n_mine; ++i) {
        const uint4 *p = body + (uint64_t)(t0 + i * stride) * kTileChunks + lane;
        if constexpr (VARIANT == 2) {
            // chunk by chunk with one chunk prefetched: 64 counters plus a
            // whole tile would not fit the register file
            uint4 cur = load_stream(p);
#pragma unroll 1
            for (int j = 0; j < kLoadsPerTile; ++j) {
                const uint4 nxt = j + 1 < kLoadsPerTile ? load_stream(p + (j + 1) * kWave) : zero4();
                pc.add<0>(cur);
                cur = nxt;
            }
        } else {
            uint4 v[kLoadsPerTile];
            load_tile(v, p);
            add_tile(v);
        }
    }
    const uint32_t t = t0 + n_mine * stride;
    if (t < t_end && t == n_full && (uint64_t)n_full * kTileChunks < n_chunks) {
        const uint64_t base = (uint64_t)t * kTileChunks + lane;
        if constexpr (VARIANT == 2) {
#pragma unroll 1
            for (int j = 0; j < kLoadsPerTile; ++j) {
                const uint64_t idx = base + (uint64_t)j * kWave;
                pc.add<0>(idx < n_chunks ? body[idx] : zero4());
            }
        } else {
            uint4 v[kLoadsPerTile];
#pragma unroll
            for (int j = 0; j < kLoadsPerTile; ++j) {
                const uint64_t idx = base + (uint64_t)j * kWave;
                v[j] = idx < n_chunks ? body[idx] : zero4();
            }
            add_tile(v);
        }
    }
    if constexpr (VARIANT == 1) {  // what is left in the 4-bit accumulator
        pc.add<0>(a1);
        pc.add<1>(a2);
        pc.add<2>(a4);
        pc.add<3>(a8);
    }
    (void)has_edge;
    return pc.wave_sum();
}

template <int WPB, int VARIANT>
__global__ __launch_bounds__(WPB *kWave) void pospop_variant_kernel(ArrayInfo ai) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wib = wave_in_block();
    const uint32_t gw = blockIdx.x * WPB + wib;
    const uint32_t nw = gridDim.x * WPB;
    uint4 edge = zero4();
    if (gw == 0) {
        if (lane < 32) {
            if (lane < ai.edge0_len) edge = byte_as_chunk((uint64_t)(ai.edge0 + lane), ai.edge0[lane]);
        } else if (lane - 32 < ai.edge1_len) {
            edge = byte_as_chunk((uint64_t)(ai.edge1 + (lane - 32)), ai.edge1[lane - 32]);
        }
    }
    const uint32_t acc =
        wave_count_variant<VARIANT>(ai.body, ai.n_chunks, ai.n_full, gw, ai.n_tiles, nw, edge, gw == 0);
    __shared__ uint32_t part[WPB][kWave];
    part[wib][lane] = acc;
    __syncthreads();
    if (threadIdx.x < ai.width) {
        const uint32_t s = ai.width >> 3;
        const uint32_t j = threadIdx.x;
        const uint32_t k = j & 7u;
        const uint32_t a0 = ((j >> 3) + ai.m) & (s - 1u);
        unsigned long long sum = 0;
        for (uint32_t slot = a0; slot < 8u; slot += s)
#pragma unroll
            for (int wv = 0; wv < WPB; ++wv) sum += part[wv][8u * slot + k];
        if (sum) atomicAdd(ai.counts + j, sum);
    }
}

}  // namespace ppc

using namespace ppc;

extern "C" ppc_status ppc_pospopcnt_variant(unsigned variant, unsigned width, uint64_t *counts, const void *buf,
                                            size_t nbytes, void *stream) {
    if (variant > 2) return PPC_EINVAL;
    if (variant == 0) return plain_pospopcnt(width, counts, buf, nbytes, (hipStream_t)stream);
    ArrayInfo ai;
    if (!make_array_info(ai, buf, nbytes, counts, width)) return PPC_EINVAL;
    if (nbytes == 0) return PPC_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PPC_EDEVICE;
    constexpr int kWpb = 8;
    const uint64_t waves = std::min<uint64_t>(std::max<uint32_t>(ai.n_tiles, 1u), full_grid_wave_cap(dev));
    const unsigned blocks = (unsigned)((waves + kWpb - 1) / kWpb);
    // a wave adds at most 2^11 per position per tile: keep its 32-bit
    // counts below 2^31 (one launch, no splitting, for this measurement path)
    const uint64_t total_waves = (uint64_t)blocks * kWpb;
    if ((ai.n_tiles + total_waves - 1) / total_waves > (1u << 20)) return PPC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (variant == 1)
        hipLaunchKernelGGL((pospop_variant_kernel<kWpb, 1>), dim3(blocks), dim3(kWpb * kWave), 0, st, ai);
    else
        hipLaunchKernelGGL((pospop_variant_kernel<kWpb, 2>), dim3(blocks), dim3(kWpb * kWave), 0, st, ai);
    return hipGetLastError() == hipSuccess ? PPC_OK : PPC_EDEVICE;
}
