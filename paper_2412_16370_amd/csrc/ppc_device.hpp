// ppc_device.hpp -- device building blocks of the gfx950 pospopcnt kernels.
//
// Data layout.  The input is read as 16-byte vectors ("chunks") at 16-byte
// aligned addresses, one chunk per lane per load, 64 lanes = 1 KiB per wave
// per load instruction.  Inside a chunk, dwords .x and .z cover address
// positions 0..31 (bytes 0-3 and 8-11 of the chunk) and .y and .w cover
// positions 32..63, where the "address position" of bit k of the byte at
// address a is 8*(a mod 8) + k.  The kernels count these 64 address
// positions; the width w and the caller's pointer are applied only when the
// counts are folded into the output (the accumulation function f_w of
// Section 4).
//
// Per lane, chunks are compressed into bit planes with bit-parallel full
// adders (Section 3.1) arranged as a 16-input carry-save adder network
// (Section 3.2, the CSA_{16+4} step of Section 4): planes a1, a2, a4, a8 are
// carried from tile to tile and every 16 chunks emit one plane of weight 16.
// gfx950's v_bitop3_b32 evaluates any 3-input bitwise function, so a full
// adder is two instructions (parity 0x96, majority 0xe8), as with the
// ternary-logic variant of Eq. (lut).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppc {

constexpr int kWave = 64;          // lanes per wavefront (CDNA)
constexpr int kLoadsPerTile = 16;  // chunks per lane per CSA16 step
constexpr int kTileChunks = kWave * kLoadsPerTile;  // 1024 chunks = 16 KiB

__device__ __forceinline__ uint32_t parity3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t majority3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xe8);
}

// Full adder on 128-bit vectors: (carry, sum) = FA(a, b, c), Eq. (lut).
__device__ __forceinline__ void full_add(uint4 &carry, uint4 &sum, uint4 a, uint4 b, uint4 c) {
    sum.x = parity3(a.x, b.x, c.x);
    sum.y = parity3(a.y, b.y, c.y);
    sum.z = parity3(a.z, b.z, c.z);
    sum.w = parity3(a.w, b.w, c.w);
    carry.x = majority3(a.x, b.x, c.x);
    carry.y = majority3(a.y, b.y, c.y);
    carry.z = majority3(a.z, b.z, c.z);
    carry.w = majority3(a.w, b.w, c.w);
}

__device__ __forceinline__ uint4 zero4() { return make_uint4(0u, 0u, 0u, 0u); }

// Bit-plane accumulators of one lane: a1..a8 carry between tiles (the 4-bit
// accumulator of Section 3.2); b[k] counts weight-16 planes in binary, so the
// whole is one bit-sliced number with planes {a1,a2,a4,a8,b0,b1,...}.
// A segment holds at most 2^kMaxK1 - 1 tiles, so b never overflows.
constexpr int kMaxK1 = 6;
constexpr uint32_t kSegTiles = (1u << kMaxK1) - 1u;  // 63 tiles = 1008 KiB per wave
constexpr int kPlanes = 4 + kMaxK1;
// A wave whose only data is a partial tile of at most kFewChunks chunks per
// lane (and an edge chunk) skips the top counter: 14 + 1 inputs per bit fit
// the four carry-save planes.
constexpr uint32_t kFewChunks = 14;

struct Planes {
    uint4 a1, a2, a4, a8;
    uint4 b[kMaxK1];

    __device__ __forceinline__ void clear() {
        a1 = a2 = a4 = a8 = zero4();
#pragma unroll
        for (int k = 0; k < kMaxK1; ++k) b[k] = zero4();
    }

    // CSA_{16+4}: (a1,a2,a4,a8) + 16 vectors -> (a16, a1,a2,a4,a8), 15 full
    // adders in the Harley-Seal arrangement (pairs -> twos -> fours ->
    // eights -> sixteens).
    __device__ __forceinline__ uint4 csa16(const uint4 (&v)[kLoadsPerTile]) {
        uint4 twosA, twosB, foursA, foursB, eightsA, eightsB, sixteens;
        full_add(twosA, a1, a1, v[0], v[1]);
        full_add(twosB, a1, a1, v[2], v[3]);
        full_add(foursA, a2, a2, twosA, twosB);
        full_add(twosA, a1, a1, v[4], v[5]);
        full_add(twosB, a1, a1, v[6], v[7]);
        full_add(foursB, a2, a2, twosA, twosB);
        full_add(eightsA, a4, a4, foursA, foursB);
        full_add(twosA, a1, a1, v[8], v[9]);
        full_add(twosB, a1, a1, v[10], v[11]);
        full_add(foursA, a2, a2, twosA, twosB);
        full_add(twosA, a1, a1, v[12], v[13]);
        full_add(twosB, a1, a1, v[14], v[15]);
        full_add(foursB, a2, a2, twosA, twosB);
        full_add(eightsB, a4, a4, foursA, foursB);
        full_add(sixteens, a8, a8, eightsA, eightsB);
        return sixteens;
    }

    // b += a16 as the k-th addition of the segment (k = 1..kSegTiles): the
    // counter is then at most k < 2^depth with depth = bit length of k, so
    // the half-adder ripple stops at plane depth-1 with a zero carry.
    // `depth` is wave-uniform: the skipped planes cost scalar branches only.
    __device__ __forceinline__ void add16(uint4 c, uint32_t depth) {
#pragma unroll
        for (int k = 0; k < kMaxK1; ++k) {
            if ((uint32_t)k < depth) {
                uint4 t;
                t.x = b[k].x & c.x; t.y = b[k].y & c.y; t.z = b[k].z & c.z; t.w = b[k].w & c.w;
                b[k].x ^= c.x; b[k].y ^= c.y; b[k].z ^= c.z; b[k].w ^= c.w;
                c = t;
            }
        }
    }
};

__device__ __forceinline__ uint32_t bit_length(uint32_t k) { return 32u - (uint32_t)__builtin_clz(k | 1u) - (k == 0u ? 1u : 0u); }

// ---- cross-lane helpers --------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// v_permlane16_swap of a value with itself: element 0 keeps rows 0 and 2
// (lanes 0-15, 32-47) and holds the partner's value (lane ^ 16) in rows 1
// and 3; element 1 holds the partner's value in rows 0 and 2 and keeps rows
// 1 and 3.  One VALU instruction, no LDS traffic.
__device__ __forceinline__ auto swap16(uint32_t x) { return __builtin_amdgcn_permlane16_swap(x, x, false, false); }

// Index of the calling wave inside its block, as a wave-uniform (scalar)
// value, so that loops and branches derived from it stay scalar.
__device__ __forceinline__ uint32_t wave_in_block() {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// Partner value for lane ^ S inside a 32-lane half, without the LDS: DPP
// row operations for xor 1 and 2 (quad permutation), xor 4 (a left and a
// right row shift merged per bank) and xor 8 (row rotation by 8);
// v_permlane16_swap for xor 16.
template <int S>
__device__ __forceinline__ uint32_t partner_xor(uint32_t x) {
    if constexpr (S == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
    } else if constexpr (S == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
    } else if constexpr (S == 4) {
        // banks 0 and 2 of each row (lanes 0-3, 8-11) read lane + 4; banks 1 and
        // 3 (lanes 4-7, 12-15) read lane - 4
        const int up = __builtin_amdgcn_mov_dpp((int)x, 0x104, 0xF, 0xF, true);   // row_shl:4
        return (uint32_t)__builtin_amdgcn_update_dpp(up, (int)x, 0x114, 0xF, 0xA, false);  // row_shr:4
    } else if constexpr (S == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, true);  // row_ror:8
    } else {
        static_assert(S == 16, "xor 1, 2, 4, 8 or 16");
        const auto sw = swap16(x);
        return (lane_id() & 16u) ? sw[0] : sw[1];
    }
}

// 32x32 bit-matrix transpose across the lanes of each 32-lane half (the
// recursive block transpose of Section 4.5, done across lanes instead of
// inside one register).  Row = lane, column = bit.  Stage S trades, between
// rows r and r ^ S, the bits whose column has bit S different from the row's
// bit S; the five stages commute and after all of them lane r holds column
// r.  Stages 16 and 8 move whole bytes, so one byte permute (v_perm_b32)
// merges the partner's bytes; stages 4, 2 and 1 rotate the partner's word
// and merge it by a bit mask.
struct TransposeConsts {
    // v_perm_b32 selectors.  Stage 8: bytes 0-3 = own word, 4-7 = partner's.
    // Stage 16 permutes the pair (e1, e0) of swap16, whose own/partner order
    // depends on the row: bytes 0-3 = e0, 4-7 = e1.
    uint32_t sel16, sel8;
    uint32_t take[3], rot[3];  // stages 4, 2, 1
    __device__ __forceinline__ TransposeConsts() {
        const uint32_t lane = lane_id();
        // row bit 4 clear (e0 = own, e1 = partner): keep own bytes 0,1, take
        // the partner's bytes 0,1 as 2,3; set (e0 = partner, e1 = own): take
        // the partner's bytes 2,3 as 0,1, keep own bytes 2,3
        sel16 = (lane & 16u) ? 0x07060302u : 0x05040100u;
        // row bit 3 clear: own bytes 0,2 stay, partner's bytes 0,2 go to 1,3;
        // set: partner's bytes 1,3 go to 0,2, own bytes 1,3 stay
        sel8 = (lane & 8u) ? 0x03070105u : 0x06020400u;
        const uint32_t low_mask[3] = {0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
        const uint32_t shift[3] = {4, 2, 1};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const bool upper = (lane & shift[i]) != 0;
            take[i] = upper ? low_mask[i] : ~low_mask[i];
            rot[i] = upper ? shift[i] : 32u - shift[i];
        }
    }
};

// Merge step of the bit-granular stages: the partner's word rotated so that
// its traded bits land on the own word's traded positions.
__device__ __forceinline__ uint32_t merge_rotated(uint32_t own, uint32_t partner, uint32_t take, uint32_t rot) {
    const uint32_t t = __builtin_amdgcn_alignbit(partner, partner, rot);  // rotate right
    return (take & t) | (~take & own);
}

// Transposes NZ planes stage by stage (every plane's partner fetches of a
// stage are issued before any of them is consumed, so a DPP read never
// waits on the instruction before it), then returns in lane r (inside each
// half) the sum over planes of popcount(column r of plane e) << e.  Every
// partner fetch is a VALU instruction (v_permlane16_swap, DPP): measured
// 0.05-0.15 us faster per 256 MiB launch than LDS-pipe swizzles for the
// xor-16 and xor-4 stages.
template <int NZ>
__device__ __forceinline__ uint32_t transpose_popcount(uint32_t (&z)[NZ], const TransposeConsts &tc) {
    uint32_t t[NZ];
#pragma unroll
    for (int e = 0; e < NZ; ++e) {
        const auto sw = swap16(z[e]);
        z[e] = __builtin_amdgcn_perm(sw[1], sw[0], tc.sel16);
    }
#pragma unroll
    for (int e = 0; e < NZ; ++e) t[e] = partner_xor<8>(z[e]);
#pragma unroll
    for (int e = 0; e < NZ; ++e) z[e] = __builtin_amdgcn_perm(t[e], z[e], tc.sel8);
#pragma unroll
    for (int e = 0; e < NZ; ++e) t[e] = partner_xor<4>(z[e]);
#pragma unroll
    for (int e = 0; e < NZ; ++e) z[e] = merge_rotated(z[e], t[e], tc.take[0], tc.rot[0]);
#pragma unroll
    for (int e = 0; e < NZ; ++e) t[e] = partner_xor<2>(z[e]);
#pragma unroll
    for (int e = 0; e < NZ; ++e) z[e] = merge_rotated(z[e], t[e], tc.take[1], tc.rot[1]);
#pragma unroll
    for (int e = 0; e < NZ; ++e) t[e] = partner_xor<1>(z[e]);
#pragma unroll
    for (int e = 0; e < NZ; ++e) z[e] = merge_rotated(z[e], t[e], tc.take[2], tc.rot[2]);
    uint32_t total = 0;
#pragma unroll
    for (int e = NZ - 1; e >= 0; --e) total = (total << 1) + (uint32_t)__builtin_popcount(z[e]);
    return total;
}

// End-of-segment reduction of a wave's bit planes into 64 integer counts
// (the final accumulation of Section 4.5, rebuilt for a 64-lane wavefront).
// Returns, in lane L, the number of set bits at address position L summed
// over all lanes and planes with their weights.  All 64 lanes must be
// active.  Plane e has weight 2^e; only planes e < NZ - 2 may be nonzero
// (with e_used nonzero planes, NZ >= e_used + 2 planes hold the result).
//   step A: inside each lane add dword x to z and y to w (same positions),
//           as bit-sliced numbers -> planes for positions 0..31 (X) and
//           32..63 (Y), one plane more;
//   step B: lanes L < 32 take X from lane L+32, lanes L >= 32 take Y from
//           lane L-32 (one permlane32 swap per plane), and add -> one plane
//           more again, one dword per plane;
//   step C: the planes are transposed across the lanes of each half and
//           popcounted with their weights.
template <int NZ>
__device__ __forceinline__ uint32_t reduce_planes(const uint4 (&p)[kPlanes]) {
    static_assert(NZ >= 3 && NZ <= kPlanes + 2, "plane count");
    uint32_t X[NZ - 1], Y[NZ - 1];
    {
        uint32_t cx = 0, cy = 0;
#pragma unroll
        for (int e = 0; e < NZ - 1; ++e) {
            const uint4 q = e < kPlanes ? p[e] : zero4();
            X[e] = parity3(q.x, q.z, cx);
            Y[e] = parity3(q.y, q.w, cy);
            const uint32_t ncx = majority3(q.x, q.z, cx);
            const uint32_t ncy = majority3(q.y, q.w, cy);
            cx = ncx;
            cy = ncy;
        }
        // cx, cy are zero here: the sums fit in NZ - 1 planes
    }
    uint32_t Z[NZ];
    {
        uint32_t c = 0;
#pragma unroll
        for (int e = 0; e < NZ - 1; ++e) {
            // after the swap: lo = X (lanes < 32) / Y of lane-32 (lanes >= 32),
            //                 hi = X of lane+32 (lanes < 32) / Y (lanes >= 32)
            const auto sw = __builtin_amdgcn_permlane32_swap(X[e], Y[e], false, false);
            const uint32_t lo = sw[0], hi = sw[1];
            Z[e] = parity3(lo, hi, c);
            c = majority3(lo, hi, c);
        }
        Z[NZ - 1] = c;
    }
    const TransposeConsts tc;
    return transpose_popcount<NZ>(Z, tc);
}

// Dispatch on the number of planes in use (wave-uniform): planes
// e >= e_used are zero and are not processed.
__device__ __forceinline__ uint32_t wave_position_counts(const uint4 (&p)[kPlanes], uint32_t e_used) {
    if (e_used <= 2u) return reduce_planes<4>(p);
    if (e_used <= 4u) return reduce_planes<6>(p);
    if (e_used <= 6u) return reduce_planes<8>(p);
    if (e_used <= 8u) return reduce_planes<10>(p);
    return reduce_planes<kPlanes + 2>(p);
}

__device__ __forceinline__ uint32_t planes_position_counts(const Planes &pl, uint32_t b_used) {
    uint4 p[kPlanes];
    p[0] = pl.a1;
    p[1] = pl.a2;
    p[2] = pl.a4;
    p[3] = pl.a8;
#pragma unroll
    for (int k = 0; k < kMaxK1; ++k) p[4 + k] = pl.b[k];
    return wave_position_counts(p, 4u + b_used);
}

// For the total popcount only: the lane's planes popcounted with their
// weights, sum over e of 2^e * popcount(plane e) (the Harley-Seal total of
// Section 3.3), with no cross-lane step.  The caller sums the lanes.  Planes
// e >= e_used are zero and are skipped.
__device__ __forceinline__ uint32_t lane_total(const uint4 (&p)[kPlanes], uint32_t e_used) {
    uint32_t t = 0;
#pragma unroll
    for (int e = 0; e < kPlanes; ++e) {
        if ((uint32_t)e < e_used) {
            const uint32_t c = (uint32_t)__builtin_popcount(p[e].x) + (uint32_t)__builtin_popcount(p[e].y) +
                               (uint32_t)__builtin_popcount(p[e].z) + (uint32_t)__builtin_popcount(p[e].w);
            t += c << e;
        }
    }
    return t;
}

__device__ __forceinline__ uint32_t planes_lane_total(const Planes &pl, uint32_t b_used) {
    uint4 p[kPlanes];
    p[0] = pl.a1;
    p[1] = pl.a2;
    p[2] = pl.a4;
    p[3] = pl.a8;
#pragma unroll
    for (int k = 0; k < kMaxK1; ++k) p[4 + k] = pl.b[k];
    return lane_total(p, 4u + b_used);
}

// Streaming (non-temporal) 16-byte load: the input is read exactly once, so
// it is marked as not worth keeping in the caches.
__device__ __forceinline__ uint4 load_stream(const uint4 *p) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 r = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    return make_uint4(r.x, r.y, r.z, r.w);
}

// The 16 loads of a tile are issued in chunk order (the scheduling barrier
// keeps the compiler from reordering them).  Loads complete in issue order,
// so the carry-save network, which takes the chunks in that order, can start
// on the first pairs while the rest are in flight: the compiler's wait counts
// step down two loads at a time instead of waiting for nearly the whole tile.
// That matters for the last tile of each wave, whose compression is on the
// kernel's critical path (256 MiB: -0.5 us; it also frees 25 VGPRs).
__device__ __forceinline__ void load_tile(uint4 (&v)[kLoadsPerTile], const uint4 *p) {
#pragma unroll
    for (int j = 0; j < kLoadsPerTile; ++j) {
        v[j] = load_stream(p + j * kWave);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One wave's share of a body of 16-byte chunks: tiles t0, t0+stride, ... that
// are < t_end.  Tiles below n_full are whole (1024 chunks); the tile n_full,
// if walked, is the partial last tile and its loads are predicated on
// chunk < n_chunks.  `edge` is one extra weight-1 chunk (head/tail bytes,
// zero if none).  Returns lane L = count at address position L.
//
// Software pipeline: two register sets take turns, and the steady-state
// loop issues the next tile's 16 loads unconditionally before compressing
// the current tile, so the compiler's wait counts let those loads stay in
// flight (a conditional load there makes it wait for them).  The last one
// or two whole tiles are peeled off after the loop.
//
// kColdShortPaths: the caller's waves almost always hold whole tiles (the
// plain call), so the two short paths below are laid out after the main
// loop instead of between the set-up and the first tile loads (16-64 MiB:
// 0.05 us per launch).  The batched walk, whose small items take the short
// paths often, keeps them in line.
#define PPC_SHORT_PATH(c) (kColdShortPaths ? __builtin_expect((c), 0) : (c))
template <bool kTotal = false, bool kColdShortPaths = false>
__device__ __forceinline__ uint32_t wave_count_tiles(const uint4 *body, uint64_t n_chunks, uint32_t n_full,
                                                     uint32_t t0, uint32_t t_end, uint32_t stride, uint4 edge,
                                                     bool has_edge) {
    const uint32_t lane = __lane_id();
    const uint32_t full_end = t_end < n_full ? t_end : n_full;
    // number of whole tiles this wave walks (wave-uniform)
    const uint32_t n_mine = t0 < full_end ? (full_end - t0 + stride - 1) / stride : 0u;
    {
        // Short path (the transpose-then-popcount idea of the paper's future
        // work): when the wave holds at most one chunk per lane -- no whole
        // tile, and a partial tile of at most 64 chunks or none -- the
        // carry-save front end is skipped.  The lane's chunk and its edge
        // chunk form a 2-plane bit-sliced number (half adder) that goes
        // straight into the cross-lane transposes and popcounts.
        const uint32_t t = t0 + n_mine * stride;
        const bool walks_partial = t < t_end && t == n_full && (uint64_t)n_full * kTileChunks < n_chunks;
        const uint64_t partial_chunks = walks_partial ? n_chunks - (uint64_t)n_full * kTileChunks : 0u;
        if (PPC_SHORT_PATH(n_mine == 0 && partial_chunks <= (uint64_t)kWave)) {
            if (!walks_partial && !has_edge) return 0u;
            uint4 v = zero4();
            if (walks_partial && lane < partial_chunks) v = body[(uint64_t)n_full * kTileChunks + lane];
            uint4 p[kPlanes];
#pragma unroll
            for (int e = 0; e < kPlanes; ++e) p[e] = zero4();
            p[0] = make_uint4(v.x ^ edge.x, v.y ^ edge.y, v.z ^ edge.z, v.w ^ edge.w);
            p[1] = make_uint4(v.x & edge.x, v.y & edge.y, v.z & edge.z, v.w & edge.w);
            return kTotal ? lane_total(p, 2u) : wave_position_counts(p, 2u);
        }
        // A partial tile alone, of k <= kFewChunks chunks per lane: with the
        // edge chunk a bit sees at most 15 inputs, so the carry-save network
        // leaves the lane's count in binary in its four planes (its carry-out
        // is zero), and only the low bit_length(k + 1) planes can be
        // non-zero.  The top counter and the zero planes are skipped: two to
        // four planes go into the reduction instead of five.
        if (PPC_SHORT_PATH(n_mine == 0 && partial_chunks <= (uint64_t)kFewChunks * kWave)) {
            const uint32_t k = (uint32_t)((partial_chunks + kWave - 1u) / kWave);
            const uint64_t base = (uint64_t)n_full * kTileChunks + lane;
            uint4 v[kLoadsPerTile];
#pragma unroll
            for (int j = 0; j < kLoadsPerTile; ++j) {
                const uint64_t idx = base + (uint64_t)j * kWave;
                v[j] = (uint32_t)j < k && idx < n_chunks ? body[idx] : zero4();
            }
            Planes pl;
            pl.a1 = edge;
            pl.a2 = pl.a4 = pl.a8 = zero4();
            (void)pl.csa16(v);
            uint4 p[kPlanes];
            p[0] = pl.a1;
            p[1] = pl.a2;
            p[2] = pl.a4;
            p[3] = pl.a8;
#pragma unroll
            for (int e = 4; e < kPlanes; ++e) p[e] = zero4();
            const uint32_t e_used = bit_length(k + (has_edge ? 1u : 0u));
            return kTotal ? lane_total(p, e_used) : wave_position_counts(p, e_used);
        }
    }
    Planes pl;
    pl.clear();
    pl.a1 = edge;
    bool any = has_edge;
    uint32_t acc = 0, seg = 0;
    auto tile_ptr = [&](uint32_t i) { return body + (uint64_t)(t0 + i * stride) * kTileChunks + lane; };
    auto add_tile = [&](const uint4 (&v)[kLoadsPerTile]) {
        ++seg;
        pl.add16(pl.csa16(v), bit_length(seg));
    };
    constexpr uint32_t kFlushAt = kSegTiles - 1u;  // even, <= 63: checked once per pair
    if (n_mine > 0) {
        any = true;
        uint4 va[kLoadsPerTile], vb[kLoadsPerTile];
        load_tile(va, tile_ptr(0));
        uint32_t i = 0;
        while (i + 2u < n_mine) {  // tiles i (in va), i+1, i+2 exist
            load_tile(vb, tile_ptr(i + 1u));
            __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the math
            add_tile(va);
            load_tile(va, tile_ptr(i + 2u));
            __builtin_amdgcn_sched_barrier(0);
            add_tile(vb);
            i += 2u;
            if (seg >= kFlushAt) {
                acc += kTotal ? planes_lane_total(pl, kMaxK1) : planes_position_counts(pl, kMaxK1);
                pl.clear();
                seg = 0;
            }
        }
        if (i + 1u < n_mine) {  // two tiles left: i in va, i+1
            load_tile(vb, tile_ptr(i + 1u));
            __builtin_amdgcn_sched_barrier(0);
            add_tile(va);
            add_tile(vb);
        } else {
            add_tile(va);
        }
    }
    uint32_t t = t0 + n_mine * stride;  // first walked tile at or past full_end
    if (t < t_end && t == n_full && (uint64_t)n_full * kTileChunks < n_chunks) {
        uint4 v[kLoadsPerTile];
        const uint64_t base = (uint64_t)t * kTileChunks + lane;
#pragma unroll
        for (int j = 0; j < kLoadsPerTile; ++j) {
            const uint64_t idx = base + (uint64_t)j * kWave;
            v[j] = idx < n_chunks ? body[idx] : zero4();
        }
        add_tile(v);
        any = true;
    }
    if (any) acc += kTotal ? planes_lane_total(pl, bit_length(seg)) : planes_position_counts(pl, bit_length(seg));
    return acc;
}
#undef PPC_SHORT_PATH

// The byte at address `a` (value `byte`) as a chunk holding only that byte
// at its place: dword (a mod 16)/4, bits 8*(a mod 4) .. 8*(a mod 4)+7.
__device__ __forceinline__ uint4 byte_as_chunk(uint64_t a, uint32_t byte) {
    const uint32_t o = (uint32_t)(a & 15u);
    const uint32_t v = byte << (8u * (o & 3u));
    const uint32_t d = o >> 2;
    return make_uint4(d == 0 ? v : 0u, d == 1 ? v : 0u, d == 2 ? v : 0u, d == 3 ? v : 0u);
}

// Output slot of address position P for width w and pointer residue m =
// buf mod (w/8): byte slot ((P/8) - m) mod s, same bit.
__device__ __forceinline__ uint32_t fold_position(uint32_t P, uint32_t w, uint32_t m) {
    const uint32_t s = w >> 3;
    const uint32_t a = P >> 3;
    return 8u * ((a + 8u - m) & (s - 1u)) + (P & 7u);
}

// v + (v of lane ^ S), 64-bit, for all 64 lanes: a permlane32 swap for
// S = 32, the lane exchanges of partner_xor below that.
template <int S>
__device__ __forceinline__ uint64_t add_partner_u64(uint64_t v) {
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    if constexpr (S == 32) {
        // swap(x, x): element 0 and element 1 are, in some order, the own
        // value and that of lane ^ 32
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        return (((uint64_t)h[0] << 32) | l[0]) + (((uint64_t)h[1] << 32) | l[1]);
    } else {
        const uint32_t plo = partner_xor<S>(lo), phi = partner_xor<S>(hi);
        return v + (((uint64_t)phi << 32) | plo);
    }
}

// Adds a wave's 64 position counts (lane L holds address position L) into
// the caller's counters: positions that f_w sends to the same counter are
// summed across lanes first (lane bits 5, 4, 3 select the byte slot), then
// lanes j < w add one counter each.  Width 0 sums everything into
// counts[0] (the total popcount).  All 64 lanes must be active.
__device__ __forceinline__ void fold_add(uint64_t v, uint32_t width, uint32_t m, unsigned long long *counts) {
    const uint32_t lane = __lane_id();
    const uint32_t s = width >> 3;
    if (s <= 4u) v = add_partner_u64<32>(v);
    if (s <= 2u) v = add_partner_u64<16>(v);
    if (s <= 1u) v = add_partner_u64<8>(v);
    if (width == 0u) {
        v = add_partner_u64<4>(v);
        v = add_partner_u64<2>(v);
        v = add_partner_u64<1>(v);
        if (lane == 0u && v != 0u) atomicAdd(counts, (unsigned long long)v);
        return;
    }
    if (lane < width && v != 0u) atomicAdd(counts + fold_position(lane, width, m), (unsigned long long)v);
}

}  // namespace ppc
