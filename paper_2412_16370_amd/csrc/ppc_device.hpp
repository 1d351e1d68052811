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
template <int K1>
struct Planes {
    uint4 a1, a2, a4, a8;
    uint4 b[K1];

    __device__ __forceinline__ void clear() {
        a1 = a2 = a4 = a8 = zero4();
#pragma unroll
        for (int k = 0; k < K1; ++k) b[k] = zero4();
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

    // b += a16 (bit-sliced ripple of half adders).  The caller bounds the
    // number of additions per segment to 2^K1 - 1 so the top carry is 0.
    __device__ __forceinline__ void add16(uint4 c) {
#pragma unroll
        for (int k = 0; k < K1; ++k) {
            uint4 t;
            t.x = b[k].x & c.x; t.y = b[k].y & c.y; t.z = b[k].z & c.z; t.w = b[k].w & c.w;
            b[k].x ^= c.x; b[k].y ^= c.y; b[k].z ^= c.z; b[k].w ^= c.w;
            c = t;
        }
    }

    // One more chunk of weight 1 (used for the head/tail bytes): a ripple
    // through a1..a8 whose carry-out (weight 16) goes into b.
    __device__ __forceinline__ void add1(uint4 v) {
        uint4 *pl[4] = {&a1, &a2, &a4, &a8};
        uint4 c = v;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint4 &p = *pl[k];
            uint4 t;
            t.x = p.x & c.x; t.y = p.y & c.y; t.z = p.z & c.z; t.w = p.w & c.w;
            p.x ^= c.x; p.y ^= c.y; p.z ^= c.z; p.w ^= c.w;
            c = t;
        }
        add16(c);
    }
};

// ---- cross-lane helpers --------------------------------------------------
// ds_swizzle in bit mode: lane j reads lane (j ^ x) inside its 32-lane half.
template <int X>
__device__ __forceinline__ uint32_t swz_xor(uint32_t v) {
    static_assert(X > 0 && X < 32, "xor mask inside a 32-lane group");
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1f | (X << 10));
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// One stage of a 32x32 bit-matrix transpose across the lanes of each 32-lane
// half (the recursive block transpose of Section 4.4, done across lanes
// instead of inside one register).  Row = lane, column = bit.  The rows with
// (row & S) == 0 trade their columns with (col & S) != 0 for the partner's
// columns with (col & S) == 0.
template <int S>
__device__ __forceinline__ uint32_t transpose_stage(uint32_t x, uint32_t take_mask, uint32_t rot) {
    uint32_t partner = swz_xor<S>(x);
    uint32_t t = __builtin_amdgcn_alignbit(partner, partner, rot);  // rotate right
    return (take_mask & t) | (~take_mask & x);
}

// Per-lane constants of transpose_stage<S>.
struct TransposeConsts {
    uint32_t take[5], rot[5];
    __device__ __forceinline__ TransposeConsts() {
        const uint32_t lane = lane_id();
        const uint32_t low_mask[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u,
                                      0x55555555u};
        const uint32_t shift[5] = {16, 8, 4, 2, 1};
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const bool upper = (lane & shift[i]) != 0;
            take[i] = upper ? low_mask[i] : ~low_mask[i];
            rot[i] = upper ? shift[i] : 32u - shift[i];
        }
    }
};

// After the transpose lane r (inside each half) holds column r of the
// 32x32 matrix; its popcount is the number of rows with that bit set.
__device__ __forceinline__ uint32_t column_popcount(uint32_t x, const TransposeConsts &tc) {
    x = transpose_stage<16>(x, tc.take[0], tc.rot[0]);
    x = transpose_stage<8>(x, tc.take[1], tc.rot[1]);
    x = transpose_stage<4>(x, tc.take[2], tc.rot[2]);
    x = transpose_stage<2>(x, tc.take[3], tc.rot[3]);
    x = transpose_stage<1>(x, tc.take[4], tc.rot[4]);
    return __builtin_popcount(x);
}

// End-of-segment reduction of a wave's bit planes into 64 integer counts
// (the final accumulation of Section 4.4, rebuilt for a 64-lane wavefront).
// Returns, in lane L, the number of set bits at address position L summed
// over all lanes and all planes with their weights.  All 64 lanes must be
// active.  E = number of planes, weights 1, 2, 4, ..., 2^(E-1).
//   step A: inside each lane add dword x to z and y to w (same positions),
//           as bit-sliced numbers -> E+1 planes for positions 0..31 (X) and
//           32..63 (Y);
//   step B: lanes L < 32 take X from lane L+32, lanes L >= 32 take Y from
//           lane L-32, and add -> E+2 planes, one dword each;
//   step C: per plane, a 32x32 cross-lane transpose and a popcount.
template <int E>
__device__ __forceinline__ uint32_t wave_position_counts(const uint4 (&p)[E]) {
    uint32_t X[E + 1], Y[E + 1];
    {
        uint32_t cx = 0, cy = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            X[e] = parity3(p[e].x, p[e].z, cx);
            uint32_t ncx = majority3(p[e].x, p[e].z, cx);
            Y[e] = parity3(p[e].y, p[e].w, cy);
            uint32_t ncy = majority3(p[e].y, p[e].w, cy);
            cx = ncx;
            cy = ncy;
        }
        X[E] = cx;
        Y[E] = cy;
    }
    const bool low_half = lane_id() < 32;
    uint32_t Z[E + 2];
    {
        uint32_t c = 0;
#pragma unroll
        for (int e = 0; e <= E; ++e) {
            uint32_t keep = low_half ? X[e] : Y[e];
            uint32_t send = low_half ? Y[e] : X[e];
            uint32_t recv = (uint32_t)__shfl_xor((int)send, 32);
            Z[e] = parity3(keep, recv, c);
            c = majority3(keep, recv, c);
        }
        Z[E + 1] = c;
    }
    const TransposeConsts tc;
    uint32_t total = 0;
#pragma unroll
    for (int e = 0; e < E + 2; ++e) total += column_popcount(Z[e], tc) << e;
    return total;
}

// Bit-plane reduction of one lane's planes, packaged for the kernels.
template <int K1>
__device__ __forceinline__ uint32_t planes_position_counts(const Planes<K1> &pl) {
    uint4 p[4 + K1];
    p[0] = pl.a1;
    p[1] = pl.a2;
    p[2] = pl.a4;
    p[3] = pl.a8;
#pragma unroll
    for (int k = 0; k < K1; ++k) p[4 + k] = pl.b[k];
    return wave_position_counts<4 + K1>(p);
}

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

}  // namespace ppc
