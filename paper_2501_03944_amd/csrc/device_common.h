// Device helpers shared by the MGFWA kernels: the counter-based generator, the
// uniform draw, the search-box mapping and the order-preserving fitness key.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgfwa {

// Stream tag = counter word 3 of every draw.
enum : uint32_t { TAG_INIT = 0, TAG_EXPL = 1, TAG_EXPL_MAP = 2, TAG_GUIDE_MAP = 3, TAG_REINIT = 4 };

// Device control words (int32 array in the workspace).
enum : int { CTRL_GEN = 0, CTRL_DONE = 1, CTRL_DONE_PENDING = 2, CTRL_WORDS = 4 };

struct Box {
    float lb, ub, span;  // span = ub - lb rounded once to binary32
};

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).  Each round
// takes the 64-bit products of counter words 0 and 2 with the two round
// multipliers; the new counter is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0) and
// the key advances by the two Weyl increments between rounds.  Each
// three-way XOR is one gfx950 three-input bit operation (truth table 0x96),
// so a round is two 32x32 -> 64-bit multiplies and two logic instructions.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k.x += 0x9E3779B9u;
            k.y += 0xBB67AE85u;
        }
        // one 32x32 -> 64-bit multiply per product (both halves at once)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c = make_uint4(__builtin_amdgcn_bitop3_b32(hi1, c.y, k.x, 0x96), lo1,
                       __builtin_amdgcn_bitop3_b32(hi0, c.w, k.y, 0x96), lo0);
    }
    return c;
}

// Four words of block (chunk = d/4, row, generation, tag) under the job key.
__device__ __forceinline__ uint4 draw4(uint2 key, uint32_t chunk, uint32_t row, uint32_t t,
                                       uint32_t tag)
{
    return philox4x32_10(make_uint4(chunk, row, t, tag), key);
}

// 24 random bits scaled by 2^-24: exact, in [0, 1 - 2^-24].
__device__ __forceinline__ float u01(uint32_t r)
{
    return (float)(r >> 8) * 0x1p-24f;
}

// Uniform position in the closed box: fma(u, ub - lb, lb) clamped to [lb, ub].
__device__ __forceinline__ float box_uniform(const Box &b, float u)
{
    float v = __builtin_fmaf(u, b.span, b.lb);
    v = v < b.lb ? b.lb : v;
    return v > b.ub ? b.ub : v;
}

// Random mapping of an out-of-box coordinate from its draw u: uniform in the box,
// or (lo non-null) uniform in the population's range lo..hi of that dimension,
// fma(u, hi - lo, lo), clamped into the box.
__device__ __forceinline__ float map_uniform(const Box &b, float u, const float *lo,
                                             const float *hi, int d)
{
    if (!lo) return box_uniform(b, u);
    const float width = hi[d] - lo[d];
    float v = __builtin_fmaf(u, width, lo[d]);
    v = v < b.lb ? b.lb : v;
    return v > b.ub ? b.ub : v;
}

__device__ __forceinline__ bool outside(const Box &b, float v)
{
    return v < b.lb || v > b.ub;
}

// Coordinates 4*chunk .. 4*chunk+3 of explosion spark `row` in generation tn:
// s = fma(amp, 2u - 1, x) per coordinate, an out-of-box coordinate replaced by
// its uniform draw from the mapping stream of the same (chunk, row, generation)
// (into the box, or into the population range plo..phi when given), coordinates
// at or past D zero.  Counter-based: any kernel can regenerate a spark exactly.
__device__ __forceinline__ void explosion_chunk(const float (&x)[4], float amp, uint2 key, int chunk,
                                                uint32_t row, uint32_t tn, const Box &box,
                                                const float *plo, const float *phi, int D,
                                                float (&s)[4])
{
    const uint4 r = draw4(key, (uint32_t)chunk, row, tn, TAG_EXPL);
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
    bool any_out = false;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float v = 2.0f * u01(w[e]) - 1.0f;
        s[e] = __builtin_fmaf(amp, v, x[e]);
        any_out |= outside(box, s[e]);
    }
    if (any_out) {
        const uint4 r2 = draw4(key, (uint32_t)chunk, row, tn, TAG_EXPL_MAP);
        const uint32_t w2[4] = {r2.x, r2.y, r2.z, r2.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (outside(box, s[e])) s[e] = map_uniform(box, u01(w2[e]), plo, phi, 4 * chunk + e);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (4 * chunk + e >= D) s[e] = 0.0f;
}

// Order-preserving 32-bit key of a (NaN-free) fitness value; -0 and +0 share a key.
__device__ __forceinline__ uint32_t fit_key(float y)
{
    uint32_t u = __float_as_uint(y == 0.0f ? 0.0f : y);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// The stored form of a fitness value: NaN becomes +inf.
__device__ __forceinline__ float canon_fitness(float y)
{
    return y != y ? __int_as_float(0x7f800000) : y;
}

// Block index remap so that consecutive logical blocks land on the same XCD
// (hardware dispatches linear block ids round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks)
{
    constexpr int X = 8;
    const int q = nblocks / X, rem = nblocks % X;
    const int xcd = bid % X, pos = bid / X;
    return xcd < rem ? xcd * (q + 1) + pos : rem * (q + 1) + (xcd - rem) * q + pos;
}

}  // namespace mgfwa
