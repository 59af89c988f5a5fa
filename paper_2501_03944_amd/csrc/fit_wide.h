// Fitness kernel for networks whose first layer is too wide to stage per spark
// in LDS (two layers: in -> hidden <= 256 -> out <= 16), e.g. 784-256-10.
//
// The first layer of every spark is a genuine GEMM, H = act(W1 [x; 1]) with the
// bias folded in as an extra input column of ones, so the kernel is a
// persistent, K-streamed GEMM on the matrix cores with the rest of the network
// and the loss fused into its epilogue:
//
//  * tile   = all 256 hidden units x 256 samples of one spark; a block of four
//             wavefronts owns it, each wavefront a 128 x 128 quarter (16 x 16
//             MFMA blocks: 8 x 8 accumulator tiles);
//  * K loop = 32 input columns per step through a ring of LDS stages filled by
//             direct global->LDS loads (global_load_lds_dwordx4).  BF16
//             (k_fit_wide_pipe): a 4-stage ring and one barrier per step; each
//             step refills the stage it consumed with the step 4 ahead and reads
//             the next step's MFMA fragments into the second of two register
//             sets, one load and two fragment reads interleaved with every 8
//             multiplies, so loads, LDS reads and matrix work overlap; a step
//             needs few other instructions (its look-ahead sources come from
//             tile bases set once per tile), since with one wavefront per SIMD
//             they take issue slots from the multiplies.  FP32 (k_fit_wide32):
//             a 2-stage ring of 64 KiB steps and one barrier per step, placed
//             before the step's last row block; the next step's loads are
//             issued in the first quarter of a step's multiplies, each row
//             block's fragment is read one row block ahead and the last row
//             block reads the next step's first fragments.  Past the last tile
//             the look-ahead re-loads the last step (BF16: so its wait counts
//             are constants);
//  * swizzle: a 16-byte chunk c of tile row r lives at chunk c ^ s(r), with
//             s(r) = (r >> 1) & 3 for 64-byte rows (BF16) and r & 7 for 128-byte
//             rows (FP32).  A 16-byte LDS read serves eight lanes at a time,
//             four from each half of the wavefront (lanes i..i+3 and
//             i+32..i+35: here rows 4a..4a+3 with chunks g and g + 2, measured
//             with the bank-conflict counter); for BF16 those eight land in
//             distinct 16-byte bank groups;
//  * epilogue per tile: activation, layer 2 as MFMAs whose B operand is the
//             hidden tile straight from the accumulators, the two hidden halves'
//             logits summed through LDS and stored sample-major, then every lane
//             computes one sample's loss on its own; one partial per (spark,
//             sample tile), reduced later in a fixed order;
//  * schedule: blocks are persistent (one per CU); tile groups of GS sparks go
//             to one XCD, whose blocks split the group's sample tiles round by
//             round (GS sparks x bx/GS sample tiles at a time), so a spark's rows
//             are read by one XCD only, by its blocks at about the same time.
//             A round's operand tiles (4.8 MB at 784-256-10) exceed the XCD's
//             4 MB L2, so every round fetches them once past the L2 (mostly the
//             sample tiles, from the Infinity Cache).
//
// Packed spark layout (written by k_pack_wide_rows, or by the explosion kernel
// for explosion sparks; row pitch PR bytes):
//   [0, 256*Kp*es)          W1aug as [Kp/32][256][32] (K-blocked: the tile of one
//                           K step is 16 or 32 KiB of contiguous memory): W1
//                           (zero-padded), b1 in column `in`
//   [.., + 16*256*es)       W2[16][256]; in BF16 each 32-column block is stored
//                           in the order the MFMA lanes consume it
//   [.., + 16*4)            b2[16] (FP32)
#pragma once

#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

constexpr int WT_M = 256;   // hidden units per tile
constexpr int WT_N = 256;   // samples per tile
constexpr int WT_K = 32;    // input columns per K step
constexpr int WT_NW = 4;    // wavefronts per block

typedef __attribute__((address_space(3))) void lds_void_t;

struct WideArgs {
    const char *Wp;        // packed spark rows
    size_t pr;             // packed row pitch (bytes)
    int rows;
    const char *Xw;        // packed samples, K-blocked per 256-sample tile (kernel element type)
    int Kp, nk;            // padded K and K steps
    int S, S_pad, ntn;     // samples, padded samples, sample tiles
    int fo1;               // output width (<= 16)
    int loss, act;
    const float *Y;        // [S_pad][fo1]
    const int32_t *lab;    // [S_pad]
    float *partial;        // [rows][ntn]
    int gs;                // sparks per XCD tile group
};

constexpr int ZP = 20;      // LDS pitch (floats) of a sample's logits in the loss exchange

template <bool BF>
struct WideCfg {
    static constexpr int ES = BF ? 2 : 4;                  // bytes per element
    static constexpr int ROWB = WT_K * ES;                 // bytes per tile row per K step
    static constexpr int NCH = ROWB / 16;                  // 16-byte chunks per row
    static constexpr int RPL = 64 / NCH;                   // rows per wave load (1 KiB)
    static constexpr int TILEB = WT_M * ROWB;              // bytes of one operand tile
    static constexpr int STAGEB = 2 * TILEB;               // W tile + X tile
    static constexpr int STAGES = 2;                       // FP32 ring (BF16: PipeCfg)
    static constexpr int LOADS = STAGEB / 1024 / WT_NW;    // wave loads per wave per step
    static constexpr int ZX = STAGES * STAGEB;             // logits exchange area
    static constexpr int ZXB = WT_N * ZP * 4;              // logits of the tile's samples
    static constexpr int LDS = ZX + ZXB;
    static constexpr int KMULT = WT_K;                     // padded K is a multiple
};

// BF16 software pipeline: a 4-stage ring; fragments of the next step are read
// from LDS while the current step multiplies.
struct PipeCfg {
    static constexpr int STAGES = 4;
    static constexpr int STAGEB = WideCfg<true>::STAGEB;          // 32 KiB
    static constexpr int LOADS = WideCfg<true>::LOADS;            // 8 per wave per step
    static constexpr int ZX = STAGES * STAGEB;
    static constexpr int LDS = ZX + WideCfg<true>::ZXB;           // 148 KiB
};

__device__ __forceinline__ int wide_swz(int row, int nch)
{
    return nch == 4 ? ((row >> 1) & 3) : (row & 7);
}

// The tile list of a persistent block: groups of gs sparks (gs divides the
// row count) go to XCD (group % 8); the XCD's bx blocks take the group's
// gs * ntn tiles round-robin, so block j handles cj tiles of every group.
// Inside a group, tiles are ordered so that each round of bx consecutive tiles
// covers gs sparks x (bx / gs) sample tiles when that divides evenly (fewer
// distinct weight and sample tiles live in the XCD's L2 at once), else spark by
// spark.
struct TileIter {
    int xcd, j, bx, gs, ntn, rows;
    int cj, ngx, cw;           // tiles per group for this block, groups here, cols per round
    __device__ __forceinline__ void setup()
    {
        const int t = gs * ntn;
        cj = j < t ? (t - 1 - j) / bx + 1 : 0;
        const int ngroups = rows / gs;
        ngx = xcd < ngroups ? (ngroups - 1 - xcd) / 8 + 1 : 0;
        cw = bx / gs;
        // spark by spark otherwise: with cw = ntn a round covers one spark
        if (cw < 1 || bx % gs != 0 || ntn % cw != 0) cw = ntn;
    }
    __device__ __forceinline__ int count() const { return cj * ngx; }
    // i-th tile of this block -> (spark row, sample tile)
    __device__ __forceinline__ void tile(int i, int *r, int *col) const
    {
        const int m = i / cj, ii = i - m * cj;
        const int grp = xcd + 8 * m;
        const int k = j + ii * bx;
        // branch-free: control flow here would split the accumulators' live
        // ranges inside the K loop
        const int cb = k / (gs * cw), rem = k - cb * gs * cw;
        const int sp = rem / cw;
        *r = grp * gs + sp;
        *col = cb * cw + (rem - sp * cw);
    }
};

// Compiler-only fence: no memory access moves across it.
__device__ __forceinline__ void cfence() { asm volatile("" ::: "memory"); }

// Block barrier that orders LDS traffic: this wave's LDS accesses have
// completed (lgkmcnt 0) before it arrives.
__device__ __forceinline__ void lds_barrier()
{
    cfence();
    __builtin_amdgcn_s_waitcnt(0xF | (3 << 14) | (7 << 4));   // lgkmcnt(0), others unconstrained
    __builtin_amdgcn_s_barrier();
    cfence();
}

// All of this wave's LDS reads have completed; the fragments passed through are
// tied to the wait so that nothing uses them earlier.
__device__ __forceinline__ void lgkm_wait_all(bf16x8 (&a)[8], bf16x8 (&b)[8])
{
    asm volatile("s_waitcnt lgkmcnt(0)"
                 : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]),
                   "+v"(a[6]), "+v"(a[7]), "+v"(b[0]), "+v"(b[1]), "+v"(b[2]), "+v"(b[3]),
                   "+v"(b[4]), "+v"(b[5]), "+v"(b[6]), "+v"(b[7]));
}

// Per-lane constants of the pipelined kernel.  The swizzle term of a row that
// a lane touches depends only on the row's low bits, which are the same for
// every row block the lane visits, so one offset per operand serves all of them.
struct PipeLane {
    uint32_t goff;    // lane's byte offset inside a 1 KiB block of 16 rows (global side)
    uint32_t aoff;    // LDS offset of the lane's A fragment of row block 0 (stage-relative)
    uint32_t boff;    // same for the B fragment (X half of the stage)
    int woff;         // byte offset of this wave's first 16-row block of a tile (uniform)
};

__device__ __forceinline__ PipeLane pipe_lane(int wave, int lane, int nh, int sh)
{
    using C = WideCfg<true>;
    const int n = lane & 15, g = lane >> 4;
    const int lr = lane / C::NCH, pc = lane % C::NCH;
    PipeLane L;
    L.goff = (uint32_t)(lr * C::ROWB + ((pc ^ ((lr >> 1) & 3)) << 4));
    const uint32_t fo = (uint32_t)(n * C::ROWB + ((g ^ ((n >> 1) & 3)) << 4));
    L.aoff = (uint32_t)(128 * nh * C::ROWB) + fo;
    L.boff = (uint32_t)(C::TILEB + 128 * sh * C::ROWB) + fo;
    L.woff = wave * (C::LOADS / 2) * C::RPL * C::ROWB;
    return L;
}

// Global sources of the look-ahead loads: K step kt of the current tile, or
// step kt - nk of the next one.  Past the last tile the look-ahead stays on the
// current tile's last step (re-loaded into the free stage, so the wait counts
// are constants).
struct Look {
    const char *wcur, *xcur, *wnext, *xnext;
    int nmask;        // -1 while a next tile exists, else 0
};

template <bool BF = true>
__device__ __forceinline__ void look_set(const WideArgs &a, const TileIter &it, int i, int ntiles,
                                         Look &lk)
{
    using C = WideCfg<BF>;
    int r, col;
    it.tile(i, &r, &col);
    lk.wcur = a.Wp + (size_t)r * a.pr;
    lk.xcur = a.Xw + (size_t)col * a.nk * C::TILEB;
    if (i + 1 < ntiles) {
        it.tile(i + 1, &r, &col);
        lk.wnext = a.Wp + (size_t)r * a.pr;
        lk.xnext = a.Xw + (size_t)col * a.nk * C::TILEB;
        lk.nmask = -1;
    } else {
        lk.wnext = lk.wcur + (size_t)(a.nk - 1) * C::TILEB;
        lk.xnext = lk.xcur + (size_t)(a.nk - 1) * C::TILEB;
        lk.nmask = 0;
    }
}

// Wave load T (of LOADS) of the K step whose W and X blocks start at wsrc and
// xsrc, into an LDS stage: loads 0-3 take this wave's four 1 KiB blocks of the W
// tile, loads 4-7 those of the X tile.  The 16-byte chunks are gathered in
// swizzled order on the global side and land contiguously in LDS.  The block is
// the instruction's immediate offset, which applies to the global and the LDS
// address alike, so the four loads of a tile share one address register and one
// LDS base (M0).
template <int T>
__device__ __forceinline__ void pipe_issue_one(const char *wsrc, const char *xsrc, char *stage,
                                               const PipeLane &L)
{
    using C = WideCfg<true>;
    constexpr int half = T >> 2, blk = (T & 3) * C::RPL * C::ROWB;
    const char *src = (half ? xsrc : wsrc) + L.woff + L.goff;
    char *dst = stage + half * C::TILEB + L.woff;
    __builtin_amdgcn_global_load_lds(src, (lds_void_t *)dst, 16, blk, 0);
}

// All LOADS wave loads of one K step.
template <int T = 0>
__device__ __forceinline__ void pipe_issue_all(const char *wsrc, const char *xsrc, char *stage,
                                               const PipeLane &L)
{
    pipe_issue_one<T>(wsrc, xsrc, stage, L);
    if constexpr (T + 1 < WideCfg<true>::LOADS) pipe_issue_all<T + 1>(wsrc, xsrc, stage, L);
}

// 16-byte LDS read at a lane address plus an immediate offset, issued as an
// instruction the compiler does not track; the caller waits for it with
// lgkm_wait_all before using the value.
template <int OFF>
__device__ __forceinline__ bf16x8 lds_read16_at(uint32_t addr)
{
    bf16x8 v;
    asm volatile("ds_read_b128 %0, %1 offset:%2" : "=v"(v) : "v"(addr), "i"(OFF));
    return v;
}

// Fragments of row block RB of both operands from the stage at LDS address st.
template <int RB>
__device__ __forceinline__ void pipe_read_rb(uint32_t st, const PipeLane &L, bf16x8 &fa, bf16x8 &fb)
{
    fb = lds_read16_at<RB * 16 * WideCfg<true>::ROWB>(st + L.boff);
    fa = lds_read16_at<RB * 16 * WideCfg<true>::ROWB>(st + L.aoff);
}

// Wait until this wave's loads of the next step's stage have landed (the loads
// of the two younger steps may still be in flight), then a block barrier: the
// stage is complete for every wavefront, and every wavefront has finished
// reading the stage that is refilled during this step.
__device__ __forceinline__ void pipe_wait()
{
    constexpr int n = 2 * PipeCfg::LOADS;
    static_assert(n < 64, "vmcnt holds at most 63");
    cfence();
    __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (7 << 4) | (15 << 8));
    __builtin_amdgcn_s_barrier();
    cfence();
}

// The multiply of one accumulator tile in a K step; the first step of a tile
// starts from zero (addend 0), so the accumulators need no clearing between
// tiles.
template <bool FIRST>
__device__ __forceinline__ void mfma_step(floatx4 &c, const bf16x8 &a, const bf16x8 &b)
{
    if constexpr (FIRST) asm("v_mfma_f32_16x16x32_bf16 %0, %1, %2, 0" : "=a"(c) : "v"(a), "v"(b));
    else mfma_acc(c, a, b);
}

// Row block RB of one pipelined K step (register set P holds the step's
// fragments): two fragment reads of the next step into set 1-P, four
// multiplies, one look-ahead load, four multiplies.
template <int P, bool FIRST, int RB>
__device__ __forceinline__ void pipe_rb(uint32_t next, const char *wsrc, const char *xsrc,
                                        char *fill, const PipeLane &L, floatx4 (&acc)[8][8],
                                        bf16x8 (&fa)[2][8], bf16x8 (&fb)[2][8])
{
    pipe_read_rb<RB>(next, L, fa[1 - P][RB], fb[1 - P][RB]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) mfma_step<FIRST>(acc[RB][cb], fa[P][RB], fb[P][cb]);
    __builtin_amdgcn_sched_barrier(0);
    pipe_issue_one<RB>(wsrc, xsrc, fill, L);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int cb = 4; cb < 8; ++cb) mfma_step<FIRST>(acc[RB][cb], fa[P][RB], fb[P][cb]);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (RB + 1 < 8) pipe_rb<P, FIRST, RB + 1>(next, wsrc, xsrc, fill, L, acc, fa, fb);
}

// One pipelined K step: step kt of the tile, global step q.  Refill the stage
// of step q with the step STAGES ahead, read the fragments of step q+1 into set
// 1-P, and run the 64 multiplies of step q.  The per-step address work is a
// handful of scalar operations: the look-ahead sources come from the tile
// bases in lk, the fragment addresses from the per-lane offsets in L.
template <int P, bool FIRST = false>
__device__ __forceinline__ void pipe_step(const WideArgs &a, char *smem, const Look &lk, int kt,
                                          int q, const PipeLane &L, floatx4 (&acc)[8][8],
                                          bf16x8 (&fa)[2][8], bf16x8 (&fb)[2][8])
{
    using C = WideCfg<true>;
    pipe_wait();
    const int la = kt + PipeCfg::STAGES;
    const bool wrap = la >= a.nk;
    const int lo = wrap ? ((la - a.nk) & lk.nmask) : la;
    const char *wsrc = (wrap ? lk.wnext : lk.wcur) + (size_t)lo * C::TILEB;
    const char *xsrc = (wrap ? lk.xnext : lk.xcur) + (size_t)lo * C::TILEB;
    char *fill = smem + (q & (PipeCfg::STAGES - 1)) * PipeCfg::STAGEB;
    const uint32_t next = (uint32_t)(uintptr_t)(lds_void_t *)(smem + ((q + 1) & (PipeCfg::STAGES - 1)) *
                                                                          PipeCfg::STAGEB);
    pipe_rb<P, FIRST, 0>(next, wsrc, xsrc, fill, L, acc, fa, fb);
    lgkm_wait_all(fa[1 - P], fb[1 - P]);
}

// The K steps of one tile whose first step (global step qbase) uses register
// set P0: step kt uses set (P0 + kt) & 1, i.e. the parity of its global step,
// so an odd step count per tile just alternates P0 from tile to tile.
template <int P0>
__device__ __forceinline__ void pipe_tile(const WideArgs &a, char *smem, const Look &lk, int qbase,
                                          const PipeLane &L, floatx4 (&acc)[8][8],
                                          bf16x8 (&fa)[2][8], bf16x8 (&fb)[2][8])
{
    pipe_step<P0, true>(a, smem, lk, 0, qbase, L, acc, fa, fb);
    int kt = 1;
    for (; kt + 1 < a.nk; kt += 2) {
        pipe_step<1 - P0>(a, smem, lk, kt, qbase + kt, L, acc, fa, fb);
        pipe_step<P0>(a, smem, lk, kt + 1, qbase + kt + 1, L, acc, fa, fb);
    }
    if (kt < a.nk) pipe_step<1 - P0>(a, smem, lk, kt, qbase + kt, L, acc, fa, fb);
}

// Layer-2 A fragments of this wave's hidden half, read from the packed row.
template <bool BF>
struct W2Frag {
    floatx4 f[BF ? 4 : 8];     // BF16: 4 x (8 bf16) as raw bits; FP32: 8 x float4
    floatx4 b2;
};

template <bool BF>
__device__ __forceinline__ void w2_load(const WideArgs &a, int r, int nh, int n, int g, W2Frag<BF> &w)
{
    using C = WideCfg<BF>;
    const char *base = a.Wp + (size_t)r * a.pr + (size_t)WT_M * a.Kp * C::ES;
    const char *row = base + (size_t)n * WT_M * C::ES;       // output row n (lane % 16)
    if constexpr (BF) {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
            w.f[kb] = *reinterpret_cast<const floatx4 *>(row + (128 * nh + 32 * kb + 8 * g) * 2);
    } else {
#pragma unroll
        for (int rb = 0; rb < 8; ++rb)
            w.f[rb] = *reinterpret_cast<const floatx4 *>(row + (128 * nh + 16 * rb + 4 * g) * 4);
    }
    const float *b2 = reinterpret_cast<const float *>(base + 16 * WT_M * C::ES);
    w.b2 = *reinterpret_cast<const floatx4 *>(b2 + 4 * g);
}

template <int ACT>
__device__ __forceinline__ floatx4 act4(floatx4 v)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = act_c<ACT>(v[e]);
    return v;
}

// Maximum of three values (no NaN canonicalisation: the operands are finite or
// -inf logits).
__device__ __forceinline__ float vmax3(float a, float b, float c)
{
    float d;
    asm("v_max3_f32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Loss of one sample from its 16 logit slots zz (cross-entropy: slots at or past
// the output width hold -inf): cross-entropy against its label as log-sum-exp
// around the maximum (log1p of the other terms when the label holds the
// maximum), or the squared error summed over the outputs.  FAST takes exp(x) as
// 2^(x log2 e) on the hardware exp2 unit (the BF16 kernels, whose logits carry
// BF16 rounding far above its error).
template <bool FAST>
__device__ __forceinline__ float sample_loss(const WideArgs &a, int s, int label,
                                             const float (&zz)[16])
{
    if (a.loss == 0) {
        const float *y = a.Y + (size_t)s * a.fo1;
        float acc = 0.0f;
#pragma unroll
        for (int o = 0; o < 16; ++o)
            if (o < a.fo1) {
                const float e = zz[o] - y[o];
                acc = __builtin_fmaf(e, e, acc);
            }
        return acc;
    }
    float mx = vmax3(zz[0], zz[1], zz[2]);
#pragma unroll
    for (int o = 3; o < 15; o += 2) mx = vmax3(mx, zz[o], zz[o + 1]);
    mx = vmax3(mx, zz[15], zz[15]);
    float se = 0.0f, rest = 0.0f, zl = 0.0f;
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        const float d = zz[o] - mx;
        const float e = FAST ? __builtin_amdgcn_exp2f(d * 1.44269504088896341f) : expf(d);
        se += e;
        rest += o == label ? 0.0f : e;
        zl = o == label ? zz[o] : zl;
    }
    return zl == mx ? log1pf(rest) : (mx - zl) + logf(se);
}

// Label of the sample this lane scores in the epilogue of tile column col
// (fetched early: its load latency would otherwise sit in the epilogue).
__device__ __forceinline__ int tile_label(const WideArgs &a, int col, int wave, int lane)
{
    const int s = col * WT_N + 64 * wave + lane;
    return (a.loss == 1 && s < a.S) ? a.lab[s] : 0;
}

// Sum of a float over the wavefront, exact in lane 0 (other lanes hold partial
// sums), added in the order of an xor butterfly as lane 0 sees it: pairs and
// quads by quad permutations, 8 and 16 lanes by rotations within each row of
// 16 (lane j takes lane j+4, then j+8), then (row 0 + row 1) + (row 2 + row 3)
// from the rows' first lanes.  All register-to-register: no LDS round trips.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL,
                                                                 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum_lane0(float v)
{
    v = v + dpp_mov<0xB1>(v);     // quad_perm [1,0,3,2]: lane j ^ 1
    v = v + dpp_mov<0x4E>(v);     // quad_perm [2,3,0,1]: lane j ^ 2
    v = v + dpp_mov<0x12C>(v);    // row_ror 12: lane (j + 4) mod 16
    v = v + dpp_mov<0x128>(v);    // row_ror 8: lane (j + 8) mod 16
    const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
    const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
    const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
    return (v + r1) + (r2 + r3);
}

template <bool BF, int ACT>
__device__ void wide_epilogue(const WideArgs &a, char *smem, int r, int col, int wave, int lane,
                              floatx4 (&acc)[8][8], const W2Frag<BF> &w2, float *red, int label,
                              int zx_off = WideCfg<BF>::ZX)
{
    using C = WideCfg<BF>;
    const int n = lane & 15, g = lane >> 4, nh = wave & 1, sh = wave >> 1;
    // layer 2: logits of this wave's hidden half.  The activation of the hidden
    // tile (its bias came in through the ones column) is applied as each
    // accumulator is turned into a layer-2 operand: rewriting all 256
    // accumulators in place first would need them all in VGPRs at once.
    floatx4 z[8][1];
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) z[cb][0] = zero4();
    if constexpr (BF) {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 afr = __builtin_bit_cast(bf16x8, w2.f[kb]);
#pragma unroll
            for (int cb = 0; cb < 8; ++cb) {
                const bf16x8 bfr = ACT == 1 ? relu_to_bf16x8(acc[2 * kb][cb], acc[2 * kb + 1][cb])
                                            : to_bf16x8(act4<ACT>(acc[2 * kb][cb]),
                                                        act4<ACT>(acc[2 * kb + 1][cb]));
                z[cb][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr, z[cb][0], 0, 0, 0);
            }
        }
    } else {
#pragma unroll
        for (int rb = 0; rb < 8; ++rb)
#pragma unroll
            for (int cb = 0; cb < 8; ++cb) {
                const floatx4 h = act4<ACT>(acc[rb][cb]);
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    z[cb][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(w2.f[rb][v], h[v], z[cb][0], 0, 0, 0);
            }
    }
    // the upper hidden half hands its partial logits to the lower half
    float *zx = reinterpret_cast<float *>(smem + zx_off);
    // (block cb of the 64 lanes' 16-byte partials is contiguous: consecutive
    // lanes hit consecutive bank groups)
    float *mine = zx + ((size_t)sh * 8 * 64 + lane) * 4;
    if (nh == 1) {
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) *reinterpret_cast<floatx4 *>(mine + cb * 64 * 4) = z[cb][0];
    }
    lds_barrier();
    if (nh == 0) {
        // cross-entropy: the logit slots past the output width become -inf (their
        // weights and bias are zero), so the loss needs no per-output predicate
        floatx4 b2 = w2.b2;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (a.loss == 1 && 4 * g + v >= a.fo1) b2[v] = -__builtin_huge_valf();
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) {
            const floatx4 o = *reinterpret_cast<const floatx4 *>(mine + cb * 64 * 4);
#pragma unroll
            for (int v = 0; v < 4; ++v) z[cb][0][v] = z[cb][0][v] + o[v] + b2[v];
        }
    }
    lds_barrier();
    // ... which stores them sample-major (lane g of sample n holds outputs 4g..4g+3),
    // so that afterwards every lane of the block owns one sample's logits
    if (nh == 0) {
#pragma unroll
        for (int cb = 0; cb < 8; ++cb)
            *reinterpret_cast<floatx4 *>(zx + (size_t)(128 * sh + 16 * cb + n) * ZP + 4 * g) = z[cb][0];
    }
    lds_barrier();
    const int sl = 64 * wave + lane;                // sample within the tile
    const int s = col * WT_N + sl;
    float ls = 0.0f;
    if (s < a.S) {
        float zz[16];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            const floatx4 v = *reinterpret_cast<const floatx4 *>(zx + (size_t)sl * ZP + 4 * q4);
#pragma unroll
            for (int e = 0; e < 4; ++e) zz[4 * q4 + e] = v[e];
        }
        ls = sample_loss<BF>(a, s, label, zz);
    }
    // fixed-order reduction: the wavefront's sum, then the four wavefronts in order
    ls = wave_sum_lane0(ls);
    if (lane == 0) red[wave] = ls;
    lds_barrier();
    if (threadIdx.x == 0) a.partial[(size_t)r * a.ntn + col] = (red[0] + red[1]) + (red[2] + red[3]);
}

// FP32 pipeline: a 2-stage ring of 32-column K steps (64 KiB each), one barrier
// per step.  A step runs its 512 multiplies (halves kk = 0, 1 of the step's
// columns, each 8 row blocks x 4 columns x 8 column blocks) while it reads every
// row block's A fragment one row block ahead and the second half's B fragments
// during the first half, issues the next step's 16 loads into the other stage
// within the first four row blocks (they have ~10 row blocks, ~4 us, to land),
// and passes the barrier before its last row block, which reads the next step's
// first fragments.  Same tiles, layout, multiply order and results as the
// two-barrier form it replaces; the step's sources come from the tile bases
// (no divisions).
struct Lane32 {
    uint32_t goff;       // lane's byte offset inside a 1 KiB block of 8 rows (global side)
    uint32_t aoff[2];    // LDS offset of the lane's A fragment of row block 0, half kk
    uint32_t boff[2];    // same for the B fragments (X half of the stage)
    int woff;            // byte offset of this wave's first 8-row block of a tile (uniform)
};

__device__ __forceinline__ Lane32 lane32(int wave, int lane, int nh, int sh)
{
    using C = WideCfg<false>;
    static_assert(C::NCH == 8 && C::RPL == 8, "128-byte rows, 8 rows per wave load");
    const int n = lane & 15, g = lane >> 4;
    const int lr = lane / C::NCH, pc = lane % C::NCH;
    Lane32 L;
    // a wave load covers rows r0..r0+7 with r0 a multiple of 8, so the swizzle
    // term of a lane's row is lr; a fragment row 16 cb + n has term n & 7
    L.goff = (uint32_t)(lr * C::ROWB + ((pc ^ lr) << 4));
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        const uint32_t ch = (uint32_t)(((4 * kk + g) ^ (n & 7)) << 4);
        L.aoff[kk] = (uint32_t)((128 * nh + n) * C::ROWB) + ch;
        L.boff[kk] = (uint32_t)(C::TILEB + (128 * sh + n) * C::ROWB) + ch;
    }
    L.woff = wave * (C::LOADS / 2) * C::RPL * C::ROWB;
    return L;
}

// Wave load T (of 16) of a K step: loads 0-7 take this wave's eight 1 KiB
// blocks of the W tile, 8-15 those of the X tile.  Blocks 0-3 and 4-7 of an
// operand each share one address and one LDS base, the block being the
// instruction's immediate offset (which must stay below 4 KiB).
template <int T>
__device__ __forceinline__ void issue32(const char *wsrc, const char *xsrc, char *stage, const Lane32 &L)
{
    using C = WideCfg<false>;
    constexpr int half = T >> 3, blk = T & 7;
    constexpr int hi = (blk >> 2) * 4096, lo = (blk & 3) * 1024;
    const char *src = (half ? xsrc : wsrc) + L.woff + hi + L.goff;
    char *dst = stage + half * C::TILEB + L.woff + hi;
    __builtin_amdgcn_global_load_lds(src, (lds_void_t *)dst, 16, lo, 0);
}

template <int OFF>
__device__ __forceinline__ floatx4 lds_read4_at(uint32_t addr)
{
    floatx4 v;
    asm volatile("ds_read_b128 %0, %1 offset:%2" : "=v"(v) : "v"(addr), "i"(OFF));
    return v;
}

// This wave's LDS reads have completed; the fragments passed through are tied
// to the wait so that nothing uses them earlier.
__device__ __forceinline__ void lgkm_wait1(floatx4 &a) { asm volatile("s_waitcnt lgkmcnt(0)" : "+v"(a)); }

__device__ __forceinline__ void lgkm_wait9(floatx4 &a, floatx4 (&b)[8])
{
    asm volatile("s_waitcnt lgkmcnt(0)"
                 : "+v"(a), "+v"(b[0]), "+v"(b[1]), "+v"(b[2]), "+v"(b[3]), "+v"(b[4]), "+v"(b[5]),
                   "+v"(b[6]), "+v"(b[7]));
}

template <int CB>
__device__ __forceinline__ void read_b32(uint32_t addr, floatx4 (&b)[8])
{
    b[CB] = lds_read4_at<CB * 16 * WideCfg<false>::ROWB>(addr);
    if constexpr (CB + 1 < 8) read_b32<CB + 1>(addr, b);
}

template <bool FIRST>
__device__ __forceinline__ void mfma32(floatx4 &c, float a, float b)
{
    if constexpr (FIRST) asm("v_mfma_f32_16x16x4_f32 %0, %1, %2, 0" : "=a"(c) : "v"(a), "v"(b));
    else mfma_acc(c, a, b);
}

// Stage complete for every wavefront: this wave's loads have landed and its
// LDS reads are done; after the barrier, so are every wavefront's.
__device__ __forceinline__ void stage_barrier()
{
    cfence();
    __builtin_amdgcn_s_waitcnt(7 << 4);                        // vmcnt(0) lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    cfence();
}

// Row block RB of half KK of a step: read the next A fragment (row block RB+1,
// or row block 0 of the second half), in the first half also two of the second
// half's B fragments (row blocks 4-7) or four of the next step's loads (row
// blocks 0-3), then the row block's 32 multiplies.  After row block 6 of the
// second half the step's last A fragment is in registers: the stage barrier
// there publishes the next step's stage (its loads were issued in row blocks
// 0-3), and row block 7 reads the next step's first fragments (B of its first
// half, A of its row block 0) while it multiplies, so a step starts multiplying
// at once.  (A read may target the registers of the A fragment that the
// multiplies just issued read: the matrix core reads its A and B operands at
// issue; only its accumulator input has a write-after-read hazard, and
// accumulators live in AGPRs nothing else writes.)
template <int KK, int RB, bool FIRST>
__device__ __forceinline__ void rb32(uint32_t st, uint32_t stn, const char *wsrc, const char *xsrc,
                                     char *fill, const Lane32 &L, floatx4 (&acc)[8][8],
                                     floatx4 (&fa)[2], floatx4 (&b0)[8], floatx4 (&b1)[8])
{
    using C = WideCfg<false>;
    constexpr int RB1 = RB + 1 < 8 ? RB + 1 : 0;
    constexpr int J = 8 * KK + RB;              // A fragment J of the step lives in fa[J % 2]
    if constexpr (J < 15)
        fa[(J + 1) % 2] = lds_read4_at<RB1 * 16 * C::ROWB>(st + L.aoff[RB + 1 < 8 ? KK : 1]);
    if constexpr (KK == 0 && RB >= 4) {
        constexpr int c0 = 2 * (RB - 4);
        b1[c0] = lds_read4_at<c0 * 16 * C::ROWB>(st + L.boff[1]);
        b1[c0 + 1] = lds_read4_at<(c0 + 1) * 16 * C::ROWB>(st + L.boff[1]);
    }
    if constexpr (KK == 0 && RB < 4) {
        issue32<4 * RB>(wsrc, xsrc, fill, L);
        issue32<4 * RB + 1>(wsrc, xsrc, fill, L);
        issue32<4 * RB + 2>(wsrc, xsrc, fill, L);
        issue32<4 * RB + 3>(wsrc, xsrc, fill, L);
    }
    if constexpr (J == 15) {
        read_b32<0>(stn + L.boff[0], b0);
        fa[0] = lds_read4_at<0>(stn + L.aoff[0]);
    }
    __builtin_amdgcn_sched_barrier(0);
    const floatx4 a = fa[J % 2];
    floatx4 (&bk)[8] = KK == 0 ? b0 : b1;
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) mfma32<FIRST && KK == 0>(acc[RB][cb], a[0], bk[cb][0]);
#pragma unroll
    for (int v = 1; v < 4; ++v)
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) mfma32<false>(acc[RB][cb], a[v], bk[cb][v]);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (J == 7) {
        lgkm_wait9(fa[0], b1);
    } else if constexpr (J == 14) {
        lgkm_wait1(fa[1]);
        stage_barrier();
    } else if constexpr (J == 15) {
        lgkm_wait9(fa[0], b0);
    } else {
        lgkm_wait1(fa[(J + 1) % 2]);
    }
    if constexpr (RB + 1 < 8) rb32<KK, RB + 1, FIRST>(st, stn, wsrc, xsrc, fill, L, acc, fa, b0, b1);
}

// K step kt of a tile, global step q of the block (stage q & 1: a tile with an
// odd step count hands the other stage to the next).  On entry the step's
// stage is complete for every wavefront and its first fragments are in b0 and
// fa[0]; on exit the same holds for the next step (the next tile's first step
// after a tile's last).
template <bool FIRST>
__device__ __forceinline__ void step32(const WideArgs &a, char *smem, const Look &lk, int kt, int q,
                                       const Lane32 &L, floatx4 (&acc)[8][8], floatx4 (&fa)[2],
                                       floatx4 (&b0)[8], floatx4 (&b1)[8])
{
    using C = WideCfg<false>;
    const bool wrap = kt + 1 >= a.nk;
    const char *wsrc = wrap ? lk.wnext : lk.wcur + (size_t)(kt + 1) * C::TILEB;
    const char *xsrc = wrap ? lk.xnext : lk.xcur + (size_t)(kt + 1) * C::TILEB;
    char *fill = smem + ((q + 1) & 1) * C::STAGEB;
    const uint32_t st = (uint32_t)(uintptr_t)(lds_void_t *)(smem + (q & 1) * C::STAGEB);
    const uint32_t stn = (uint32_t)(uintptr_t)(lds_void_t *)fill;
    rb32<0, 0, FIRST>(st, stn, wsrc, xsrc, fill, L, acc, fa, b0, b1);
    rb32<1, 0, FIRST>(st, stn, wsrc, xsrc, fill, L, acc, fa, b0, b1);
}

template <int ACT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_fit_wide32(WideArgs a)
{
    using C = WideCfg<false>;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ float red[4];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform
    const int n = lane & 15, g = lane >> 4, nh = wave & 1, sh = wave >> 1;
    TileIter it;
    it.xcd = blockIdx.x % 8;
    it.j = blockIdx.x / 8;
    it.bx = (gridDim.x - it.xcd + 7) / 8;
    it.gs = a.gs;
    it.ntn = a.ntn;
    it.rows = a.rows;
    it.setup();
    const int ntiles = it.count();
    if (ntiles == 0) return;
    const Lane32 L = lane32(wave, lane, nh, sh);
    Look lk;
    look_set<false>(a, it, 0, ntiles, lk);
    // prologue: step 0 of tile 0 into stage 0
    issue32<0>(lk.wcur, lk.xcur, smem, L);
    issue32<1>(lk.wcur, lk.xcur, smem, L);
    issue32<2>(lk.wcur, lk.xcur, smem, L);
    issue32<3>(lk.wcur, lk.xcur, smem, L);
    issue32<4>(lk.wcur, lk.xcur, smem, L);
    issue32<5>(lk.wcur, lk.xcur, smem, L);
    issue32<6>(lk.wcur, lk.xcur, smem, L);
    issue32<7>(lk.wcur, lk.xcur, smem, L);
    issue32<8>(lk.wcur, lk.xcur, smem, L);
    issue32<9>(lk.wcur, lk.xcur, smem, L);
    issue32<10>(lk.wcur, lk.xcur, smem, L);
    issue32<11>(lk.wcur, lk.xcur, smem, L);
    issue32<12>(lk.wcur, lk.xcur, smem, L);
    issue32<13>(lk.wcur, lk.xcur, smem, L);
    issue32<14>(lk.wcur, lk.xcur, smem, L);
    issue32<15>(lk.wcur, lk.xcur, smem, L);
    stage_barrier();
    floatx4 fa[2], b0[8], b1[8];
    {
        const uint32_t st0 = (uint32_t)(uintptr_t)(lds_void_t *)smem;
        read_b32<0>(st0 + L.boff[0], b0);
        fa[0] = lds_read4_at<0>(st0 + L.aoff[0]);
        lgkm_wait9(fa[0], b0);
    }
    for (int i = 0; i < ntiles; ++i) {
        int r, col;
        it.tile(i, &r, &col);
        if (i > 0) look_set<false>(a, it, i, ntiles, lk);
        floatx4 acc[8][8];
        const int qbase = i * a.nk;
        step32<true>(a, smem, lk, 0, qbase, L, acc, fa, b0, b1);
        // the epilogue's global inputs, fetched while the tile's K loop runs
        // (after its first step: the next step's wait covers them)
        W2Frag<false> w2;
        w2_load<false>(a, r, nh, n, g, w2);
        const int label = tile_label(a, col, wave, lane);
        for (int kt = 1; kt < a.nk; ++kt) step32<false>(a, smem, lk, kt, qbase + kt, L, acc, fa, b0, b1);
        mfma_acc_sync(acc);
        wide_epilogue<false, ACT>(a, smem, r, col, wave, lane, acc, w2, red, label);
    }
    __builtin_amdgcn_s_waitcnt(0);
}

// BF16 wide kernel with the software pipeline above (same tiles, layout and
// epilogue as the FP32 kernel).
template <int ACT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_fit_wide_pipe(WideArgs a)
{
    using C = WideCfg<true>;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ float red[4];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform
    const int n = lane & 15, g = lane >> 4, nh = wave & 1, sh = wave >> 1;
    TileIter it;
    it.xcd = blockIdx.x % 8;
    it.j = blockIdx.x / 8;
    it.bx = (gridDim.x - it.xcd + 7) / 8;
    it.gs = a.gs;
    it.ntn = a.ntn;
    it.rows = a.rows;
    it.setup();
    const int ntiles = it.count();
    if (ntiles == 0) return;
    // K steps per tile: at least STAGES, so the look-ahead of a step lies in its
    // own tile or the next one
    const PipeLane L = pipe_lane(wave, lane, nh, sh);
    Look lk;
    look_set(a, it, 0, ntiles, lk);
    // prologue: steps 0..3 of tile 0 into stages 0..3, then the fragments of step 0
#pragma unroll
    for (int s = 0; s < PipeCfg::STAGES; ++s)
        pipe_issue_all(lk.wcur + (size_t)s * C::TILEB, lk.xcur + (size_t)s * C::TILEB,
                       smem + s * PipeCfg::STAGEB, L);
    {
        constexpr int n3 = 3 * PipeCfg::LOADS;
        cfence();
        __builtin_amdgcn_s_waitcnt((n3 & 0xF) | ((n3 >> 4) << 14) | (7 << 4) | (15 << 8));
        __builtin_amdgcn_s_barrier();
        cfence();
    }
    bf16x8 fa[2][8], fb[2][8];
    {
        const uint32_t st0 = (uint32_t)(uintptr_t)(lds_void_t *)smem;
        pipe_read_rb<0>(st0, L, fa[0][0], fb[0][0]);
        pipe_read_rb<1>(st0, L, fa[0][1], fb[0][1]);
        pipe_read_rb<2>(st0, L, fa[0][2], fb[0][2]);
        pipe_read_rb<3>(st0, L, fa[0][3], fb[0][3]);
        pipe_read_rb<4>(st0, L, fa[0][4], fb[0][4]);
        pipe_read_rb<5>(st0, L, fa[0][5], fb[0][5]);
        pipe_read_rb<6>(st0, L, fa[0][6], fb[0][6]);
        pipe_read_rb<7>(st0, L, fa[0][7], fb[0][7]);
    }
    lgkm_wait_all(fa[0], fb[0]);
    for (int i = 0; i < ntiles; ++i) {
        int r, col;
        it.tile(i, &r, &col);
        if (i > 0) look_set(a, it, i, ntiles, lk);
        floatx4 acc[8][8];
        // the epilogue's global inputs are fetched at the start of the tile;
        // then every load in flight (the tile's first look-ahead steps
        // included) is waited for.  Measured on 784-256-10: with this drain
        // at each tile start the XCD's blocks stay closer in step and the
        // kernel is 4 % faster at tile groups of 4-8 sparks than without it.
        W2Frag<true> w2;
        w2_load<true>(a, r, nh, n, g, w2);
        const int label = tile_label(a, col, wave, lane);
        __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));   // vmcnt(0)
        const int qbase = i * a.nk;
        if (qbase & 1) pipe_tile<1>(a, smem, lk, qbase, L, acc, fa, fb);
        else pipe_tile<0>(a, smem, lk, qbase, L, acc, fa, fb);
        mfma_acc_sync(acc);
        wide_epilogue<true, ACT>(a, smem, r, col, wave, lane, acc, w2, red, label, PipeCfg::ZX);
    }
    __builtin_amdgcn_s_waitcnt(0);
}

}  // namespace fit
}  // namespace mgfwa
