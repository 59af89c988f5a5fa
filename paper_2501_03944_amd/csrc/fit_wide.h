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
//             direct global->LDS loads (global_load_lds_dwordx4): every step
//             issues the loads of the step STAGES-1 ahead, waits for the current
//             one with an explicit vmcnt and a barrier, then runs its MFMAs.  Each
//             step issues the same number of loads (past the end it re-loads the
//             last tile into the free stage) so the wait count is a constant;
//  * swizzle: a 16-byte chunk c of tile row r lives at chunk c ^ s(r), with
//             s(r) = (r >> 2) & 3 for 64-byte rows (BF16) and (r >> 1) & 7 for
//             128-byte rows (FP32), so the 16 rows read by a quarter-wavefront
//             fall in distinct bank groups;
//  * epilogue per tile: activation, layer 2 as MFMAs whose B operand is the
//             hidden tile straight from the accumulators, the two hidden halves'
//             logits summed through LDS, then the loss; one partial per
//             (spark, sample tile), reduced later in a fixed order;
//  * schedule: blocks are persistent (one per CU); tile groups of GS sparks go
//             to one XCD, whose blocks split the group's sample tiles, so a
//             spark's weights are fetched from HBM into that XCD's L2 once.
//
// Packed spark layout (written by k_pack_wide, row pitch PR bytes):
//   [0, 256*Kp*es)          W1aug[256][Kp]: W1 (zero-padded), b1 in column `in`
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
    const char *Xw;        // packed samples [S_pad][Kp] (element type of the kernel)
    int Kp, nk;            // padded K and K steps
    int S, S_pad, ntn;     // samples, padded samples, sample tiles
    int fo1;               // output width (<= 16)
    int loss, act;
    const float *Y;        // [S_pad][fo1]
    const int32_t *lab;    // [S_pad]
    float *partial;        // [rows][ntn]
    int gs;                // sparks per XCD tile group
};

template <bool BF>
struct WideCfg {
    static constexpr int ES = BF ? 2 : 4;                  // bytes per element
    static constexpr int ROWB = WT_K * ES;                 // bytes per tile row per K step
    static constexpr int NCH = ROWB / 16;                  // 16-byte chunks per row
    static constexpr int RPL = 64 / NCH;                   // rows per wave load (1 KiB)
    static constexpr int TILEB = WT_M * ROWB;              // bytes of one operand tile
    static constexpr int STAGEB = 2 * TILEB;               // W tile + X tile
    static constexpr int STAGES = BF ? 3 : 2;
    static constexpr int LOADS = STAGEB / 1024 / WT_NW;    // wave loads per wave per step
    static constexpr int ZX = STAGES * STAGEB;             // logits exchange area
    static constexpr int ZXB = 2 * 64 * 32 * 4;            // two wavefronts x 64 lanes x 32 floats
    static constexpr int LDS = ZX + ZXB;
};

__device__ __forceinline__ int wide_swz(int row, int nch)
{
    return nch == 4 ? ((row >> 2) & 3) : ((row >> 1) & 7);
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

// Issue this wave's loads of one K step (W and X tiles) into an LDS stage.
template <bool BF>
__device__ __forceinline__ void wide_issue(const WideArgs &a, char *stage, int r, int col, int kt,
                                           int wave, int lane)
{
    using C = WideCfg<BF>;
    const char *wrow = a.Wp + (size_t)r * a.pr + (size_t)kt * C::ROWB;
    const char *xrow = a.Xw + ((size_t)col * WT_N) * a.Kp * C::ES + (size_t)kt * C::ROWB;
    const size_t gpitch = (size_t)a.Kp * C::ES;
    const int lr = lane / C::NCH, pc = lane % C::NCH;
#pragma unroll
    for (int t = 0; t < C::LOADS; ++t) {
        // wave loads alternate between the W tile and the X tile
        const int half = t & 1;
        const int r0 = (wave * (C::LOADS / 2) + (t >> 1)) * C::RPL;
        const int row = r0 + lr;
        const int q = pc ^ wide_swz(row, C::NCH);
        const char *src = (half ? xrow : wrow) + (size_t)row * gpitch + q * 16;
        char *dst = stage + half * C::TILEB + r0 * C::ROWB;
        __builtin_amdgcn_global_load_lds(src, (lds_void_t *)dst, 16, 0, 0);
    }
}

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

// Wait until the current step's stage has landed: the loads of the STAGES-1
// younger steps may still be in flight.
template <bool BF>
__device__ __forceinline__ void wait_stage()
{
    constexpr int n = (WideCfg<BF>::STAGES - 1) * WideCfg<BF>::LOADS;
    static_assert(n < 64, "vmcnt holds at most 63");
    cfence();
    __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (7 << 4) | (15 << 8));
    __builtin_amdgcn_s_barrier();
    cfence();
}

// MFMAs of one K step on the stage: acc[rb][cb] over this wave's quarter.
template <bool BF>
__device__ __forceinline__ void wide_mma(const char *stage, int nh, int sh, int n, int g,
                                         floatx4 (&acc)[8][8])
{
    using C = WideCfg<BF>;
    const char *wt = stage;
    const char *xt = stage + C::TILEB;
    if constexpr (BF) {
        bf16x8 bfr[8];
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) {
            const int row = 128 * sh + 16 * cb + n;
            bfr[cb] = *reinterpret_cast<const bf16x8 *>(xt + row * C::ROWB +
                                                        ((g ^ wide_swz(row, 4)) << 4));
        }
#pragma unroll
        for (int rb = 0; rb < 8; ++rb) {
            const int row = 128 * nh + 16 * rb + n;
            const bf16x8 afr = *reinterpret_cast<const bf16x8 *>(wt + row * C::ROWB +
                                                                 ((g ^ wide_swz(row, 4)) << 4));
#pragma unroll
            for (int cb = 0; cb < 8; ++cb)
                mfma_acc(acc[rb][cb], afr, bfr[cb]);
        }
    } else {
        // lane group g holds k = 16kk + 4g + v of the two 16-column halves kk
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            floatx4 bfr[8];
#pragma unroll
            for (int cb = 0; cb < 8; ++cb) {
                const int row = 128 * sh + 16 * cb + n;
                bfr[cb] = *reinterpret_cast<const floatx4 *>(
                    xt + row * C::ROWB + (((4 * kk + g) ^ wide_swz(row, 8)) << 4));
            }
#pragma unroll
            for (int rb = 0; rb < 8; ++rb) {
                const int row = 128 * nh + 16 * rb + n;
                const floatx4 afr = *reinterpret_cast<const floatx4 *>(
                    wt + row * C::ROWB + (((4 * kk + g) ^ wide_swz(row, 8)) << 4));
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int cb = 0; cb < 8; ++cb)
                        mfma_acc(acc[rb][cb], afr[v], bfr[cb][v]);
            }
        }
    }
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
__device__ __forceinline__ void wide_act(floatx4 (&acc)[8][8])
{
#pragma unroll
    for (int rb = 0; rb < 8; ++rb)
#pragma unroll
        for (int cb = 0; cb < 8; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[rb][cb][v] = act_c<ACT>(acc[rb][cb][v]);
}

template <bool BF, int ACT>
__device__ void wide_epilogue(const WideArgs &a, char *smem, int r, int col, int wave, int lane,
                              floatx4 (&acc)[8][8], const W2Frag<BF> &w2, float *red)
{
    using C = WideCfg<BF>;
    const int n = lane & 15, g = lane >> 4, nh = wave & 1, sh = wave >> 1;
    // activation of the hidden tile (the bias came in through the ones column)
    wide_act<ACT>(acc);
    // layer 2: logits of this wave's hidden half
    floatx4 z[8][1];
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) z[cb][0] = zero4();
    if constexpr (BF) {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 afr = __builtin_bit_cast(bf16x8, w2.f[kb]);
#pragma unroll
            for (int cb = 0; cb < 8; ++cb) {
                const bf16x8 bfr = to_bf16x8(acc[2 * kb][cb], acc[2 * kb + 1][cb]);
                z[cb][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr, z[cb][0], 0, 0, 0);
            }
        }
    } else {
#pragma unroll
        for (int rb = 0; rb < 8; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int cb = 0; cb < 8; ++cb)
                    z[cb][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(w2.f[rb][v], acc[rb][cb][v], z[cb][0], 0, 0, 0);
    }
    // the upper hidden half hands its logits to the lower half through LDS
    float *zx = reinterpret_cast<float *>(smem + C::ZX) + (size_t)sh * 64 * 32 + lane * 32;
    if (nh == 1) {
#pragma unroll
        for (int cb = 0; cb < 8; ++cb)
            *reinterpret_cast<floatx4 *>(zx + 4 * cb) = z[cb][0];
    }
    lds_barrier();
    float lsum = 0.0f;
    if (nh == 0) {
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) {
            const floatx4 o = *reinterpret_cast<const floatx4 *>(zx + 4 * cb);
#pragma unroll
            for (int v = 0; v < 4; ++v) z[cb][0][v] = z[cb][0][v] + o[v] + w2.b2[v];
        }
        // slab_loss reads the loss inputs through a FitArgs view
        FitArgs fa;
        fa.loss = a.loss;
        fa.Y = a.Y;
        fa.lab = a.lab;
        fa.S = a.S;
        fa.fo[0] = a.fo1;
        lsum = slab_loss<8, 1>(fa, 0, col * WT_N + 128 * sh, n, g, z);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) lsum += __shfl_xor(lsum, off);
        if (lane == 0) red[sh] = lsum;
    }
    lds_barrier();
    if (threadIdx.x == 0) a.partial[(size_t)r * a.ntn + col] = red[0] + red[1];
}

// One K step: issue the loads STAGES-1 steps ahead, wait for this step's
// stage, multiply, release the stage.
template <bool BF, int S>
__device__ __forceinline__ void wide_step(const WideArgs &a, char *smem, const TileIter &it, int q,
                                          int Q, int wave, int lane, int nh, int sh, int n, int g,
                                          floatx4 (&acc)[8][8])
{
    using C = WideCfg<BF>;
    {
        int qq = q + C::STAGES - 1;
        qq = qq < Q ? qq : Q - 1;                 // past the end: re-load into the free stage
        int r, col;
        it.tile(qq / a.nk, &r, &col);
        wide_issue<BF>(a, smem + ((S + C::STAGES - 1) % C::STAGES) * C::STAGEB, r, col, qq % a.nk,
                       wave, lane);
    }
    wait_stage<BF>();
    wide_mma<BF>(smem + S * C::STAGEB, nh, sh, n, g, acc);
    lds_barrier();
}

// One round of STAGES consecutive K steps starting at step q0 (q0 % STAGES == 0).
template <bool BF, int S = 0>
__device__ __forceinline__ void wide_round(const WideArgs &a, char *smem, const TileIter &it,
                                           int q0, int Q, int wave, int lane, int nh, int sh,
                                           int n, int g, floatx4 (&acc)[8][8])
{
    wide_step<BF, S>(a, smem, it, q0 + S, Q, wave, lane, nh, sh, n, g, acc);
    if constexpr (S + 1 < WideCfg<BF>::STAGES)
        wide_round<BF, S + 1>(a, smem, it, q0, Q, wave, lane, nh, sh, n, g, acc);
}

template <bool BF, int ACT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_fit_wide(WideArgs a)
{
    using C = WideCfg<BF>;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ float red[2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
    const int Q = ntiles * a.nk;          // K steps of this block; nk is a multiple of STAGES
    // prologue: the first STAGES-1 steps
#pragma unroll
    for (int s = 0; s < C::STAGES - 1; ++s) {
        const int qq = s < Q ? s : Q - 1;
        int r, col;
        it.tile(qq / a.nk, &r, &col);
        wide_issue<BF>(a, smem + s * C::STAGEB, r, col, qq % a.nk, wave, lane);
    }
    for (int i = 0; i < ntiles; ++i) {
        int r, col;
        it.tile(i, &r, &col);
        floatx4 acc[8][8];
#pragma unroll
        for (int rb = 0; rb < 8; ++rb)
#pragma unroll
            for (int cb = 0; cb < 8; ++cb) acc[rb][cb] = zero4();
        mfma_acc_sync(acc);
        const int qbase = i * a.nk;
        for (int kt0 = 0; kt0 + C::STAGES < a.nk; kt0 += C::STAGES)
            wide_round<BF>(a, smem, it, qbase + kt0, Q, wave, lane, nh, sh, n, g, acc);
        // last round of the tile; BF16 fetches the layer-2 weights while it runs
        // (its tiles are short), FP32 after it (fewer live registers)
        W2Frag<BF> w2;
        if constexpr (BF) w2_load<BF>(a, r, nh, n, g, w2);
        wide_round<BF>(a, smem, it, qbase + a.nk - C::STAGES, Q, wave, lane, nh, sh, n, g, acc);
        if constexpr (!BF) w2_load<BF>(a, r, nh, n, g, w2);
        mfma_acc_sync(acc);
        wide_epilogue<BF, ACT>(a, smem, r, col, wave, lane, acc, w2, red);
    }
    __builtin_amdgcn_s_waitcnt(0);
}

}  // namespace fit
}  // namespace mgfwa
