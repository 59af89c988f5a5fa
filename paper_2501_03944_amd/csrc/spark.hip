// Initial fireworks and explosion sparks (Alg. 1, the initialisation step, the
// explosion step and the mapping step after it).
//
// One thread produces four consecutive coordinates from one Philox block and
// writes them as a single 16-byte store, so a wavefront writes 1 KiB of a spark
// row contiguously.  Grid: x over the row's 4-coordinate chunks, y over rows.
#include "internal.h"

namespace mgfwa {

namespace {

constexpr int TPB = 256;
constexpr int MAX_GRID_Y = 65535;

__global__ __launch_bounds__(TPB) void k_init_positions(float *__restrict__ F,
                                                        float *__restrict__ A, int rows, int D,
                                                        int Dp, uint2 key, Box box, float amp0)
{
    const int chunk = blockIdx.x * TPB + threadIdx.x;
    const int nchunk = Dp >> 2;
    for (int row = blockIdx.y; row < rows; row += gridDim.y) {
        if (chunk == 0) A[row] = amp0;
        if (chunk >= nchunk) continue;
        const uint4 r = draw4(key, (uint32_t)chunk, (uint32_t)row, 0u, TAG_INIT);
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[e] = box_uniform(box, u01(w[e]));
            if (4 * chunk + e >= D) v[e] = 0.0f;
        }
        reinterpret_cast<float4 *>(F + (size_t)row * Dp)[chunk] = make_float4(v[0], v[1], v[2], v[3]);
    }
}

// Per-dimension minimum and maximum over the N fireworks of every population
// (the range the range-mapping variant draws into), fireworks in index order.
__device__ __forceinline__ void pop_range_body(const float *__restrict__ F, int N, int B, int Dp,
                                               float *__restrict__ lo, float *__restrict__ hi,
                                               const int32_t *__restrict__ ctrl, Blk blk)
{
    if (ctrl[CTRL_DONE]) return;
    const int d = blk.x * TPB + threadIdx.x;
    if (d >= Dp) return;
    for (int b = blk.y; b < B; b += blk.gy) {
        const float *f0 = F + (size_t)b * N * Dp;
        float a = f0[d], c = f0[d];
        for (int f = 1; f < N; ++f) {
            const float v = f0[(size_t)f * Dp + d];
            if (v < a) a = v;
            if (v > c) c = v;
        }
        lo[(size_t)b * Dp + d] = a;
        hi[(size_t)b * Dp + d] = c;
    }
}

__global__ __launch_bounds__(TPB) void k_pop_range(const float *__restrict__ F, int N, int B,
                                                   int Dp, float *__restrict__ lo,
                                                   float *__restrict__ hi,
                                                   const int32_t *__restrict__ ctrl)
{
    pop_range_body(F, N, B, Dp, lo, hi, ctrl, own_block());
}

__global__ __launch_bounds__(TPB) void k_pop_range_group(GroupTable t)
{
    const int j = group_job(t, blockIdx.x);
    Blk gb;
    if (!group_block(t, j, blockIdx.x, &gb)) return;   // padding
    // private copies: read through a pointer into global memory, the
    // arguments would be reloaded after every store the body makes
    const Shape js = t.job[j]->s;
    const DevState jd = t.job[j]->d;
    pop_range_body(jd.F, js.N, js.B, js.Dp, jd.lo, jd.hi, jd.ctrl,
                   gb);
}

// Explosion spark j of firework f (row = f*lambda + j) for generation t+1:
// s = fma(A_f, 2u - 1, x_f); out-of-box coordinates take a uniform draw from
// the mapping stream of the same (chunk, row, generation).
// With PACK the spark is also written in the wide fitness kernel's packed
// layout (row `row` of wp.Wp): four coordinates of one W1 row inside one
// 32-column block (the common case) as one store, others one by one.
template <bool BF>
__device__ __forceinline__ void pack_four(const WidePack &wp, int row, int j0, int D,
                                          const float (&s)[4])
{
    char *dst = wp.Wp + (size_t)row * wp.pr;
    int o = -1, k = 0;
    if (j0 >= wp.woff1 && j0 + 3 < wp.woff1 + wp.hid * wp.in) {
        const int rel = j0 - wp.woff1;
        o = rel / wp.in;
        k = rel - o * wp.in;
    }
    // four columns of one W1 row inside one 32-column block, 4-aligned
    if (o >= 0 && k + 3 < wp.in && (k & 31) <= 28 && (k & 3) == 0) {
        const size_t off = wide_w1_offset(o, k, BF ? 2 : 4);
        if constexpr (BF) {
            const uint32_t lo = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)s[0]) |
                                ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)s[1]) << 16);
            const uint32_t hi = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)s[2]) |
                                ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)s[3]) << 16);
            *reinterpret_cast<uint2 *>(dst + off) = make_uint2(lo, hi);
        } else {
            *reinterpret_cast<float4 *>(dst + off) = make_float4(s[0], s[1], s[2], s[3]);
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (j0 + e >= D) break;
        bool f32;
        const size_t off = wide_pack_offset(wp, j0 + e, &f32);
        if (BF && !f32) *reinterpret_cast<uint16_t *>(dst + off) = __builtin_bit_cast(uint16_t, (__bf16)s[e]);
        else *reinterpret_cast<float *>(dst + off) = s[e];
    }
}

// SE null: the FP32 rows are not stored (the packed rows are the only copy the
// fitness needs; later steps regenerate the sparks they read).
template <int PACK>   // 0: no packing, 1: FP32 packed rows, 2: BF16
__device__ __forceinline__ void explode_body(const float *__restrict__ F, const float *__restrict__ A,
                                             float *__restrict__ SE, int lam, int rows, int D,
                                             int Dp, uint2 key, Box box,
                                             const int32_t *__restrict__ ctrl, int N,
                                             const float *__restrict__ lo,
                                             const float *__restrict__ hi, const WidePack &wp,
                                             Blk b)
{
    if (ctrl[CTRL_DONE]) return;
    const uint32_t tn = (uint32_t)ctrl[CTRL_GEN] + 1u;
    const int chunk = b.x * TPB + threadIdx.x;
    if (chunk >= (Dp >> 2)) return;
    for (int row = b.y; row < rows; row += b.gy) {
        const int gf = row / lam;
        const float amp = A[gf];
        const float4 x4 = reinterpret_cast<const float4 *>(F + (size_t)gf * Dp)[chunk];
        const float x[4] = {x4.x, x4.y, x4.z, x4.w};
        const size_t pb = (size_t)(gf / N) * Dp;
        const float *plo = lo ? lo + pb : nullptr, *phi = hi ? hi + pb : nullptr;
        float s[4];
        explosion_chunk(x, amp, key, chunk, (uint32_t)row, tn, box, plo, phi, D, s);
        if (SE)
            reinterpret_cast<float4 *>(SE + (size_t)row * Dp)[chunk] = make_float4(s[0], s[1], s[2], s[3]);
        if constexpr (PACK != 0)
            if (4 * chunk < D) pack_four<PACK == 2>(wp, row, 4 * chunk, D, s);
    }
}

template <int PACK>
__global__ __launch_bounds__(TPB) void k_explode(const float *__restrict__ F,
                                                 const float *__restrict__ A,
                                                 float *__restrict__ SE, int lam, int rows, int D,
                                                 int Dp, uint2 key, Box box,
                                                 const int32_t *__restrict__ ctrl, int N,
                                                 const float *__restrict__ lo,
                                                 const float *__restrict__ hi, WidePack wp)
{
    explode_body<PACK>(F, A, SE, lam, rows, D, Dp, key, box, ctrl, N, lo, hi, wp, own_block());
}

// The explosion of many jobs (stored FP32 sparks, no packed rows) in one launch.
__global__ __launch_bounds__(TPB) void k_explode_group(GroupTable t)
{
    const int j = group_job(t, blockIdx.x);
    Blk gb;
    if (!group_block(t, j, blockIdx.x, &gb)) return;   // padding
    // private copies: read through a pointer into global memory, the
    // arguments would be reloaded after every store the body makes
    const Shape js = t.job[j]->s;
    const DevState jd = t.job[j]->d;
    const Shape &s = js;
    const DevState &d = jd;
    explode_body<0>(d.F, d.A, d.SE, s.lam, s.BN * s.lam, s.D, s.Dp, s.key, s.box, d.ctrl, s.N,
                    s.map_range ? d.lo : nullptr, s.map_range ? d.hi : nullptr, WidePack{},
                    gb);
}

// Explosion sparks written only as the wide fitness kernel's packed rows, in the
// rows' own K-blocked order (the FP32 rows are not stored).  x-blocks below
// `units`: a wavefront produces 16 rows x 32 columns of one K block of W1aug (b1
// is column `in`), 8 consecutive columns per lane, and writes them as one
// contiguous 1 KiB (BF16) or 2 KiB (FP32) segment; rows past the hidden width
// and the zero columns past `in` are left to the initial zeroing except inside a
// written segment.  The x-blocks from `units` on take the W2 and b2
// coordinates, four per thread, placed one by one.  Values are those of
// explosion_chunk, as in k_explode.
constexpr int XP_ROWS = 64;   // W1aug rows per block (16 per wavefront)

template <bool BF>
__global__ __launch_bounds__(TPB) void k_explode_packed(const float *__restrict__ F,
                                                        const float *__restrict__ A, int lam,
                                                        int rows, int D, int Dp, uint2 key, Box box,
                                                        const int32_t *__restrict__ ctrl, int N,
                                                        const float *__restrict__ lo,
                                                        const float *__restrict__ hi, WidePack wp,
                                                        int units)
{
    if (ctrl[CTRL_DONE]) return;
    const uint32_t tn = (uint32_t)ctrl[CTRL_GEN] + 1u;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nob = (wp.hid + XP_ROWS - 1) / XP_ROWS;       // 64-row blocks of hidden units
    // W1 columns k..k+7 of a row start on a 4-coordinate chunk of the spark
    const bool aligned = (wp.in & 3) == 0 && (wp.woff1 & 3) == 0;
    const int woff2 = wp.boff1 + wp.hid;                      // W2, then b2, up to D
    for (int row = blockIdx.y; row < rows; row += gridDim.y) {
        const int gf = row / lam;
        const float amp = A[gf];
        const float4 *xrow = reinterpret_cast<const float4 *>(F + (size_t)gf * Dp);
        const size_t pb = (size_t)(gf / N) * Dp;
        const float *plo = lo ? lo + pb : nullptr, *phi = hi ? hi + pb : nullptr;
        char *dst = wp.Wp + (size_t)row * wp.pr;
        if ((int)blockIdx.x < units) {
            const int kb = blockIdx.x / nob, ob = blockIdx.x - kb * nob;
            const int o = ob * XP_ROWS + wave * 16 + (lane >> 2);
            const int k0 = kb * 32 + 8 * (lane & 3);
            if (o >= wp.hid) continue;
            char *p = dst + wide_w1_offset(o, k0, BF ? 2 : 4);
            if (aligned && k0 + 8 <= wp.in) {
                float v[8];
                const int c0 = (wp.woff1 + o * wp.in + k0) >> 2;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float4 x4 = xrow[c0 + h];
                    const float x[4] = {x4.x, x4.y, x4.z, x4.w};
                    float s4[4];
                    explosion_chunk(x, amp, key, c0 + h, (uint32_t)row, tn, box, plo, phi, D, s4);
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[4 * h + e] = s4[e];
                }
                if constexpr (BF) {
                    uint32_t h[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        h[e] = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[2 * e]) |
                               ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[2 * e + 1]) << 16);
                    *reinterpret_cast<uint4 *>(p) = make_uint4(h[0], h[1], h[2], h[3]);
                } else {
                    reinterpret_cast<float4 *>(p)[0] = make_float4(v[0], v[1], v[2], v[3]);
                    reinterpret_cast<float4 *>(p)[1] = make_float4(v[4], v[5], v[6], v[7]);
                }
            } else {
                // the K block holding b1, or unaligned rows: coordinate by
                // coordinate (a rolled loop: rare, and it keeps registers low)
                int cached = -1;
                float s4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
                for (int e = 0; e < 8; ++e) {
                    const int k = k0 + e;
                    const int j = k < wp.in ? wp.woff1 + o * wp.in + k : k == wp.in ? wp.boff1 + o : -1;
                    float val = 0.0f;
                    if (j >= 0) {
                        if ((j >> 2) != cached) {
                            cached = j >> 2;
                            const float4 x4 = xrow[cached];
                            const float x[4] = {x4.x, x4.y, x4.z, x4.w};
                            explosion_chunk(x, amp, key, cached, (uint32_t)row, tn, box, plo, phi, D, s4);
                        }
                        const int q = j & 3;
                        val = q == 0 ? s4[0] : q == 1 ? s4[1] : q == 2 ? s4[2] : s4[3];
                    }
                    if constexpr (BF)
                        reinterpret_cast<uint16_t *>(p)[e] = __builtin_bit_cast(uint16_t, (__bf16)val);
                    else
                        reinterpret_cast<float *>(p)[e] = val;
                }
            }
        } else {
            // W2 and b2: chunk c covers coordinates 4c..4c+3; those below woff2 (b1)
            // belong to the W1aug blocks
            const int c = (woff2 >> 2) + ((int)blockIdx.x - units) * TPB + threadIdx.x;
            if (4 * c >= D) continue;
            const float4 x4 = xrow[c];
            const float x[4] = {x4.x, x4.y, x4.z, x4.w};
            float s4[4];
            explosion_chunk(x, amp, key, c, (uint32_t)row, tn, box, plo, phi, D, s4);
#pragma unroll 1
            for (int e = 0; e < 4; ++e) {
                const int j = 4 * c + e;
                if (j < woff2 || j >= D) continue;
                bool f32;
                const size_t off = wide_pack_offset(wp, j, &f32);
                const float val = e == 0 ? s4[0] : e == 1 ? s4[1] : e == 2 ? s4[2] : s4[3];
                if (BF && !f32) *reinterpret_cast<uint16_t *>(dst + off) = __builtin_bit_cast(uint16_t, (__bf16)val);
                else *reinterpret_cast<float *>(dst + off) = val;
            }
        }
    }
}

// Blocks over (chunk range, rows); a block takes rows_per_block rows (strided by
// the grid), so that launches of many rows are not bound by block dispatch.
dim3 row_grid(int Dp, int rows, int rows_per_block = 1)
{
    const int nchunk = Dp >> 2;
    const int ry = (rows + rows_per_block - 1) / rows_per_block;
    return dim3((nchunk + TPB - 1) / TPB, ry < MAX_GRID_Y ? ry : MAX_GRID_Y);
}

}  // namespace

hipError_t launch_init_positions(const Shape &s, const DevState &d, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_positions, row_grid(s.Dp, s.BN), dim3(TPB), 0, st, d.F, d.A, s.BN,
                       s.D, s.Dp, s.key, s.box, s.amp0);
    return hipGetLastError();
}

dim3 pop_range_grid(const Shape &s)
{
    return dim3((s.Dp + TPB - 1) / TPB, s.B < MAX_GRID_Y ? s.B : MAX_GRID_Y);
}

dim3 explode_grid(const Shape &s)
{
    const int rows = s.BN * s.lam;
    // 32 or 8 rows per block while there are enough blocks to fill the device
    const long blocks_x = ((s.Dp >> 2) + TPB - 1) / TPB;
    const int rpb = blocks_x * (rows / 32) >= 2048 ? 32 : blocks_x * (rows / 8) >= 2048 ? 8 : 1;
    return row_grid(s.Dp, rows, rpb);
}

hipError_t launch_pop_range(const Shape &s, const DevState &d, hipStream_t st)
{
    hipLaunchKernelGGL(k_pop_range, pop_range_grid(s), dim3(TPB), 0, st, d.F, s.N,
                       s.B, s.Dp, d.lo, d.hi, d.ctrl);
    return hipGetLastError();
}

hipError_t launch_pop_range_group(const GroupTable &t, hipStream_t st)
{
    hipLaunchKernelGGL(k_pop_range_group, dim3(t.start[t.njobs]), dim3(TPB), 0, st, t);
    return hipGetLastError();
}

hipError_t launch_explode_group(const GroupTable &t, hipStream_t st)
{
    hipLaunchKernelGGL(k_explode_group, dim3(t.start[t.njobs]), dim3(TPB), 0, st, t);
    return hipGetLastError();
}

hipError_t launch_explode(const Shape &s, const DevState &d, hipStream_t st, const WidePack *wp,
                          bool write_se)
{
    const int rows = s.BN * s.lam;
    if (wp && !write_se) {
        // packed rows only, written in their own order
        const int units = (wp->Kp / 32) * ((wp->hid + XP_ROWS - 1) / XP_ROWS);
        const int woff2 = wp->boff1 + wp->hid;
        const int tail = ((s.D - (woff2 & ~3)) / 4 + 1 + TPB - 1) / TPB;
        const int bx = units + tail;
        const int rpb = (long)bx * (rows / 8) >= 4096 ? 8 : 1;
        const int ry = (rows + rpb - 1) / rpb;
        const dim3 grid((unsigned)bx, ry < MAX_GRID_Y ? ry : MAX_GRID_Y);
        const float *lo = s.map_range ? d.lo : nullptr, *hi = s.map_range ? d.hi : nullptr;
        if (wp->bf16)
            hipLaunchKernelGGL(k_explode_packed<true>, grid, dim3(TPB), 0, st, d.F, d.A, s.lam, rows,
                               s.D, s.Dp, s.key, s.box, d.ctrl, s.N, lo, hi, *wp, units);
        else
            hipLaunchKernelGGL(k_explode_packed<false>, grid, dim3(TPB), 0, st, d.F, d.A, s.lam, rows,
                               s.D, s.Dp, s.key, s.box, d.ctrl, s.N, lo, hi, *wp, units);
        return hipGetLastError();
    }
    const WidePack none{};
    const WidePack &w = wp ? *wp : none;
    auto *k = !wp ? &k_explode<0> : wp->bf16 ? &k_explode<2> : &k_explode<1>;
    hipLaunchKernelGGL(k, explode_grid(s), dim3(TPB), 0, st, d.F, d.A,
                       write_se || !wp ? d.SE : nullptr, s.lam, rows,
                       s.D, s.Dp, s.key, s.box, d.ctrl, s.N, s.map_range ? d.lo : nullptr,
                       s.map_range ? d.hi : nullptr, w);
    return hipGetLastError();
}

}  // namespace mgfwa
