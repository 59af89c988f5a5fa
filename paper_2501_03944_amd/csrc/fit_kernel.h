// Fitness kernel template, instantiated by the fit_*.hip files.
//
// Fitness of every spark (Alg. 1, the evaluation step): the
// loss of the MLP whose weights are the spark, over the shared sample set.
//
// Each spark's layer is a dense contraction, so the evaluation is a grouped
// GEMM on the matrix cores.  The kernel works in the transposed frame,
// H_l^T = act(W_l H_{l-1}^T + b_l): the spark's weights are the MFMA A operand
// and 16-sample slabs are the B operand.  An MFMA accumulator tile holds, in
// lane (n, g) = (lane % 16, lane / 16), rows 4g..4g+3 of column n, which is
// exactly the B-operand fragment the next layer needs once its K index is
// permuted the same way on the A side; so every layer after the first reads its
// input straight from registers and only the first layer touches memory
// (16-byte loads of the packed sample matrix, L2-resident).  Bias, activation
// and the loss run in the accumulator registers; a block reduces its samples'
// losses in a fixed order into one partial per (spark, block) and a second
// kernel sums the partials of a spark in order.  No floating-point atomics:
// the result is deterministic.
//
// FP32:  v_mfma_f32_16x16x4_f32,  K step 4 per MFMA (4 MFMAs per 16-row block).
// BF16:  v_mfma_f32_16x16x32_bf16, K step 32; operands rounded to bf16 (RNE),
//        FP32 accumulation, bias/activation/loss in FP32.
//
// Weight source (template flag WL):
//   WL = true   the block copies its spark's weights once into LDS, every
//               layer zero-padded to whole 16-row blocks and to the padded K;
//               biases in an FP32 area after the weights.  FP32: the row pitch
//               is 2 (mod 8) 16-byte chunks and chunk c of row r sits at
//               c ^ (r & 1), so the 16-byte fragment reads served together (four
//               lanes from each half of the wavefront: rows 4a..4a+3, chunks g
//               and g + 2) hit eight distinct bank groups.  BF16: rows padded by
//               16 bytes.
//   WL = false  fragments are read from the spark row in global memory (L2),
//               with row/column guards; used when the weights exceed the LDS.
//
// Template parameters also fix the number of 16-row output blocks of every
// layer (R1..R4, 0 = absent), the wavefronts per block (NW) and the number P of
// 16-sample slabs a wavefront keeps in flight, so that all activation tiles
// live in registers.
#pragma once

#include "internal.h"

#include <math.h>

#include <type_traits>

namespace mgfwa {
namespace fit {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// FitArgs (the kernel's arguments) is declared in internal.h.


__device__ __forceinline__ floatx4 zero4()
{
    floatx4 z = {0.0f, 0.0f, 0.0f, 0.0f};
    return z;
}

// Matrix-core multiply-accumulate in place: c += a x b with the result written
// over the addend (dst = srcC) in accumulation registers.  Written as inline
// assembly because with the builtin the register allocator is free to give the
// result another register than the addend, and in a K loop over 64
// accumulator tiles it then copies accumulators around on every step.  The
// compiler does not track the matrix-core latency of these instructions:
// mfma_acc_sync() must separate them from any other write or read of the
// accumulators (zeroing before, the epilogue after).  Not volatile: a volatile
// statement is a scheduling barrier, which would keep the LDS reads of the next
// fragments from being issued ahead of the multiplies; the data dependences on
// the accumulators and operands fix the order that matters.
__device__ __forceinline__ void mfma_acc(floatx4 &c, const bf16x8 &a, const bf16x8 &b)
{
    asm("v_mfma_f32_16x16x32_bf16 %0, %1, %2, %0" : "+a"(c) : "v"(a), "v"(b));
}

__device__ __forceinline__ void mfma_acc(floatx4 &c, float a, float b)
{
    asm("v_mfma_f32_16x16x4_f32 %0, %1, %2, %0" : "+a"(c) : "v"(a), "v"(b));
}

// Orders the accumulators against mfma_acc: every earlier write of them is
// complete and 24 wait states have passed before any later instruction reads or
// writes them (more than the longest matrix-core result latency).
template <int RB, int CB>
__device__ __forceinline__ void mfma_acc_sync(floatx4 (&acc)[RB][CB])
{
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) asm volatile("" : "+a"(acc[rb][cb]));
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) asm volatile("" : "+a"(acc[rb][cb]));
}

// Four consecutive weights W[row][kbase..kbase+3] from global memory; zero
// outside the layer.
__device__ __forceinline__ floatx4 ldw4(const float *p, bool row_ok, int kbase, int fi, int vec)
{
    floatx4 r = zero4();
    if (vec) {
        if (row_ok && kbase < fi) r = *reinterpret_cast<const floatx4 *>(p);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (row_ok && kbase + e < fi) r[e] = p[e];
    }
    return r;
}

typedef unsigned uintx4 __attribute__((ext_vector_type(4)));

// ReLU of eight values as they are converted to BF16: each pair converted with
// round to nearest even (which keeps the sign), then the packed 16-bit integer
// maximum against zero (a non-negative BF16 is a non-negative integer, a
// negative one or -0 a negative integer), so this is ReLU before or after
// rounding alike.  Written with the compiler's vector conversion and
// element-wise maximum: the result feeds a matrix-core operand, and the
// compiler inserts the wait states between a vector write and a matrix-core read
// only for instructions it generates itself (an inline-assembly maximum here
// once let the multiply read stale operands).
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short shortx2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t relu_pk_bf16(float a, float b)
{
    const floatx2 f = {a, b};
    const shortx2 h = __builtin_bit_cast(shortx2, __builtin_convertvector(f, bf16x2));
    const shortx2 zero = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(h, zero));
}

__device__ __forceinline__ bf16x8 relu_to_bf16x8(floatx4 lo, floatx4 hi)
{
    const uintx4 u = {relu_pk_bf16(lo[0], lo[1]), relu_pk_bf16(lo[2], lo[3]),
                      relu_pk_bf16(hi[0], hi[1]), relu_pk_bf16(hi[2], hi[3])};
    return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ bf16x8 to_bf16x8(floatx4 lo, floatx4 hi)
{
    bf16x8 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        r[e] = (__bf16)lo[e];
        r[e + 4] = (__bf16)hi[e];
    }
    return r;
}

// One lane's view of one layer's weights, anchored at row n of output block 0
// and column 4g.
template <bool BF, bool WL>
struct WView {
    const float *gp;     // global source (WL = false)
    const char *sp;      // LDS source (WL = true)
    int fi, fo, vec, pitch, n, gq;

    __device__ __forceinline__ WView(const FitArgs &a, const float *w, const char *smem, int l,
                                     int n_, int g_)
    {
        n = n_;
        gq = g_;
        fi = a.fi[l];
        fo = a.fo[l];
        vec = a.vec[l];
        pitch = a.lpitch[l];
        if constexpr (WL) {
            constexpr int es = BF ? 2 : 4;
            // FP32: 16-byte chunk c of row r is stored at chunk c ^ (r & 1) (see
            // stage_weights); the lane's chunk in every K block is 4kb + g
            const int gq = BF ? g_ : (g_ ^ (n & 1));
            sp = smem + (size_t)(a.lw[l] + n * pitch + 4 * gq) * es;
            gp = nullptr;
        } else {
            gp = w + a.woff[l] + (size_t)n * fi + 4 * g_;
            sp = nullptr;
        }
    }

    // FP32 fragment: row 16rb + n, k = 16kb + 4g .. +3
    __device__ __forceinline__ floatx4 f32(int rb, int kb) const
    {
        if constexpr (WL) {
            return *reinterpret_cast<const floatx4 *>(sp + (size_t)(16 * rb * pitch + 16 * kb) * 4);
        } else {
            const bool ok = 16 * rb + n < fo;
            return ldw4(gp + (size_t)(ok ? 16 * rb : 0) * fi + 16 * kb, ok, 16 * kb + 4 * gq, fi,
                        vec);
        }
    }

    // BF16 fragment: row 16rb + n, k = 32kb + 4g .. +3 then 32kb + 16 + 4g .. +3
    __device__ __forceinline__ bf16x8 b16(int rb, int kb) const
    {
        if constexpr (WL) {
            const char *p = sp + (size_t)(16 * rb * pitch + 32 * kb) * 2;
            const uint2 lo = *reinterpret_cast<const uint2 *>(p);
            const uint2 hi = *reinterpret_cast<const uint2 *>(p + 32);
            return __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
        } else {
            floatx4 lo, hi;
            b16_raw(rb, kb, lo, hi);
            return to_bf16x8(lo, hi);
        }
    }

    // The FP32 weights of a BF16 fragment from global memory (WL = false),
    // converted where they are used: lo = k 32kb + 4g.., hi = k 32kb + 16 + 4g..
    __device__ __forceinline__ void b16_raw(int rb, int kb, floatx4 &lo, floatx4 &hi) const
    {
        const bool ok = 16 * rb + n < fo;
        const float *p = gp + (size_t)(ok ? 16 * rb : 0) * fi + 32 * kb;
        lo = ldw4(p, ok, 32 * kb + 4 * gq, fi, vec);
        hi = ldw4(p + 16, ok, 32 * kb + 16 + 4 * gq, fi, vec);
    }
};

// Coordinates 4c..4c+3 of explosion spark r (the regenerating staging).
__device__ __forceinline__ floatx4 regen_chunk(const SparkRegen &g, int r, int c)
{
    const int gf = r / g.lam;
    const uint32_t t = (uint32_t)g.ctrl[CTRL_GEN] + 1u;
    const float4 x4 = reinterpret_cast<const float4 *>(g.F + (size_t)gf * g.Dp)[c];
    const float x[4] = {x4.x, x4.y, x4.z, x4.w};
    const size_t pb = (size_t)(gf / g.N) * g.Dp;
    float v[4];
    explosion_chunk(x, g.A[gf], g.key, c, (uint32_t)r, t, g.box, g.lo ? g.lo + pb : nullptr,
                    g.hi ? g.hi + pb : nullptr, g.D, v);
    floatx4 out = {v[0], v[1], v[2], v[3]};
    return out;
}

// Spark coordinate j of row r: read from w, or regenerated.
__device__ __forceinline__ float spark_at(const FitArgs &a, const float *w, int r, int j)
{
    if (!a.rg.F) return w[j];
    return regen_chunk(a.rg, r, j >> 2)[j & 3];
}

// Copy the spark's weights into LDS (zero-padded layout) and its biases into
// the FP32 bias area; with a.rg.F the spark (row r) is regenerated instead of read.
template <bool BF>
__device__ __forceinline__ void stage_weights(const FitArgs &a, const float *w, int r, char *smem)
{
    float *bias = reinterpret_cast<float *>(smem + a.lbias_byte);
    const bool regen = a.rg.F != nullptr;
    for (int l = 0; l < a.nl; ++l) {
        const int fo = a.fo[l], fi = a.fi[l], rows = a.lrows[l], cols = a.lcols[l];
        const int pitch = a.lpitch[l], base = a.lw[l];
        const float *src = w + a.woff[l];
        if (a.vec[l]) {
            // 16-byte loads, four in flight per thread (fi, cols and the row
            // offsets are multiples of 4, so a chunk is all-valid or all-padding)
            const int n4 = rows * cols / 4;
            const int nt = blockDim.x;
            for (int i0 = threadIdx.x; i0 < n4; i0 += 4 * nt) {
                floatx4 v[4];
                int dst[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int idx = i0 + u * nt;
                    const int o = (4 * idx) / cols, k = 4 * idx - o * cols;
                    dst[u] = idx < n4 ? base + o * pitch + (BF ? k : k ^ ((o & 1) << 2)) : -1;
                    const bool live = idx < n4 && o < fo && k < fi;
                    v[u] = !live ? zero4()
                           : regen ? regen_chunk(a.rg, r, (a.woff[l] + o * fi + k) >> 2)
                                   : *reinterpret_cast<const floatx4 *>(src + (size_t)o * fi + k);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (dst[u] < 0) continue;
                    if constexpr (BF) {
                        const uint32_t lo = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[u][0]) |
                                            ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[u][1]) << 16);
                        const uint32_t hi = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[u][2]) |
                                            ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[u][3]) << 16);
                        *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(smem) + dst[u]) =
                            make_uint2(lo, hi);
                    } else {
                        *reinterpret_cast<floatx4 *>(reinterpret_cast<float *>(smem) + dst[u]) = v[u];
                    }
                }
            }
            for (int o = threadIdx.x; o < rows; o += blockDim.x)
                bias[a.lb[l] + o] = o < fo ? spark_at(a, w, r, a.boff[l] + o) : 0.0f;
            continue;
        }
        const int n = rows * cols;
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            const int o = idx / cols, k = idx - o * cols;
            const float v = (o < fo && k < fi) ? spark_at(a, w, r, a.woff[l] + o * fi + k) : 0.0f;
            if constexpr (BF)
                reinterpret_cast<uint16_t *>(smem)[base + o * pitch + k] =
                    __builtin_bit_cast(uint16_t, (__bf16)v);
            else
                reinterpret_cast<float *>(smem)[base + o * pitch + (k ^ ((o & 1) << 2))] = v;
        }
        for (int o = threadIdx.x; o < rows; o += blockDim.x)
            bias[a.lb[l] + o] = o < fo ? spark_at(a, w, r, a.boff[l] + o) : 0.0f;
    }
    __syncthreads();
}

// ---- first layer: B operand from the packed samples ------------------------
// SCHED bit 0: fetch the next row block's weight fragment before the current
// block's MFMAs (else right before use); bit 1: the first K block multiplies
// with a zero addend instead of clearing the accumulators first (fewer
// instructions, but more registers in most instances: enabled only where it
// measured faster).
template <bool BF, bool WL, int P, int RO, int SCHED = 1, bool FOLD = false>
__device__ __forceinline__ void layer_x(const FitArgs &a, const WView<BF, WL> &wv, int s0, int n,
                                        int g, floatx4 (&out)[P][RO], const floatx4 *c0 = nullptr)
{
    constexpr bool PF = (SCHED & 1) != 0, ZA = (SCHED & 2) != 0;
    if constexpr (!ZA) {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int rb = 0; rb < RO; ++rb) out[p][rb] = zero4();
    }
    if constexpr (!BF) {
        const float *xp[P];
#pragma unroll
        for (int p = 0; p < P; ++p) xp[p] = a.X + (size_t)(s0 + 16 * p + n) * a.in_pad + 4 * g;
        const int nkb = a.in_pad >> 4;
        // one K block of 16 columns; FIRST: zero addend
        auto kblock = [&](int kb, auto first) {
            floatx4 bx[P];
#pragma unroll
            for (int p = 0; p < P; ++p) bx[p] = *reinterpret_cast<const floatx4 *>(xp[p] + 16 * kb);
            floatx4 aw = wv.f32(0, kb);
#pragma unroll
            for (int rb = 0; rb < RO; ++rb) {
                const floatx4 an = PF && rb + 1 < RO ? wv.f32(rb + 1, kb) : aw;
                if constexpr (!PF) aw = wv.f32(rb, kb);
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int p = 0; p < P; ++p)
                        out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            aw[v], bx[p][v], decltype(first)::value && v == 0 ? zero4() : out[p][rb], 0, 0, 0);
                aw = an;
            }
        };
        if constexpr (ZA) {
            kblock(0, std::true_type());
            for (int kb = 1; kb < nkb; ++kb) kblock(kb, std::false_type());
        } else {
            for (int kb = 0; kb < nkb; ++kb) {
                floatx4 bx[P];
#pragma unroll
                for (int p = 0; p < P; ++p) bx[p] = *reinterpret_cast<const floatx4 *>(xp[p] + 16 * kb);
                floatx4 aw = wv.f32(0, kb);
#pragma unroll
                for (int rb = 0; rb < RO; ++rb) {
                    // fetch the next block's fragment before this block's MFMAs
                    const floatx4 an = PF && rb + 1 < RO ? wv.f32(rb + 1, kb) : aw;
                    if constexpr (!PF) aw = wv.f32(rb, kb);
#pragma unroll
                    for (int v = 0; v < 4; ++v)
#pragma unroll
                        for (int p = 0; p < P; ++p)
                            out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[v], bx[p][v], out[p][rb], 0, 0, 0);
                    aw = an;
                }
            }
        }
    } else {
        // lane (n, g) element e: k = 32kb + 4g + e (e < 4), 32kb + 16 + 4g + e - 4 (e >= 4)
        const uint16_t *xp[P];
#pragma unroll
        for (int p = 0; p < P; ++p) xp[p] = a.Xb + (size_t)(s0 + 16 * p + n) * a.in_pad + 4 * g;
        const int nkb = a.in_pad >> 5;
        auto kblock = [&](int kb, auto first) {
            bf16x8 bx[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const uint2 lo = *reinterpret_cast<const uint2 *>(xp[p] + 32 * kb);
                const uint2 hi = *reinterpret_cast<const uint2 *>(xp[p] + 32 * kb + 16);
                bx[p] = __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
            }
            bf16x8 aw = wv.b16(0, kb);
#pragma unroll
            for (int rb = 0; rb < RO; ++rb) {
                const bf16x8 an = PF && rb + 1 < RO ? wv.b16(rb + 1, kb) : aw;
                if constexpr (!PF) aw = wv.b16(rb, kb);
#pragma unroll
                for (int p = 0; p < P; ++p)
                    out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        aw, bx[p], decltype(first)::value ? (FOLD ? c0[rb] : zero4()) : out[p][rb],
                        0, 0, 0);
                aw = an;
            }
        };
        if constexpr (ZA) {
            kblock(0, std::true_type());
            for (int kb = 1; kb < nkb; ++kb) kblock(kb, std::false_type());
        } else {
            for (int kb = 0; kb < nkb; ++kb) {
                bf16x8 bx[P];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const uint2 lo = *reinterpret_cast<const uint2 *>(xp[p] + 32 * kb);
                    const uint2 hi = *reinterpret_cast<const uint2 *>(xp[p] + 32 * kb + 16);
                    bx[p] = __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
                }
                bf16x8 aw = wv.b16(0, kb);
#pragma unroll
                for (int rb = 0; rb < RO; ++rb) {
                    const bf16x8 an = PF && rb + 1 < RO ? wv.b16(rb + 1, kb) : aw;
                    if constexpr (!PF) aw = wv.b16(rb, kb);
#pragma unroll
                    for (int p = 0; p < P; ++p)
                        out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bx[p], out[p][rb], 0, 0, 0);
                    aw = an;
                }
            }
        }
    }
}

// ---- later layers: B operand from the previous layer's accumulators ----------
template <bool BF, bool WL, int P, int RI, int RO, int SCHED = 1, bool FOLD = false>
__device__ __forceinline__ void layer_h(const WView<BF, WL> &wv, const floatx4 (&in)[P][RI],
                                        floatx4 (&out)[P][RO], const floatx4 *c0 = nullptr)
{
    constexpr bool PF = (SCHED & 1) != 0, ZA = (SCHED & 2) != 0;
    if constexpr (!ZA) {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int rb = 0; rb < RO; ++rb) out[p][rb] = zero4();
    }
    if constexpr (!BF && !WL) {
        // fragments from the spark row in global memory (L2): a ring of GD loads
        // in flight in (kb, rb) order, so the multiplies of one fragment overlap
        // the latency of the next GD - 1 (one load ahead left the kernel waiting
        // on every fragment).  A fragment past the layer's columns is zero and
        // issues no load; K blocks past them are skipped (a predicate, not an
        // early exit, so that the loop stays fully unrolled).
        constexpr int T = RI * RO, GD = T < 8 ? T : 8;
        const int nkb = (wv.fi + 15) >> 4 < RI ? (wv.fi + 15) >> 4 : RI;
        floatx4 ring[GD];
#pragma unroll
        for (int t = 0; t < GD; ++t) ring[t] = wv.f32(t % RO, t / RO);
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int kb = t / RO, rb = t % RO;
            const floatx4 aw = ring[t % GD];
            if (t + GD < T) ring[t % GD] = wv.f32((t + GD) % RO, (t + GD) / RO);
            if (kb < nkb) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int p = 0; p < P; ++p)
                        out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            aw[v], in[p][kb][v], ZA && kb == 0 && v == 0 ? zero4() : out[p][rb], 0,
                            0, 0);
            }
        }
    } else if constexpr (!BF) {
        // fragments of (kb, rb) in order; the next one is fetched before the
        // current one's MFMAs so the LDS latency overlaps matrix work
        // staged weights are zero-padded to RI blocks: no early exit needed
        const int nkb = WL ? RI : ((wv.fi + 15) >> 4 < RI ? (wv.fi + 15) >> 4 : RI);
        floatx4 aw = wv.f32(0, 0);
#pragma unroll
        for (int kb = 0; kb < RI; ++kb) {
            if (kb >= nkb) break;
#pragma unroll
            for (int rb = 0; rb < RO; ++rb) {
                floatx4 an = aw;
                if constexpr (!PF) aw = wv.f32(rb, kb);
                else if (rb + 1 < RO) an = wv.f32(rb + 1, kb);
                else if (kb + 1 < nkb) an = wv.f32(0, kb + 1);
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int p = 0; p < P; ++p)
                        out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            aw[v], in[p][kb][v], ZA && kb == 0 && v == 0 ? zero4() : out[p][rb], 0, 0, 0);
                aw = an;
            }
        }
    } else if constexpr (!WL && RI <= 8) {
        // BF16 with fragments from global memory, input layer up to 128 wide: a
        // ring of GD fragment loads in flight (their FP32 weights, converted at
        // use), as in the FP32 case.  (With 256-wide input layers the ring's
        // registers add spills and it measured slower: 0.85 -> 1.39 ms at
        // 32-240-240-10, against 0.41 -> 0.34 ms at 32-128-128-128-10.)
        constexpr int NKB = (RI + 1) / 2, T = NKB * RO, GD = T < 4 ? T : 4;
        const int nkb = (wv.fi + 31) >> 5 < NKB ? (wv.fi + 31) >> 5 : NKB;
        floatx4 rlo[GD], rhi[GD];
#pragma unroll
        for (int t = 0; t < GD; ++t) wv.b16_raw(t % RO, t / RO, rlo[t], rhi[t]);
        bf16x8 bx[P];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int kb = t / RO, rb = t % RO;
            if (rb == 0 && kb < nkb) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    floatx4 hi = zero4();
                    if (2 * kb + 1 < RI) hi = in[p][(2 * kb + 1) < RI ? 2 * kb + 1 : 0];
                    if constexpr (FOLD) bx[p] = relu_to_bf16x8(in[p][2 * kb], hi);
                    else bx[p] = to_bf16x8(in[p][2 * kb], hi);
                }
            }
            const bf16x8 aw = to_bf16x8(rlo[t % GD], rhi[t % GD]);
            if (t + GD < T) wv.b16_raw((t + GD) % RO, (t + GD) / RO, rlo[t % GD], rhi[t % GD]);
            if (kb < nkb) {
#pragma unroll
                for (int p = 0; p < P; ++p)
                    out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        aw, bx[p], ZA && kb == 0 ? (FOLD ? c0[rb] : zero4()) : out[p][rb], 0, 0,
                        0);
            }
        }
    } else {
        constexpr int NKB = (RI + 1) / 2;
        const int nkb = WL ? NKB : ((wv.fi + 31) >> 5 < NKB ? (wv.fi + 31) >> 5 : NKB);
        bf16x8 aw = wv.b16(0, 0);
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            if (kb >= nkb) break;
            bf16x8 bx[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                floatx4 hi = zero4();
                if (2 * kb + 1 < RI) hi = in[p][(2 * kb + 1) < RI ? 2 * kb + 1 : 0];
                if constexpr (FOLD) bx[p] = relu_to_bf16x8(in[p][2 * kb], hi);
                else bx[p] = to_bf16x8(in[p][2 * kb], hi);
            }
#pragma unroll
            for (int rb = 0; rb < RO; ++rb) {
                bf16x8 an = aw;
                if constexpr (!PF) aw = wv.b16(rb, kb);
                else if (rb + 1 < RO) an = wv.b16(rb + 1, kb);
                else if (kb + 1 < nkb) an = wv.b16(0, kb + 1);
#pragma unroll
                for (int p = 0; p < P; ++p)
                    out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        aw, bx[p], ZA && kb == 0 ? (FOLD ? c0[rb] : zero4()) : out[p][rb], 0, 0, 0);
                aw = an;
            }
        }
    }
}

// ---- bias, activation, loss ---------------------------------------------------
// ReLU as a signed integer maximum against zero: a positive float is a positive
// integer, a negative one and -0 negative integers, so this is z > 0 ? z : +0
// for every non-NaN z in one instruction (the float maximum takes two: the
// compiler quiets a possible signalling NaN first).
template <int ACT>
__device__ __forceinline__ float act_c(float z)
{
    if constexpr (ACT == 1) {
        const int i = __builtin_bit_cast(int, z);
        return __builtin_bit_cast(float, i > 0 ? i : 0);
    }
    else if constexpr (ACT == 2) return tanhf(z);
    else if constexpr (ACT == 3) return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
    else return z;
}

template <int ACT, int P, int R>
__device__ __forceinline__ void add_act(floatx4 (&h)[P][R], const floatx4 (&bb)[R])
{
#pragma unroll
    for (int rb = 0; rb < R; ++rb)
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int v = 0; v < 4; ++v) h[p][rb][v] = act_c<ACT>(h[p][rb][v] + bb[rb][v]);
}

// This lane's biases of layer l (rows 16rb + 4g .. +3 of every output block).
template <bool WL, int R>
__device__ __forceinline__ void load_bias(const FitArgs &a, const float *w, const char *smem, int l,
                                          int g, floatx4 (&bb)[R])
{
    const int fo = a.fo[l];
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
        if constexpr (WL) {
            bb[rb] = *reinterpret_cast<const floatx4 *>(smem + a.lbias_byte +
                                                        (size_t)(a.lb[l] + 16 * rb + 4 * g) * 4);
        } else {
            const float *bias = w + a.boff[l];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = 16 * rb + 4 * g + v;
                bb[rb][v] = o < fo ? bias[o] : 0.0f;
            }
        }
    }
}

// Bias then activation of layer l.  ACT >= 0 fixes the hidden activation at
// compile time; ACT < 0 dispatches once per call on the runtime code.
template <int ACT, bool WL, int P, int R>
__device__ __forceinline__ void bias_act(const FitArgs &a, const float *w, const char *smem, int l,
                                         int g, bool apply_act, floatx4 (&h)[P][R])
{
    floatx4 bb[R];
    load_bias<WL, R>(a, w, smem, l, g, bb);
    if (!apply_act) {
        add_act<0, P, R>(h, bb);
        return;
    }
    if constexpr (ACT >= 0) {
        add_act<ACT, P, R>(h, bb);
    } else {
        switch (a.act[l]) {
        case 1: add_act<1, P, R>(h, bb); break;
        case 2: add_act<2, P, R>(h, bb); break;
        case 3: add_act<3, P, R>(h, bb); break;
        default: add_act<0, P, R>(h, bb); break;
        }
    }
}

// v and its partner in lane l ^ 16 (or l ^ 32), exchanged with gfx950's row-swap
// instructions (plain VALU work, no LDS round trip).  Each lane gets both values,
// its own and its partner's in some order; sums and maxima of the pair are then
// the same in every lane, bit for bit, as v op shfl_xor(v, 16).
__device__ __forceinline__ void pair16(float v, float &a, float &b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

__device__ __forceinline__ void pair32(float v, float &a, float &b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

// Sum / maximum over the four lanes l, l^16, l^32, l^48.
__device__ __forceinline__ float xor_sum4(float v)
{
    float a, b;
    pair16(v, a, b);
    v = a + b;
    pair32(v, a, b);
    return a + b;
}

__device__ __forceinline__ float xor_max4(float v)
{
    float a, b;
    pair16(v, a, b);
    v = fmaxf(a, b);
    pair32(v, a, b);
    return fmaxf(a, b);
}

// Sum of the per-sample losses of this wavefront's P slabs (valid in lanes g == 0).
template <int P, int R>
__device__ __forceinline__ float slab_loss(const FitArgs &a, int l, int s0, int n, int g,
                                           const floatx4 (&z)[P][R])
{
    const int fo = a.fo[l];
    float total = 0.0f;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int s = s0 + 16 * p + n;
        float ls;
        if (a.loss == 0) {
            float acc = 0.0f;
            const float *yrow = a.Y + (size_t)s * fo;
#pragma unroll
            for (int rb = 0; rb < R; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int o = 16 * rb + 4 * g + v;
                    if (o < fo) {
                        const float e = z[p][rb][v] - yrow[o];
                        acc = __builtin_fmaf(e, e, acc);
                    }
                }
            ls = xor_sum4(acc);
        } else {
            const int label = a.lab[s];
            float mx = -__builtin_huge_valf(), zl = 0.0f;
#pragma unroll
            for (int rb = 0; rb < R; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int o = 16 * rb + 4 * g + v;
                    if (o < fo) {
                        mx = fmaxf(mx, z[p][rb][v]);
                        if (o == label) zl = z[p][rb][v];
                    }
                }
            mx = xor_max4(mx);
            // se = sum over all classes, rest = sum over classes other than the label
            float se = 0.0f, rest = 0.0f;
#pragma unroll
            for (int rb = 0; rb < R; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int o = 16 * rb + 4 * g + v;
                    if (o < fo) {
                        const float e = expf(z[p][rb][v] - mx);
                        se += e;
                        if (o != label) rest += e;
                    }
                }
            se = xor_sum4(se);
            rest = xor_sum4(rest);
            zl = xor_sum4(zl);
            // When the label holds the maximum the loss is log(1 + rest): log1p
            // keeps small losses accurate instead of cancelling max + log(se) - z.
            ls = zl == mx ? log1pf(rest) : (mx - zl) + logf(se);
        }
        if (s < a.S && g == 0) total += ls;
    }
    return total;
}

// Block `bid` of a fitness launch: spark r = bid / bpr, sample range c = bid % bpr.
template <bool BF, bool WL, int NW, int P, int ACT, int R1, int R2, int R3, int R4, int SCHED>
__device__ __forceinline__ void fit_body(const FitArgs &a, int bid)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ float red[NW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int r = bid / a.bpr, c = bid % a.bpr;
    const float *w = a.W + (size_t)r * a.ld;
    if constexpr (WL) stage_weights<BF>(a, w, r, smem);
    const WView<BF, WL> w0(a, w, smem, 0, n, g), w1(a, w, smem, 1, n, g);
    const WView<BF, WL> w2(a, w, smem, 2, n, g), w3(a, w, smem, 3, n, g);
    const int s_begin = c * a.spb;
    const int s_end = min(s_begin + a.spb, a.S_pad);
    float lsum = 0.0f;
    for (int s0 = s_begin + wave * 16 * P; s0 < s_end; s0 += NW * 16 * P) {
        // The staged weights are re-read from LDS for every slab: without this
        // fence the compiler hoists those reads out of the loop and, short of
        // registers, spills the whole weight fragment set to scratch memory.
        asm volatile("" ::: "memory");
        // FOLD (BF16, zero-addend instances, ReLU): each layer's bias is the
        // addend of its first K block and the ReLU of a hidden layer is applied
        // to its BF16-rounded values as the next layer converts them, so no
        // per-value bias or activation pass runs.
        constexpr bool FOLD = BF && (SCHED & 2) != 0 && ACT == 1;
        floatx4 h1[P][R1], c1[R1];
        if constexpr (FOLD) load_bias<WL, R1>(a, w, smem, 0, g, c1);
        layer_x<BF, WL, P, R1, SCHED, FOLD>(a, w0, s0, n, g, h1, c1);
        if constexpr (R2 == 0) {
            if constexpr (!FOLD) bias_act<ACT, WL, P, R1>(a, w, smem, 0, g, false, h1);
            lsum += slab_loss<P, R1>(a, 0, s0, n, g, h1);
        } else {
            if constexpr (!FOLD) bias_act<ACT, WL, P, R1>(a, w, smem, 0, g, true, h1);
            floatx4 h2[P][R2], c2[R2];
            if constexpr (FOLD) load_bias<WL, R2>(a, w, smem, 1, g, c2);
            layer_h<BF, WL, P, R1, R2, SCHED, FOLD>(w1, h1, h2, c2);
            if constexpr (R3 == 0) {
                if constexpr (!FOLD) bias_act<ACT, WL, P, R2>(a, w, smem, 1, g, false, h2);
                lsum += slab_loss<P, R2>(a, 1, s0, n, g, h2);
            } else {
                if constexpr (!FOLD) bias_act<ACT, WL, P, R2>(a, w, smem, 1, g, true, h2);
                floatx4 h3[P][R3], c3[R3];
                if constexpr (FOLD) load_bias<WL, R3>(a, w, smem, 2, g, c3);
                layer_h<BF, WL, P, R2, R3, SCHED, FOLD>(w2, h2, h3, c3);
                if constexpr (R4 == 0) {
                    if constexpr (!FOLD) bias_act<ACT, WL, P, R3>(a, w, smem, 2, g, false, h3);
                    lsum += slab_loss<P, R3>(a, 2, s0, n, g, h3);
                } else {
                    if constexpr (!FOLD) bias_act<ACT, WL, P, R3>(a, w, smem, 2, g, true, h3);
                    floatx4 h4[P][R4], c4[R4];
                    if constexpr (FOLD) load_bias<WL, R4>(a, w, smem, 3, g, c4);
                    layer_h<BF, WL, P, R3, R4, SCHED, FOLD>(w3, h3, h4, c4);
                    if constexpr (!FOLD) bias_act<ACT, WL, P, R4>(a, w, smem, 3, g, false, h4);
                    lsum += slab_loss<P, R4>(a, 3, s0, n, g, h4);
                }
            }
        }
    }
    // fixed-order reduction: wavefront butterfly, then the wavefronts in order
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) red[wave] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = red[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t += red[i];
        a.partial[(size_t)r * a.bpr + c] = t;
    }
}

template <bool BF, bool WL, int NW, int P, int ACT, int R1, int R2, int R3, int R4, int SCHED = 1>
__global__ __launch_bounds__(NW * 64) void k_fit(FitArgs a)
{
    fit_body<BF, WL, NW, P, ACT, R1, R2, R3, R4, SCHED>(a, xcd_remap(blockIdx.x, gridDim.x));
}

// The same kernel over the fitness launch `which` of many jobs that share it.
// A job's range of grouped blocks starts on XCD 0, so its blocks take the XCD
// remap of its own launch and each runs the block it would have run there.
template <bool BF, bool WL, int NW, int P, int ACT, int R1, int R2, int R3, int R4, int SCHED = 1>
__global__ __launch_bounds__(NW * 64) void k_fit_group(GroupTable t, int which)
{
    const int j = group_job(t, blockIdx.x);
    const int local = blockIdx.x - t.start[j], n = t.gx[j] * t.gy[j];
    if (local >= n) return;   // padding
    // a private copy: read through a pointer into global memory, the arguments
    // would be reloaded after every store the body makes
    const FitArgs a = t.job[j]->fit[which].a;
    fit_body<BF, WL, NW, P, ACT, R1, R2, R3, R4, SCHED>(a, xcd_remap(local, n));
}

// One compiled fitness kernel: precision, weight source, wavefronts per block,
// slabs in flight, hidden activation (-1: chosen at run time), 16-row blocks
// per layer.
struct KernelEntry {
    int bf16, wl, nw, P, act, R[MAXL];
    const void *fn;         // k_fit
    const void *gfn;        // k_fit_group of the same instance
};

#define FIT_ENTRY_SCHED(BF, WL, NW, P, ACT, SCHED, R1, R2, R3, R4)                          \
    {BF, WL, NW, P, ACT, {R1, R2, R3, R4},                                                   \
     reinterpret_cast<const void *>(&::mgfwa::fit::k_fit<BF, WL, NW, P, ACT, R1, R2, R3, R4, SCHED>), \
     reinterpret_cast<const void *>(&::mgfwa::fit::k_fit_group<BF, WL, NW, P, ACT, R1, R2, R3, R4, SCHED>)}
#define FIT_ENTRY_ACT(BF, WL, NW, P, ACT, R1, R2, R3, R4) \
    FIT_ENTRY_SCHED(BF, WL, NW, P, ACT, 1, R1, R2, R3, R4)
#define FIT_ENTRY(BF, WL, NW, P, R1, R2, R3, R4) FIT_ENTRY_ACT(BF, WL, NW, P, -1, R1, R2, R3, R4)
// global-weight kernels in both precisions
#define FIT_BOTH(P, R1, R2, R3, R4) \
    FIT_ENTRY(false, false, 4, P, R1, R2, R3, R4), FIT_ENTRY(true, false, 4, P, R1, R2, R3, R4)
// LDS-weight kernels in both precisions
#define FIT_BOTH_LDS(P, R1, R2, R3, R4) \
    FIT_ENTRY(false, true, 4, P, R1, R2, R3, R4), FIT_ENTRY(true, true, 4, P, R1, R2, R3, R4)

}  // namespace fit
}  // namespace mgfwa
