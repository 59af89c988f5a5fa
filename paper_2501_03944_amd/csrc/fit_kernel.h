// Fitness kernel template, instantiated by the fit_*.hip files.
//
// Fitness of every spark (Alg. 1: evaluate all the sparks in parallel): the
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
// the result is deterministic and independent of the launch geometry's timing.
//
// FP32:  v_mfma_f32_16x16x4_f32,  K step 4 per MFMA (4 MFMAs per 16-row block).
// BF16:  v_mfma_f32_16x16x32_bf16, K step 32; operands rounded to bf16 (RNE),
//        FP32 accumulation, bias/activation/loss in FP32.
//
// Template parameters fix the number of 16-row output blocks of every layer
// (R1..R4, 0 = absent) and the number P of 16-sample slabs a wavefront keeps in
// flight, so that all activation tiles live in registers.
#pragma once

#include "internal.h"

#include <math.h>

namespace mgfwa {
namespace fit {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TPB = 256;   // 4 wavefronts
constexpr int WAVES = TPB / 64;

struct FitArgs {
    const float *W;        // spark rows
    size_t ld;             // row pitch (floats)
    int rows;
    const float *X;        // [S_pad][in_pad] (FP32 kernels)
    const uint16_t *Xb;    // [S_pad][in_pad] bf16 bits (BF16 kernels)
    int in_pad, S, S_pad;
    int nl;
    int fi[MAXL], fo[MAXL], woff[MAXL], boff[MAXL], act[MAXL], vec[MAXL];
    int loss;
    const float *Y;        // [S_pad][out]
    const int32_t *lab;    // [S_pad]
    int bpr, spb;
    float *partial;        // [rows][bpr]
};

__device__ __forceinline__ floatx4 zero4()
{
    floatx4 z = {0.0f, 0.0f, 0.0f, 0.0f};
    return z;
}

// Four consecutive weights W[row][kbase..kbase+3]; zero outside the layer.
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

__device__ __forceinline__ float act_fn(int act, float z)
{
    switch (act) {
    case 1: return z > 0.0f ? z : 0.0f;
    case 2: return tanhf(z);
    case 3: return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
    default: return z;
    }
}

// ---- first layer: B operand from the packed samples ------------------------
template <int P, int RO>
__device__ __forceinline__ void layer_x_f32(const FitArgs &a, const float *w, int s0, int n, int g,
                                            floatx4 (&out)[P][RO])
{
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int rb = 0; rb < RO; ++rb) out[p][rb] = zero4();
    const int fi = a.fi[0], fo = a.fo[0], vec = a.vec[0];
    const float *xp[P];
#pragma unroll
    for (int p = 0; p < P; ++p) xp[p] = a.X + (size_t)(s0 + 16 * p + n) * a.in_pad + 4 * g;
    const float *wr[RO];
    bool rok[RO];
#pragma unroll
    for (int rb = 0; rb < RO; ++rb) {
        const int row = 16 * rb + n;
        rok[rb] = row < fo;
        wr[rb] = w + a.woff[0] + (size_t)(rok[rb] ? row : 0) * fi + 4 * g;
    }
    const int nkb = a.in_pad >> 4;
    for (int kb = 0; kb < nkb; ++kb) {
        floatx4 bx[P];
#pragma unroll
        for (int p = 0; p < P; ++p) bx[p] = *reinterpret_cast<const floatx4 *>(xp[p] + 16 * kb);
        const int kbase = 16 * kb + 4 * g;
#pragma unroll
        for (int rb = 0; rb < RO; ++rb) {
            const floatx4 aw = ldw4(wr[rb] + 16 * kb, rok[rb], kbase, fi, vec);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int p = 0; p < P; ++p)
                    out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[v], bx[p][v], out[p][rb], 0, 0, 0);
        }
    }
}

template <int P, int RO>
__device__ __forceinline__ void layer_x_bf16(const FitArgs &a, const float *w, int s0, int n,
                                             int g, floatx4 (&out)[P][RO])
{
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int rb = 0; rb < RO; ++rb) out[p][rb] = zero4();
    const int fi = a.fi[0], fo = a.fo[0], vec = a.vec[0];
    const uint16_t *xp[P];
#pragma unroll
    for (int p = 0; p < P; ++p) xp[p] = a.Xb + (size_t)(s0 + 16 * p + n) * a.in_pad + 4 * g;
    const float *wr[RO];
    bool rok[RO];
#pragma unroll
    for (int rb = 0; rb < RO; ++rb) {
        const int row = 16 * rb + n;
        rok[rb] = row < fo;
        wr[rb] = w + a.woff[0] + (size_t)(rok[rb] ? row : 0) * fi + 4 * g;
    }
    const int nkb = a.in_pad >> 5;
    for (int kb = 0; kb < nkb; ++kb) {
        // lane (n, g) element e: k = 32kb + 4g + e (e < 4), 32kb + 16 + 4g + e - 4 (e >= 4)
        bf16x8 bx[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint2 lo = *reinterpret_cast<const uint2 *>(xp[p] + 32 * kb);
            const uint2 hi = *reinterpret_cast<const uint2 *>(xp[p] + 32 * kb + 16);
            const uint4 q = make_uint4(lo.x, lo.y, hi.x, hi.y);
            bx[p] = __builtin_bit_cast(bf16x8, q);
        }
        const int k0 = 32 * kb + 4 * g;
#pragma unroll
        for (int rb = 0; rb < RO; ++rb) {
            const floatx4 lo = ldw4(wr[rb] + 32 * kb, rok[rb], k0, fi, vec);
            const floatx4 hi = ldw4(wr[rb] + 32 * kb + 16, rok[rb], k0 + 16, fi, vec);
            const bf16x8 aw = to_bf16x8(lo, hi);
#pragma unroll
            for (int p = 0; p < P; ++p)
                out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bx[p], out[p][rb], 0, 0, 0);
        }
    }
}

// ---- later layers: B operand from the previous layer's accumulators ----------
template <int P, int RI, int RO>
__device__ __forceinline__ void layer_h_f32(const FitArgs &a, const float *w, int l, int n, int g,
                                            const floatx4 (&in)[P][RI], floatx4 (&out)[P][RO])
{
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int rb = 0; rb < RO; ++rb) out[p][rb] = zero4();
    const int fi = a.fi[l], fo = a.fo[l], vec = a.vec[l];
    const float *wr[RO];
    bool rok[RO];
#pragma unroll
    for (int rb = 0; rb < RO; ++rb) {
        const int row = 16 * rb + n;
        rok[rb] = row < fo;
        wr[rb] = w + a.woff[l] + (size_t)(rok[rb] ? row : 0) * fi + 4 * g;
    }
#pragma unroll
    for (int kb = 0; kb < RI; ++kb) {
        if (16 * kb >= fi) break;
        const int kbase = 16 * kb + 4 * g;
#pragma unroll
        for (int rb = 0; rb < RO; ++rb) {
            const floatx4 aw = ldw4(wr[rb] + 16 * kb, rok[rb], kbase, fi, vec);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int p = 0; p < P; ++p)
                    out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[v], in[p][kb][v], out[p][rb], 0, 0, 0);
        }
    }
}

template <int P, int RI, int RO>
__device__ __forceinline__ void layer_h_bf16(const FitArgs &a, const float *w, int l, int n,
                                             int g, const floatx4 (&in)[P][RI],
                                             floatx4 (&out)[P][RO])
{
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int rb = 0; rb < RO; ++rb) out[p][rb] = zero4();
    const int fi = a.fi[l], fo = a.fo[l], vec = a.vec[l];
    const float *wr[RO];
    bool rok[RO];
#pragma unroll
    for (int rb = 0; rb < RO; ++rb) {
        const int row = 16 * rb + n;
        rok[rb] = row < fo;
        wr[rb] = w + a.woff[l] + (size_t)(rok[rb] ? row : 0) * fi + 4 * g;
    }
    constexpr int NKB = (RI + 1) / 2;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
        if (32 * kb >= fi) break;
        bf16x8 bx[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const floatx4 lo = in[p][2 * kb];
            floatx4 hi = zero4();
            if (2 * kb + 1 < RI) hi = in[p][(2 * kb + 1) < RI ? 2 * kb + 1 : 0];
            bx[p] = to_bf16x8(lo, hi);
        }
        const int k0 = 32 * kb + 4 * g;
#pragma unroll
        for (int rb = 0; rb < RO; ++rb) {
            const floatx4 lo = ldw4(wr[rb] + 32 * kb, rok[rb], k0, fi, vec);
            const floatx4 hi = ldw4(wr[rb] + 32 * kb + 16, rok[rb], k0 + 16, fi, vec);
            const bf16x8 aw = to_bf16x8(lo, hi);
#pragma unroll
            for (int p = 0; p < P; ++p)
                out[p][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bx[p], out[p][rb], 0, 0, 0);
        }
    }
}

// ---- bias, activation, loss ---------------------------------------------------
template <int P, int R>
__device__ __forceinline__ void bias_act(const FitArgs &a, const float *w, int l, int g,
                                         bool apply_act, floatx4 (&h)[P][R])
{
    const int fo = a.fo[l];
    const float *bias = w + a.boff[l];
    const int act = apply_act ? a.act[l] : 0;
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
        floatx4 bb;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = 16 * rb + 4 * g + v;
            bb[v] = o < fo ? bias[o] : 0.0f;
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int v = 0; v < 4; ++v) h[p][rb][v] = act_fn(act, h[p][rb][v] + bb[v]);
    }
}

__device__ __forceinline__ float xor_sum4(float v)
{
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

__device__ __forceinline__ float xor_max4(float v)
{
    v = fmaxf(v, __shfl_xor(v, 16));
    v = fmaxf(v, __shfl_xor(v, 32));
    return v;
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

template <bool BF, int P, int RI, int RO>
__device__ __forceinline__ void layer_h(const FitArgs &a, const float *w, int l, int n, int g,
                                        const floatx4 (&in)[P][RI], floatx4 (&out)[P][RO])
{
    if constexpr (BF) layer_h_bf16<P, RI, RO>(a, w, l, n, g, in, out);
    else layer_h_f32<P, RI, RO>(a, w, l, n, g, in, out);
}

template <bool BF, int P, int R1, int R2, int R3, int R4>
__global__ __launch_bounds__(TPB) void k_fit(FitArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int r = bid / a.bpr, c = bid % a.bpr;
    const float *w = a.W + (size_t)r * a.ld;
    const int s_begin = c * a.spb;
    const int s_end = min(s_begin + a.spb, a.S_pad);
    float lsum = 0.0f;
    for (int s0 = s_begin + wave * 16 * P; s0 < s_end; s0 += WAVES * 16 * P) {
        floatx4 h1[P][R1];
        if constexpr (BF) layer_x_bf16<P, R1>(a, w, s0, n, g, h1);
        else layer_x_f32<P, R1>(a, w, s0, n, g, h1);
        if constexpr (R2 == 0) {
            bias_act<P, R1>(a, w, 0, g, false, h1);
            lsum += slab_loss<P, R1>(a, 0, s0, n, g, h1);
        } else {
            bias_act<P, R1>(a, w, 0, g, true, h1);
            floatx4 h2[P][R2];
            layer_h<BF, P, R1, R2>(a, w, 1, n, g, h1, h2);
            if constexpr (R3 == 0) {
                bias_act<P, R2>(a, w, 1, g, false, h2);
                lsum += slab_loss<P, R2>(a, 1, s0, n, g, h2);
            } else {
                bias_act<P, R2>(a, w, 1, g, true, h2);
                floatx4 h3[P][R3];
                layer_h<BF, P, R2, R3>(a, w, 2, n, g, h2, h3);
                if constexpr (R4 == 0) {
                    bias_act<P, R3>(a, w, 2, g, false, h3);
                    lsum += slab_loss<P, R3>(a, 2, s0, n, g, h3);
                } else {
                    bias_act<P, R3>(a, w, 2, g, true, h3);
                    floatx4 h4[P][R4];
                    layer_h<BF, P, R3, R4>(a, w, 3, n, g, h3, h4);
                    bias_act<P, R4>(a, w, 3, g, false, h4);
                    lsum += slab_loss<P, R4>(a, 3, s0, n, g, h4);
                }
            }
        }
    }
    // fixed-order reduction: wavefront butterfly, then the 4 wavefronts in order
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) lsum += __shfl_xor(lsum, off);
    __shared__ float red[WAVES];
    if (lane == 0) red[wave] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = red[0];
#pragma unroll
        for (int i = 1; i < WAVES; ++i) t += red[i];
        a.partial[(size_t)r * a.bpr + c] = t;
    }
}


// One compiled fitness kernel: precision, slabs in flight, 16-row blocks per layer.
struct KernelEntry {
    int bf16, P, R[MAXL];
    const void *fn;
};

#define FIT_ENTRY(BF, P, R1, R2, R3, R4) \
    {BF, P, {R1, R2, R3, R4}, reinterpret_cast<const void *>(&::mgfwa::fit::k_fit<BF, P, R1, R2, R3, R4>)}
#define FIT_BOTH(P, R1, R2, R3, R4) FIT_ENTRY(false, P, R1, R2, R3, R4), FIT_ENTRY(true, P, R1, R2, R3, R4)

}  // namespace fit
}  // namespace mgfwa
