// Wide-first-layer fitness: packing of sparks and samples, kernel instances,
// plan selection and launches (kernel template in fit_wide.h).
#include "fit_wide.h"

#include <cstdlib>

namespace mgfwa {

using namespace fit;

namespace {

constexpr int TPB = 256;
constexpr int MAX_GRID_Y = 65535;

// One 16-byte chunk of a packed spark row per thread.  Chunk ranges:
//   W1aug  [Kp/32][256][32]  K-blocked: value(o, k) = W1[o][k] (k < in),
//                        b1[o] (k == in), 0 otherwise, at ((k/32)*256 + o)*32 + k%32
//   W2     [16][256]     BF16: chunk (i, kb, g) holds W2[i][32kb + p(g, e)], e = 0..7,
//                        p(g, e) = 4g + e (e < 4) or 16 + 4g + e - 4 (e >= 4);
//                        FP32: natural order
//   b2     [16]          FP32
constexpr int PACK_CPT = 4;   // 16-byte chunks per thread (strided by the block)
constexpr int PACK_RPB = 4;   // spark rows per block

// One 16-byte output chunk of a packed row (see the layout above).
template <bool BF>
__device__ __forceinline__ void pack_chunk(const float *__restrict__ w, char *__restrict__ wp,
                                           int chunk, int c1, int c2, int in, int hid, int out,
                                           int woff1, int boff1, int woff2, int boff2)
{
    constexpr int ES = BF ? 2 : 4, EPC = 16 / ES;   // elements per chunk
    float v[EPC];
    if (chunk < c1) {
        const int e0 = chunk * EPC, kb = e0 / (WT_M * WT_K), rem = e0 % (WT_M * WT_K);
        const int o = rem / WT_K, k0 = kb * WT_K + rem % WT_K;
        const float *src = w + woff1 + (size_t)o * in + k0;
        if (o < hid && k0 + EPC <= in && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
            // inside W1 and 16-byte aligned: vector loads
#pragma unroll
            for (int e = 0; e < EPC; e += 4) {
                const float4 t = *reinterpret_cast<const float4 *>(src + e);
                v[e] = t.x;
                v[e + 1] = t.y;
                v[e + 2] = t.z;
                v[e + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const int k = k0 + e;
                float x = 0.0f;
                if (o < hid) {
                    if (k < in) x = w[woff1 + (size_t)o * in + k];
                    else if (k == in) x = w[boff1 + o];
                }
                v[e] = x;
            }
        }
    } else if (chunk < c1 + c2) {
        const int e0 = (chunk - c1) * EPC, i = e0 / WT_M, c0 = e0 % WT_M;
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            int col = c0 + e;
            if (BF) {
                const int blk = c0 & ~31, g = (c0 & 31) >> 3;   // c0 = 32kb + 8g
                col = blk + (e < 4 ? 4 * g + e : 16 + 4 * g + e - 4);
            }
            v[e] = (i < out && col < hid) ? w[woff2 + (size_t)i * hid + col] : 0.0f;
        }
    } else {
        const int i0 = (chunk - c1 - c2) * 4;
        float *dst = reinterpret_cast<float *>(wp + (size_t)c1 * 16 + (size_t)c2 * 16);
        float4 b;
        b.x = i0 + 0 < out ? w[boff2 + i0 + 0] : 0.0f;
        b.y = i0 + 1 < out ? w[boff2 + i0 + 1] : 0.0f;
        b.z = i0 + 2 < out ? w[boff2 + i0 + 2] : 0.0f;
        b.w = i0 + 3 < out ? w[boff2 + i0 + 3] : 0.0f;
        reinterpret_cast<float4 *>(dst)[i0 / 4] = b;
        return;
    }
    uint4 q;
    if constexpr (BF) {
        uint32_t h[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            h[e] = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[2 * e]) |
                   ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[2 * e + 1]) << 16);
        q = make_uint4(h[0], h[1], h[2], h[3]);
    } else {
        q = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                       __float_as_uint(v[3]));
    }
    reinterpret_cast<uint4 *>(wp)[chunk] = q;
}

// A block packs PACK_RPB rows x (PACK_CPT * TPB) chunks: fat blocks, so the
// dispatcher is not what bounds the pass.
template <bool BF>
__global__ __launch_bounds__(TPB) void k_pack_wide_rows(const float *__restrict__ W, size_t ld,
                                                        int rows, char *__restrict__ Wp, size_t pr,
                                                        int in, int hid, int out, int Kp, int woff1,
                                                        int boff1, int woff2, int boff2)
{
    constexpr int ES = BF ? 2 : 4, EPC = 16 / ES;   // elements per chunk
    const int c1 = WT_M * Kp / EPC;                  // chunks of W1aug
    const int c2 = 16 * WT_M / EPC;                  // chunks of W2
    const int nchunk = c1 + c2 + 4;
    const int cfirst = blockIdx.x * TPB * PACK_CPT + threadIdx.x;
    for (int r0 = blockIdx.y * PACK_RPB; r0 < rows; r0 += gridDim.y * PACK_RPB) {
        const int rend = r0 + PACK_RPB < rows ? r0 + PACK_RPB : rows;
        for (int r = r0; r < rend; ++r) {
            const float *w = W + (size_t)r * ld;
            char *wp = Wp + (size_t)r * pr;
#pragma unroll
            for (int i = 0; i < PACK_CPT; ++i) {
                const int chunk = cfirst + i * TPB;
                if (chunk < nchunk)
                    pack_chunk<BF>(w, wp, chunk, c1, c2, in, hid, out, woff1, boff1, woff2, boff2);
            }
        }
    }
}

// Samples for the wide kernel, column `in` = 1 (the folded bias), K-blocked per
// 256-sample tile: element (s, k) at ((s/256 * Kp/32 + k/32) * 256 + s%256) * 32 + k%32,
// so one K step of one sample tile is a contiguous 256 x 32 block.
template <bool BF>
__global__ __launch_bounds__(TPB) void k_pack_wide_x(const float *__restrict__ x, int S, int S_pad,
                                                     int in, int Kp, char *__restrict__ Xw)
{
    const size_t tid = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (tid >= (size_t)S_pad * Kp) return;
    const int s = (int)(tid / Kp), k = (int)(tid % Kp);
    float v = 0.0f;
    if (s < S) v = k < in ? x[(size_t)s * in + k] : (k == in ? 1.0f : 0.0f);
    const int nk = Kp / WT_K;
    const size_t dst = (((size_t)(s / WT_N) * nk + k / WT_K) * WT_N + s % WT_N) * WT_K + k % WT_K;
    if constexpr (BF) reinterpret_cast<uint16_t *>(Xw)[dst] = __builtin_bit_cast(uint16_t, (__bf16)v);
    else reinterpret_cast<float *>(Xw)[dst] = v;
}

__global__ __launch_bounds__(256) void k_wide_finalize(const float *__restrict__ partial, int rows,
                                                       int ntn, float inv_norm, OutMap map,
                                                       float *__restrict__ out)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    float t = 0.0f;
    for (int c = 0; c < ntn; ++c) t += partial[(size_t)r * ntn + c];
    out[map.index(r)] = canon_fitness(t * inv_norm);
}

// One instance per (precision, hidden activation): a run-time activation
// switch over the 256 accumulators would push them out of registers.
const void *const kWide[2][4] = {
    {reinterpret_cast<const void *>(&k_fit_wide32<0>), reinterpret_cast<const void *>(&k_fit_wide32<1>),
     reinterpret_cast<const void *>(&k_fit_wide32<2>), reinterpret_cast<const void *>(&k_fit_wide32<3>)},
    {reinterpret_cast<const void *>(&k_fit_wide_pipe<0>), reinterpret_cast<const void *>(&k_fit_wide_pipe<1>),
     reinterpret_cast<const void *>(&k_fit_wide_pipe<2>), reinterpret_cast<const void *>(&k_fit_wide_pipe<3>)},
};

const void *wide_kernel(const Net &net)
{
    const int act = net.act[0] >= 0 && net.act[0] <= 3 ? net.act[0] : 0;
    return kWide[net.bf16 ? 1 : 0][act];
}

// Sparks per XCD tile group.  Enough tiles for the XCD's blocks; when the
// group's rounds can be gs x (bx/gs) rectangles, the gs minimising the distinct
// weight + sample tiles per round (gs + bx/gs); gs always divides rows.
int wide_group(const Net &net, int rows, int ntn)
{
    const int bx = (net.num_cu + 7) / 8;
    int gs = 1;
    while (gs * ntn < bx && rows % (2 * gs) == 0 && gs < 64) gs *= 2;
    if (gs * ntn < bx) return gs;
    int best = gs, best_cost = gs + bx;
    for (int g = gs; g <= 16; g *= 2) {
        if (rows % g || bx % g || ntn % (bx / g)) continue;
        const int cost = g + bx / g;
        if (cost < best_cost) {
            best = g;
            best_cost = cost;
        }
    }
    // a small launch (e.g. one row per firework) gives every XCD a group while
    // the groups still hold a tile per block
    while (best > 1 && rows / best < 8 && (best / 2) * ntn >= bx) best /= 2;
    return best;
}

}  // namespace

bool wide_applicable(const Net &net)
{
    return net.nl == 2 && net.fo[0] <= WT_M && net.fo[1] <= 16;
}

// K (inputs plus the ones column) padded to the kernels' K-step rounds
int wide_kp(const Net &net)
{
    const int step = net.bf16 ? WideCfg<true>::KMULT : WideCfg<false>::KMULT;
    const int kp = (net.fi[0] + 1 + step - 1) / step * step;
    // the BF16 pipeline looks STAGES K steps ahead within a tile and the next
    const int kmin = net.bf16 ? PipeCfg::STAGES * WT_K : 0;
    return kp > kmin ? kp : kmin;
}

size_t wide_row_bytes(const Net &net)
{
    const size_t es = net.bf16 ? 2 : 4;
    const size_t b = (size_t)WT_M * wide_kp(net) * es + 16 * WT_M * es + 64;
    return (b + 255) / 256 * 256;
}

int wide_lds_bytes(const Net &net) { return net.bf16 ? PipeCfg::LDS : WideCfg<false>::LDS; }

hipError_t wide_prepare(const Net &net)
{
    return hipFuncSetAttribute(wide_kernel(net), hipFuncAttributeMaxDynamicSharedMemorySize,
                               wide_lds_bytes(net));
}

hipError_t launch_pack_wide_x(const Net &net, const float *x, char *Xw, hipStream_t st)
{
    const int Kp = wide_kp(net);
    const size_t n = (size_t)net.S_pad * Kp;
    const unsigned blocks = (unsigned)((n + TPB - 1) / TPB);
    if (net.bf16)
        hipLaunchKernelGGL(k_pack_wide_x<true>, dim3(blocks), dim3(TPB), 0, st, x, net.S, net.S_pad,
                           net.fi[0], Kp, Xw);
    else
        hipLaunchKernelGGL(k_pack_wide_x<false>, dim3(blocks), dim3(TPB), 0, st, x, net.S, net.S_pad,
                           net.fi[0], Kp, Xw);
    return hipGetLastError();
}

WidePack wide_pack_geometry(const Net &net, const DevState &d)
{
    static_assert(WT_M == 256 && WT_K == 32, "wide_pack_offset assumes 256 x 32 K blocks");
    WidePack p;
    p.Wp = d.Wpack;
    p.pr = wide_row_bytes(net);
    p.in = net.fi[0];
    p.hid = net.fo[0];
    p.out = net.fo[1];
    p.Kp = wide_kp(net);
    p.bf16 = net.bf16;
    p.woff1 = net.woff[0];
    p.boff1 = net.boff[0];
    p.woff2 = net.woff[1];
    p.boff2 = net.boff[1];
    return p;
}

hipError_t launch_fitness_wide(const Net &net, const DevState &d, const float *W, size_t ld,
                               int rows, OutMap map, float *out, hipStream_t st, hipEvent_t mid,
                               hipEvent_t pre, int prepacked)
{
    if (rows <= 0) return hipSuccess;
    const int Kp = wide_kp(net);
    const size_t pr = wide_row_bytes(net);
    hipError_t e = hipSuccess;
    const int npack = rows - prepacked;
    if (npack > 0) {
        const int es = net.bf16 ? 2 : 4, epc = 16 / es;
        const int nchunk = WT_M * Kp / epc + 16 * WT_M / epc + 4;
        const int rgroups = (npack + PACK_RPB - 1) / PACK_RPB;
        dim3 pg((nchunk + TPB * PACK_CPT - 1) / (TPB * PACK_CPT),
                rgroups < MAX_GRID_Y ? rgroups : MAX_GRID_Y);
        const float *Wsrc = W + (size_t)prepacked * ld;
        char *Wdst = d.Wpack + (size_t)prepacked * pr;
        if (net.bf16)
            hipLaunchKernelGGL(k_pack_wide_rows<true>, pg, dim3(TPB), 0, st, Wsrc, ld, npack, Wdst, pr,
                               net.fi[0], net.fo[0], net.fo[1], Kp, net.woff[0], net.boff[0],
                               net.woff[1], net.boff[1]);
        else
            hipLaunchKernelGGL(k_pack_wide_rows<false>, pg, dim3(TPB), 0, st, Wsrc, ld, npack, Wdst,
                               pr, net.fi[0], net.fo[0], net.fo[1], Kp, net.woff[0], net.boff[0],
                               net.woff[1], net.boff[1]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (pre) {                          // packing done: the GEMM kernel starts here
        e = hipEventRecord(pre, st);
        if (e != hipSuccess) return e;
    }
    WideArgs a;
    a.Wp = d.Wpack;
    a.pr = pr;
    a.rows = rows;
    a.Xw = d.Xw;
    a.Kp = Kp;
    a.nk = Kp / WT_K;
    a.S = net.S;
    a.S_pad = net.S_pad;
    a.ntn = net.S_pad / WT_N;
    a.fo1 = net.fo[1];
    a.loss = net.loss;
    a.act = net.act[0];
    a.Y = d.Ypad;
    a.lab = d.Lpad;
    a.partial = d.partial;
    a.gs = wide_group(net, rows, a.ntn);
    void *args[] = {&a};
    e = hipLaunchKernel(wide_kernel(net), dim3((unsigned)net.num_cu), dim3(TPB), args,
                        (size_t)wide_lds_bytes(net), st);
    if (e != hipSuccess) return e;
    if (mid) {
        e = hipEventRecord(mid, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_wide_finalize, dim3((rows + 255) / 256), dim3(256), 0, st, d.partial, rows,
                       a.ntn, net.inv_norm, map, out);
    return hipGetLastError();
}

}  // namespace mgfwa
