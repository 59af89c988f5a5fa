// Multi-guiding sparks (Alg. 1, the guiding-spark step and the mapping step
// that follows it).
//
// Ranking: the members of every guiding group ordered by (fitness key, spark
//            index) give the top-k and bottom-k member lists in ascending spark
//            index and the all-tie flag.  Groups of up to 64 members are ranked
//            inside k_guide by one wavefront, one lane per member (keys
//            broadcast by lane shuffles, list positions from ballots); larger
//            groups by k_rank, one block per firework over LDS.
// k_guide -- grid over (group, 4-coordinate chunk): the guiding vector is
//            (sum of top sparks - sum of bottom sparks) * (1/k), each sum taken
//            in ascending spark index (zero when the group ties); the guiding
//            spark x + boost*delta is mapped back into the box like an
//            explosion spark.  HBM-bound: it streams 2k spark rows per group.
#include "internal.h"

namespace mgfwa {

namespace {

constexpr int TPB = 256;
constexpr int MAX_GRID_Y = 65535;

__device__ __forceinline__ void rank_body(const float *__restrict__ Yc, int C, int lam, int G, int m,
                                          int k, int32_t *__restrict__ top,
                                          int32_t *__restrict__ bottom, int32_t *__restrict__ tie,
                                          const int32_t *__restrict__ ctrl, int lag, uint32_t *sh,
                                          Blk b)
{
    if (ctrl[CTRL_DONE]) return;
    if (lag && ctrl[CTRL_GEN] == 0) {
        // lagged guiding before any explosion: every guiding vector is zero
        const int gf = b.x;
        for (int i = threadIdx.x; i < G * k; i += blockDim.x) {
            const int g = i / k, j = i % k;
            top[((size_t)gf * G + g) * k + j] = g * m + j;
            bottom[((size_t)gf * G + g) * k + j] = g * m + m - k + j;
        }
        for (int g = threadIdx.x; g < G; g += blockDim.x) tie[(size_t)gf * G + g] = 1;
        return;
    }
    uint32_t *key = sh;               // [lam]
    int32_t *rank = (int32_t *)(sh + lam);  // [lam]
    const int gf = b.x;
    for (int j = threadIdx.x; j < lam; j += blockDim.x) key[j] = fit_key(Yc[(size_t)gf * C + j]);
    __syncthreads();
    for (int j = threadIdx.x; j < lam; j += blockDim.x) {
        const int j0 = (j / m) * m;
        const uint32_t kj = key[j];
        int r = 0;
        for (int i = j0; i < j0 + m; ++i) {
            const uint32_t ki = key[i];
            r += (ki < kj) || (ki == kj && i < j);
        }
        rank[j] = r;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < lam; j += blockDim.x) {
        const int g = j / m, j0 = g * m, rj = rank[j];
        const size_t base = ((size_t)gf * G + g) * k;
        if (rj < k) {
            int pos = 0;
            for (int i = j0; i < j; ++i) pos += rank[i] < k;
            top[base + pos] = j;
        }
        if (rj >= m - k) {
            int pos = 0;
            for (int i = j0; i < j; ++i) pos += rank[i] >= m - k;
            bottom[base + pos] = j;
        }
        if (rj == 0) {
            // the group ties iff its first and last ranked members share a key
            uint32_t kmax = 0;
            for (int i = j0; i < j0 + m; ++i)
                if (rank[i] == m - 1) kmax = key[i];
            tie[(size_t)gf * G + g] = (key[j] == kmax);
        }
    }
}

__global__ __launch_bounds__(TPB) void k_rank(const float *__restrict__ Yc, int C, int lam, int G,
                                              int m, int k, int32_t *__restrict__ top,
                                              int32_t *__restrict__ bottom,
                                              int32_t *__restrict__ tie,
                                              const int32_t *__restrict__ ctrl, int lag)
{
    extern __shared__ uint32_t sh[];
    rank_body(Yc, C, lam, G, m, k, top, bottom, tie, ctrl, lag, sh, own_block());
}

__global__ __launch_bounds__(TPB) void k_rank_group(GroupTable t)
{
    extern __shared__ uint32_t sh[];
    const int j = group_job(t, blockIdx.x);
    Blk gb;
    if (!group_block(t, j, blockIdx.x, &gb)) return;   // padding
    // private copies: read through a pointer into global memory, the
    // arguments would be reloaded after every store the body makes
    const Shape js = t.job[j]->s;
    const DevState jd = t.job[j]->d;
    const Shape &s = js;
    rank_body(jd.Yc, s.C, s.lam, s.G, s.m, s.k, jd.top, jd.bottom, jd.tie, jd.ctrl, s.lag, sh,
              gb);
}

// Groups of m <= 64 members: the calling wavefront ranks group gi (g = gi % G
// of firework gi / G), one lane per member, and writes its top-k and bottom-k
// lists (spark indices within the firework, ascending) and tie flag through
// the given pointers (LDS, and global memory when g_top is non-null).
__device__ __forceinline__ void rank_group_wave(const float *__restrict__ Yc, int C, int G, int m,
                                                int k, int gi, bool zero_guide, int32_t *l_top,
                                                int32_t *l_bottom, int32_t *l_tie, int32_t *g_top,
                                                int32_t *g_bottom, int32_t *g_tie)
{
    const int lane = threadIdx.x & 63;
    const int gf = gi / G, g = gi % G;
    const size_t base = (size_t)gi * k;
    if (zero_guide) {
        // lagged guiding before any explosion: every guiding vector is zero
        if (lane < k) {
            l_top[lane] = g * m + lane;
            l_bottom[lane] = g * m + m - k + lane;
            if (g_top) {
                g_top[base + lane] = g * m + lane;
                g_bottom[base + lane] = g * m + m - k + lane;
            }
        }
        if (lane == 0) {
            *l_tie = 1;
            if (g_tie) g_tie[gi] = 1;
        }
        return;
    }
    const bool in = lane < m;
    const uint32_t kj = in ? fit_key(Yc[(size_t)gf * C + g * m + lane]) : 0xffffffffu;
    int r = 0;
    for (int i = 0; i < m; ++i) {
        const uint32_t ki = (uint32_t)__shfl((int)kj, i);
        r += (ki < kj) || (ki == kj && i < lane);
    }
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const bool is_top = in && r < k, is_bottom = in && r >= m - k;
    const uint64_t tmask = __ballot(is_top), bmask = __ballot(is_bottom);
    if (is_top) {
        const int pos = __popcll(tmask & below);
        l_top[pos] = g * m + lane;
        if (g_top) g_top[base + pos] = g * m + lane;
    }
    if (is_bottom) {
        const int pos = __popcll(bmask & below);
        l_bottom[pos] = g * m + lane;
        if (g_bottom) g_bottom[base + pos] = g * m + lane;
    }
    // the group ties iff its first and last ranked members share a key, i.e.
    // iff its smallest and largest keys are equal
    uint32_t lo = in ? kj : 0xffffffffu, hi = in ? kj : 0u;
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t l2 = (uint32_t)__shfl_xor((int)lo, off), h2 = (uint32_t)__shfl_xor((int)hi, off);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
    }
    if (lane == 0) {
        *l_tie = lo == hi;
        if (g_tie) g_tie[gi] = lo == hi;
    }
}

// RANK: groups of m <= 64 members are ranked inside the kernel (wavefront 0 of
// each block, into LDS; the x-block 0 also stores the lists); otherwise the
// lists come from k_rank.  REGEN: the member sparks are regenerated from the
// counter-based generator (firework row, amplitude A) instead of read from SE.
template <bool RANK, bool REGEN>
__device__ __forceinline__ void guide_body(const float *__restrict__ F, const float *__restrict__ A,
                                           const float *__restrict__ SE, float *__restrict__ SG,
                                           int32_t *__restrict__ top, int32_t *__restrict__ bottom,
                                           int32_t *__restrict__ tie, int G, int lam, int k,
                                           float inv_k, float boost, int groups, int D, int Dp,
                                           uint2 key, Box box, const int32_t *__restrict__ ctrl,
                                           int N, const float *__restrict__ lo,
                                           const float *__restrict__ hi,
                                           const float *__restrict__ Yc, int C, int m, int lag,
                                           Blk b)
{
    __shared__ int32_t s_top[64], s_bottom[64], s_tie;
    if (ctrl[CTRL_DONE]) return;
    const uint32_t tn = (uint32_t)ctrl[CTRL_GEN] + 1u;
    const int chunk = b.x * TPB + threadIdx.x;
    const bool active = chunk < (Dp >> 2);
    const bool zero_guide = lag && ctrl[CTRL_GEN] == 0;
    for (int gi = b.y; gi < groups; gi += b.gy) {
        const int32_t *tp, *bp;
        int tied;
        if constexpr (RANK) {
            if (threadIdx.x < 64) {
                const bool store = b.x == 0;
                rank_group_wave(Yc, C, G, m, k, gi, zero_guide, s_top, s_bottom, &s_tie,
                                store ? top : nullptr, store ? bottom : nullptr,
                                store ? tie : nullptr);
            }
            __syncthreads();
            tp = s_top;
            bp = s_bottom;
            tied = s_tie;
        } else {
            tp = top + (size_t)gi * k;
            bp = bottom + (size_t)gi * k;
            tied = tie[gi];
        }
        if (!active) {
            if constexpr (RANK) __syncthreads();   // the lists are read before the next group
            continue;
        }
        const int gf = gi / G;
        const float4 x4 = reinterpret_cast<const float4 *>(F + (size_t)gf * Dp)[chunk];
        const float x[4] = {x4.x, x4.y, x4.z, x4.w};
        const size_t pb = (size_t)(gf / N) * Dp;
        const float *plo = lo ? lo + pb : nullptr, *phi = hi ? hi + pb : nullptr;
        float dlt[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (!tied) {
            float st[4] = {0.0f, 0.0f, 0.0f, 0.0f}, sb[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if constexpr (REGEN) {
                const float amp = A[gf];
                const uint32_t row0 = (uint32_t)gf * (uint32_t)lam;
                for (int i = 0; i < k; ++i) {
                    float a[4], b[4];
                    explosion_chunk(x, amp, key, chunk, row0 + (uint32_t)tp[i], tn, box, plo, phi,
                                    D, a);
                    explosion_chunk(x, amp, key, chunk, row0 + (uint32_t)bp[i], tn, box, plo, phi,
                                    D, b);
                    st[0] = st[0] + a[0]; st[1] = st[1] + a[1]; st[2] = st[2] + a[2]; st[3] = st[3] + a[3];
                    sb[0] = sb[0] + b[0]; sb[1] = sb[1] + b[1]; sb[2] = sb[2] + b[2]; sb[3] = sb[3] + b[3];
                }
            } else {
                const float *base = SE + (size_t)gf * lam * Dp;
                for (int i = 0; i < k; ++i) {
                    const float4 a = reinterpret_cast<const float4 *>(base + (size_t)tp[i] * Dp)[chunk];
                    const float4 b = reinterpret_cast<const float4 *>(base + (size_t)bp[i] * Dp)[chunk];
                    st[0] = st[0] + a.x; st[1] = st[1] + a.y; st[2] = st[2] + a.z; st[3] = st[3] + a.w;
                    sb[0] = sb[0] + b.x; sb[1] = sb[1] + b.y; sb[2] = sb[2] + b.z; sb[3] = sb[3] + b.w;
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) dlt[e] = (st[e] - sb[e]) * inv_k;
        }
        float v[4];
        bool any_out = false;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[e] = boost == 1.0f ? x[e] + dlt[e] : __builtin_fmaf(boost, dlt[e], x[e]);
            any_out |= outside(box, v[e]);
        }
        if (any_out) {
            const uint4 r2 = draw4(key, (uint32_t)chunk, (uint32_t)gi, tn, TAG_GUIDE_MAP);
            const uint32_t w2[4] = {r2.x, r2.y, r2.z, r2.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (outside(box, v[e])) v[e] = map_uniform(box, u01(w2[e]), plo, phi, 4 * chunk + e);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (4 * chunk + e >= D) v[e] = 0.0f;
        reinterpret_cast<float4 *>(SG + (size_t)gi * Dp)[chunk] = make_float4(v[0], v[1], v[2], v[3]);
        if constexpr (RANK) __syncthreads();   // the lists are read before the next group
    }
}

template <bool RANK, bool REGEN>
__device__ __forceinline__ void guide_job(const Shape &s, const DevState &d, Blk b)
{
    guide_body<RANK, REGEN>(d.F, d.A, d.SE, d.SG, d.top, d.bottom, d.tie, s.G, s.lam, s.k, s.inv_k,
                            s.boost, s.BN * s.G, s.D, s.Dp, s.key, s.box, d.ctrl, s.N,
                            s.map_range ? d.lo : nullptr, s.map_range ? d.hi : nullptr, d.Yc, s.C,
                            s.m, s.lag, b);
}

template <bool RANK, bool REGEN>
__global__ __launch_bounds__(TPB) void k_guide(Shape s, DevState d)
{
    guide_job<RANK, REGEN>(s, d, own_block());
}

// The guiding step of many jobs; each job takes its own variant (in-kernel
// ranking for groups of <= 64 members, regenerated member sparks).
__global__ __launch_bounds__(TPB) void k_guide_group(GroupTable t)
{
    const int j = group_job(t, blockIdx.x);
    Blk gb;
    if (!group_block(t, j, blockIdx.x, &gb)) return;   // padding
    // private copies: read through a pointer into global memory, the
    // arguments would be reloaded after every store the body makes
    const Shape js = t.job[j]->s;
    const DevState jd = t.job[j]->d;
    const Blk b = gb;
    if (js.m <= 64) {
        if (js.regen) guide_job<true, true>(js, jd, b);
        else guide_job<true, false>(js, jd, b);
    } else {
        if (js.regen) guide_job<false, true>(js, jd, b);
        else guide_job<false, false>(js, jd, b);
    }
}

}  // namespace

dim3 rank_grid(const Shape &s) { return dim3(s.BN); }

dim3 guide_grid(const Shape &s)
{
    const int groups = s.BN * s.G;
    const int nchunk = s.Dp >> 2;
    return dim3((nchunk + TPB - 1) / TPB, groups < MAX_GRID_Y ? groups : MAX_GRID_Y);
}

hipError_t launch_rank(const Shape &s, const DevState &d, hipStream_t st)
{
    if (s.m <= 64) return hipSuccess;   // ranked inside k_guide
    const size_t shmem = (size_t)s.lam * 8;
    hipLaunchKernelGGL(k_rank, rank_grid(s), dim3(TPB), shmem, st, d.Yc, s.C, s.lam, s.G, s.m, s.k,
                       d.top, d.bottom, d.tie, d.ctrl, s.lag);
    return hipGetLastError();
}

hipError_t launch_rank_group(const GroupTable &t, int max_lam, hipStream_t st)
{
    hipLaunchKernelGGL(k_rank_group, dim3(t.start[t.njobs]), dim3(TPB), (size_t)max_lam * 8, st, t);
    return hipGetLastError();
}

hipError_t launch_guide(const Shape &s, const DevState &d, hipStream_t st)
{
    auto *k = s.m <= 64 ? (s.regen ? &k_guide<true, true> : &k_guide<true, false>)
                        : (s.regen ? &k_guide<false, true> : &k_guide<false, false>);
    hipLaunchKernelGGL(k, guide_grid(s), dim3(TPB), 0, st, s, d);
    return hipGetLastError();
}

hipError_t launch_guide_group(const GroupTable &t, hipStream_t st)
{
    hipLaunchKernelGGL(k_guide_group, dim3(t.start[t.njobs]), dim3(TPB), 0, st, t);
    return hipGetLastError();
}

}  // namespace mgfwa
