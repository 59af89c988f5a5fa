// Selection, dynamic amplitude, loser-out tournament and best-so-far (Alg. 1,
// the selection step and the loser-out step; the best-so-far row and fitness
// are the answer the algorithm returns).
//
// k_select  -- one block per population.  Per firework: Yprev <- Y; c* =
//              argmin over the lambda+G candidates (lower index on ties); move
//              when Y[c*] < Y, amplitude *amp_up, else *amp_down.  Then b = the
//              population best; every other firework that was not re-initialised
//              in the previous generation is a loser when
//              fma(-(Yprev - Y), max(T - t, 0), Y) > Y_b and restarts with A0 and
//              fitness +inf.  Decisions go to src/reinit; rows move in k_apply.
//              With BF16 fitness, c* is still taken on the BF16 values, but the
//              comparison uses c*'s FP32 fitness (k_gather_best + an FP32 fitness
//              launch), so firework and best-so-far fitness stay FP32.
// k_apply   -- grid over (firework, 4-coordinate chunk): copies the chosen
//              candidate row, or draws the restart position, and refreshes the
//              best-so-far row.
// k_gather_best -- (BF16 fitness) grid over (firework, 4-coordinate chunk):
//              c* of every firework and that candidate's row, for its FP32
//              re-evaluation before k_select compares it with the firework.
// k_finish  -- one thread: advances the generation counter, raises the stop flag.
#include "internal.h"

namespace mgfwa {

namespace {

constexpr int TPB = 256;
constexpr int MAX_GRID_Y = 65535;
constexpr int SRC_NONE = -1;

// Lowest candidate fitness of one firework and its index (lower index on ties),
// over one wavefront: lanes scan strided candidates, then a (value, index)
// butterfly; every lane returns the result.
__device__ __forceinline__ void best_candidate(const float *yc, int C, int lane, float *ymin_out,
                                               int *cs_out)
{
    float ymin = __int_as_float(0x7f800000);
    int cs = 0x7fffffff;
    for (int c = lane; c < C; c += 64) {
        const float v = yc[c];
        if (v < ymin || (v == ymin && c < cs)) {
            ymin = v;
            cs = c;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(ymin, off);
        const int oc = __shfl_xor(cs, off);
        if (ov < ymin || (ov == ymin && oc < cs)) {
            ymin = ov;
            cs = oc;
        }
    }
    *ymin_out = ymin;
    *cs_out = cs;
}

__device__ void population_best(const float *Y, int N, int *fb_out, float *yb_out)
{
    // lowest fitness, lower index on ties; N is small, one thread scans in order
    int fb = 0;
    float yb = Y[0];
    for (int f = 1; f < N; ++f)
        if (Y[f] < yb) {
            yb = Y[f];
            fb = f;
        }
    *fb_out = fb;
    *yb_out = yb;
}

__device__ __forceinline__ void select_body(const Shape &s, const DevState &d, bool checked,
                                            Blk blk)
{
    float *__restrict__ Yc = d.Yc;
    float *__restrict__ Y = d.Y;
    float *__restrict__ Yprev = d.Yprev;
    float *__restrict__ A = d.A;
    float *__restrict__ Aexp = d.Aexp;
    int32_t *__restrict__ fresh = d.fresh;
    int32_t *__restrict__ cstar = d.cstar;
    int32_t *__restrict__ improved = d.improved;
    int32_t *__restrict__ reinit = d.reinit;
    int32_t *__restrict__ src = d.src;
    float *__restrict__ best_y = d.best_y;
    int32_t *__restrict__ best_f = d.best_f;
    int32_t *__restrict__ best_gen = d.best_gen;
    int32_t *__restrict__ best_upd = d.best_upd;
    const float *__restrict__ ystar = checked ? d.Ystar : nullptr;
    int32_t *__restrict__ ctrl = d.ctrl;
    if (ctrl[CTRL_DONE]) return;
    const int t = ctrl[CTRL_GEN] + 1;
    const int b = blk.x, N = s.N;
    __shared__ int s_fb;
    __shared__ float s_yb;
    // one wavefront per firework: c* and its fitness (with ystar, both come from
    // the gather step: c* by the BF16 fitness, its value re-evaluated in FP32)
    const int lane = threadIdx.x & 63, nwave = blockDim.x >> 6;
    for (int f = threadIdx.x >> 6; f < N; f += nwave) {
        const int gf = b * N + f;
        float ymin;
        int cs;
        if (ystar) {
            ymin = ystar[gf];
            cs = cstar[gf];
        } else {
            best_candidate(Yc + (size_t)gf * s.C, s.C, lane, &ymin, &cs);
        }
        if (lane == 0) {
            const float yold = Y[gf];
            Yprev[gf] = yold;
            Aexp[gf] = A[gf];   // the amplitude this generation's sparks were drawn with
            cstar[gf] = cs;
            reinit[gf] = 0;
            if (ymin < yold) {
                Y[gf] = ymin;
                A[gf] = A[gf] * s.amp_up;
                improved[gf] = 1;
                src[gf] = cs;
            } else {
                A[gf] = A[gf] * s.amp_down;
                improved[gf] = 0;
                src[gf] = SRC_NONE;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) population_best(Y + (size_t)b * N, N, &s_fb, &s_yb);
    __syncthreads();
    const int fb = s_fb;
    const float yb = s_yb;
    const float remaining = (float)(t < s.T ? s.T - t : 0);
    for (int f = threadIdx.x; f < N; f += blockDim.x) {
        const int gf = b * N + f;
        const int was_fresh = fresh[gf];
        fresh[gf] = 0;
        if (!s.loser_out || f == fb || was_fresh) continue;
        const float improvement = Yprev[gf] - Y[gf];
        const float predicted = __builtin_fmaf(-improvement, remaining, Y[gf]);
        if (predicted > yb) {
            reinit[gf] = 1;
            src[gf] = SRC_NONE;
            A[gf] = s.amp0;
            Y[gf] = __int_as_float(0x7f800000);
            fresh[gf] = 1;
        }
    }
    if (threadIdx.x == 0) {
        const int upd = yb < best_y[b];
        best_upd[b] = upd;
        if (upd) {
            best_y[b] = yb;
            best_f[b] = fb;
            best_gen[b] = t;
        }
        if (s.use_target && best_y[b] <= s.target) atomicOr(&ctrl[CTRL_DONE_PENDING], 1);
    }
}

__global__ __launch_bounds__(TPB) void k_select(Shape s, DevState d, int checked)
{
    select_body(s, d, checked != 0, own_block());
}

// After the initial fitness: Yprev = Y, best-so-far = population best at generation 0.
__global__ __launch_bounds__(TPB) void k_init_select(Shape s, const float *__restrict__ Y,
                                                     float *__restrict__ Yprev,
                                                     int32_t *__restrict__ fresh,
                                                     int32_t *__restrict__ reinit,
                                                     int32_t *__restrict__ src,
                                                     float *__restrict__ best_y,
                                                     int32_t *__restrict__ best_f,
                                                     int32_t *__restrict__ best_gen,
                                                     int32_t *__restrict__ best_upd,
                                                     int32_t *__restrict__ ctrl)
{
    const int b = blockIdx.x, N = s.N;
    for (int f = threadIdx.x; f < N; f += blockDim.x) {
        const int gf = b * N + f;
        Yprev[gf] = Y[gf];
        fresh[gf] = 0;
        reinit[gf] = 0;
        src[gf] = SRC_NONE;
    }
    if (threadIdx.x == 0) {
        int fb;
        float yb;
        population_best(Y + (size_t)b * N, N, &fb, &yb);
        best_y[b] = yb;
        best_f[b] = fb;
        best_gen[b] = 0;
        best_upd[b] = 1;
        if (s.use_target && yb <= s.target) atomicOr(&ctrl[CTRL_DONE_PENDING], 1);
    }
}

// With s.regen a winning explosion spark is regenerated from the firework's
// row (still the generation's, read before it is overwritten), its explosion
// amplitude and the population range, exactly as the explosion drew it.  With
// wstar the winner is the row k_gather_best stored there.
__device__ __forceinline__ void apply_body(const Shape &s, const DevState &d, bool checked, Blk blk)
{
    float *__restrict__ F = d.F;
    const float *__restrict__ SE = d.SE;
    const float *__restrict__ SG = d.SG;
    const float *__restrict__ Aexp = d.Aexp;
    const float *__restrict__ lo = s.map_range ? d.lo : nullptr;
    const float *__restrict__ hi = s.map_range ? d.hi : nullptr;
    const int32_t *__restrict__ src = d.src;
    const int32_t *__restrict__ reinit = d.reinit;
    const int32_t *__restrict__ best_f = d.best_f;
    const int32_t *__restrict__ best_upd = d.best_upd;
    float *__restrict__ best_x = d.best_x;
    const float *__restrict__ wstar = checked ? d.Wstar : nullptr;
    const int32_t *__restrict__ ctrl = d.ctrl;
    if (ctrl[CTRL_DONE]) return;
    const uint32_t t = (uint32_t)ctrl[CTRL_GEN] + 1u;
    const int chunk = blk.x * TPB + threadIdx.x;
    if (chunk >= (s.Dp >> 2)) return;
    for (int gf = blk.y; gf < s.BN; gf += blk.gy) {
        const int b = gf / s.N, f = gf % s.N;
        const int sr = src[gf], ri = reinit[gf];
        const bool copy_best = best_upd[b] && best_f[b] == f;
        if (!ri && sr < 0 && !copy_best) continue;
        float4 *frow = reinterpret_cast<float4 *>(F + (size_t)gf * s.Dp);
        float4 v;
        if (ri) {
            const uint4 r = draw4(s.key, (uint32_t)chunk, (uint32_t)gf, t, TAG_REINIT);
            const uint32_t w[4] = {r.x, r.y, r.z, r.w};
            float e4[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                e4[e] = box_uniform(s.box, u01(w[e]));
                if (4 * chunk + e >= s.D) e4[e] = 0.0f;
            }
            v = make_float4(e4[0], e4[1], e4[2], e4[3]);
            frow[chunk] = v;
        } else if (sr >= 0 && wstar) {
            // the gathered candidate row (the one its FP32 fitness was taken of)
            v = reinterpret_cast<const float4 *>(wstar + (size_t)gf * s.Dp)[chunk];
            frow[chunk] = v;
        } else if (sr >= 0 && sr < s.lam && s.regen) {
            const float4 x4 = frow[chunk];
            const float x[4] = {x4.x, x4.y, x4.z, x4.w};
            const size_t pb = (size_t)b * s.Dp;
            float e4[4];
            explosion_chunk(x, Aexp[gf], s.key, chunk, (uint32_t)(gf * s.lam + sr), t, s.box,
                            lo ? lo + pb : nullptr, hi ? hi + pb : nullptr, s.D, e4);
            v = make_float4(e4[0], e4[1], e4[2], e4[3]);
            frow[chunk] = v;
        } else if (sr >= 0) {
            const float *row = sr < s.lam ? SE + ((size_t)gf * s.lam + sr) * s.Dp
                                          : SG + ((size_t)gf * s.G + (sr - s.lam)) * s.Dp;
            v = reinterpret_cast<const float4 *>(row)[chunk];
            frow[chunk] = v;
        } else {
            v = frow[chunk];
        }
        if (copy_best) reinterpret_cast<float4 *>(best_x + (size_t)b * s.Dp)[chunk] = v;
    }
}

__global__ __launch_bounds__(TPB) void k_apply(Shape s, DevState d, int checked)
{
    apply_body(s, d, checked != 0, own_block());
}

// c* of firework blk.y (every block recomputes it: C values, one
// wavefront) and coordinates 4*chunk.. of its row: an explosion spark
// (regenerated from the firework's row and amplitude when s.regen, as the
// explosion drew it) or a guiding spark.  Runs before k_select, so F and A
// still hold the generation's values.
__device__ __forceinline__ void gather_best_body(const Shape &s, const DevState &d, Blk blk)
{
    const float *__restrict__ Yc = d.Yc;
    const float *__restrict__ F = d.F;
    const float *__restrict__ A = d.A;
    const float *__restrict__ lo = s.map_range ? d.lo : nullptr;
    const float *__restrict__ hi = s.map_range ? d.hi : nullptr;
    if (d.ctrl[CTRL_DONE]) return;
    const uint32_t t = (uint32_t)d.ctrl[CTRL_GEN] + 1u;
    __shared__ int s_cs;
    const int nchunk = s.Dp >> 2;
    for (int gf = blk.y; gf < s.BN; gf += blk.gy) {
        if (threadIdx.x < 64) {
            float ymin;
            int cs;
            best_candidate(Yc + (size_t)gf * s.C, s.C, threadIdx.x, &ymin, &cs);
            if (threadIdx.x == 0) {
                s_cs = cs;
                if (blk.x == 0) d.cstar[gf] = cs;
            }
        }
        __syncthreads();
        const int cs = s_cs;
        __syncthreads();   // s_cs is rewritten for the next firework
        const int chunk = blk.x * TPB + threadIdx.x;
        if (chunk >= nchunk) continue;
        float4 v;
        if (cs < s.lam && s.regen) {
            const float4 x4 = reinterpret_cast<const float4 *>(F + (size_t)gf * s.Dp)[chunk];
            const float x[4] = {x4.x, x4.y, x4.z, x4.w};
            const size_t pb = (size_t)(gf / s.N) * s.Dp;
            float e4[4];
            explosion_chunk(x, A[gf], s.key, chunk, (uint32_t)(gf * s.lam + cs), t, s.box,
                            lo ? lo + pb : nullptr, hi ? hi + pb : nullptr, s.D, e4);
            v = make_float4(e4[0], e4[1], e4[2], e4[3]);
        } else {
            const float *row = cs < s.lam ? d.SE + ((size_t)gf * s.lam + cs) * s.Dp
                                          : d.SG + ((size_t)gf * s.G + (cs - s.lam)) * s.Dp;
            v = reinterpret_cast<const float4 *>(row)[chunk];
        }
        reinterpret_cast<float4 *>(d.Wstar + (size_t)gf * s.Dp)[chunk] = v;
    }
}

__global__ __launch_bounds__(TPB) void k_gather_best(Shape s, DevState d)
{
    gather_best_body(s, d, own_block());
}

__global__ void k_clear_ctrl(int32_t *ctrl)
{
    if (threadIdx.x < CTRL_WORDS) ctrl[threadIdx.x] = 0;
}

__device__ __forceinline__ void finish_body(int32_t *ctrl, int advance)
{
    if (threadIdx.x != 0) return;
    if (ctrl[CTRL_DONE]) return;
    if (advance) ctrl[CTRL_GEN] = ctrl[CTRL_GEN] + 1;
    if (ctrl[CTRL_DONE_PENDING]) ctrl[CTRL_DONE] = 1;
}

__global__ void k_finish(int32_t *ctrl, int advance)
{
    if (blockIdx.x != 0) return;
    finish_body(ctrl, advance);
}

// ---- grouped launches: the same bodies over many jobs (one grid) ----
__global__ __launch_bounds__(TPB) void k_select_group(GroupTable t)
{
    const int j = group_job(t, blockIdx.x);
    Blk gb;
    if (!group_block(t, j, blockIdx.x, &gb)) return;   // padding
    // private copies: read through a pointer into global memory, the
    // arguments would be reloaded after every store the body makes
    const Shape js = t.job[j]->s;
    const DevState jd = t.job[j]->d;
    select_body(js, jd, js.recheck != 0, gb);
}

__global__ __launch_bounds__(TPB) void k_apply_group(GroupTable t)
{
    const int j = group_job(t, blockIdx.x);
    Blk gb;
    if (!group_block(t, j, blockIdx.x, &gb)) return;   // padding
    // private copies: read through a pointer into global memory, the
    // arguments would be reloaded after every store the body makes
    const Shape js = t.job[j]->s;
    const DevState jd = t.job[j]->d;
    apply_body(js, jd, js.recheck != 0, gb);
}

__global__ __launch_bounds__(TPB) void k_gather_best_group(GroupTable t)
{
    const int j = group_job(t, blockIdx.x);
    Blk gb;
    if (!group_block(t, j, blockIdx.x, &gb)) return;   // padding
    // private copies: read through a pointer into global memory, the
    // arguments would be reloaded after every store the body makes
    const Shape js = t.job[j]->s;
    const DevState jd = t.job[j]->d;
    gather_best_body(js, jd, gb);
}

// one block per job (the solo launch has one block)
__global__ void k_finish_group(GroupTable t)
{
    const int j = group_job(t, blockIdx.x);
    Blk gb;
    if (!group_block(t, j, blockIdx.x, &gb)) return;   // padding
    finish_body(t.job[j]->d.ctrl, 1);
}

__global__ __launch_bounds__(TPB) void k_store_fitness(const float *__restrict__ in, int rows,
                                                       OutMap map, float *__restrict__ out,
                                                       const int32_t *__restrict__ ctrl)
{
    if (ctrl && ctrl[CTRL_DONE]) return;
    const int r = blockIdx.x * TPB + threadIdx.x;
    if (r >= rows) return;
    out[map.index(r)] = canon_fitness(in[r]);
}

}  // namespace

dim3 select_grid(const Shape &s) { return dim3(s.B); }

// grid over (4-coordinate chunk, firework): apply and gather
dim3 firework_row_grid(const Shape &s)
{
    const int nchunk = s.Dp >> 2;
    return dim3((nchunk + TPB - 1) / TPB, s.BN < MAX_GRID_Y ? s.BN : MAX_GRID_Y);
}

hipError_t launch_select(const Shape &s, const DevState &d, hipStream_t st, bool checked)
{
    hipLaunchKernelGGL(k_select, select_grid(s), dim3(TPB), 0, st, s, d, checked ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_gather_best(const Shape &s, const DevState &d, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_best, firework_row_grid(s), dim3(TPB), 0, st, s, d);
    return hipGetLastError();
}

hipError_t launch_select_group(const GroupTable &t, hipStream_t st)
{
    hipLaunchKernelGGL(k_select_group, dim3(t.start[t.njobs]), dim3(TPB), 0, st, t);
    return hipGetLastError();
}

hipError_t launch_apply_group(const GroupTable &t, hipStream_t st)
{
    hipLaunchKernelGGL(k_apply_group, dim3(t.start[t.njobs]), dim3(TPB), 0, st, t);
    return hipGetLastError();
}

hipError_t launch_gather_best_group(const GroupTable &t, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_best_group, dim3(t.start[t.njobs]), dim3(TPB), 0, st, t);
    return hipGetLastError();
}

hipError_t launch_finish_group(const GroupTable &t, hipStream_t st)
{
    hipLaunchKernelGGL(k_finish_group, dim3(t.start[t.njobs]), dim3(64), 0, st, t);
    return hipGetLastError();
}

hipError_t launch_init_select(const Shape &s, const DevState &d, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_select, dim3(s.B), dim3(TPB), 0, st, s, d.Y, d.Yprev, d.fresh,
                       d.reinit, d.src, d.best_y, d.best_f, d.best_gen, d.best_upd, d.ctrl);
    return hipGetLastError();
}

hipError_t launch_apply(const Shape &s, const DevState &d, hipStream_t st, bool checked)
{
    hipLaunchKernelGGL(k_apply, firework_row_grid(s), dim3(TPB), 0, st, s, d, checked ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_clear_ctrl(int32_t *ctrl, hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_ctrl, dim3(1), dim3(64), 0, st, ctrl);
    return hipGetLastError();
}

hipError_t launch_finish(const DevState &d, int advance, hipStream_t st)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, d.ctrl, advance);
    return hipGetLastError();
}

hipError_t launch_store_fitness(const float *src, int rows, OutMap map, float *out,
                                const int32_t *ctrl, hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_store_fitness, dim3((rows + TPB - 1) / TPB), dim3(TPB), 0, st, src, rows,
                       map, out, ctrl);
    return hipGetLastError();
}

}  // namespace mgfwa
