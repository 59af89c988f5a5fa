// Fitness host side: kernel table, plan selection and launches, plus the
// partial-sum finalisation and the packing of the problem data.  The kernel
// template lives in fit_kernel.h; the fit_*.hip files instantiate it.
#include "fit_kernel.h"

#include <cstdlib>

namespace mgfwa {

namespace fit {
// one table per instantiation file
const KernelEntry *table_std(int *n);
const KernelEntry *table_l1(int *n);
const KernelEntry *table_l2(int *n);
const KernelEntry *table_l2_wide(int *n);
const KernelEntry *table_l3(int *n);
const KernelEntry *table_l3_wide_f32(int *n);
const KernelEntry *table_l3_wide_bf16(int *n);
const KernelEntry *table_l4_f32(int *n);
const KernelEntry *table_l4_bf16(int *n);
const KernelEntry *table_l4_wide_f32(int *n);
const KernelEntry *table_l4_wide_bf16(int *n);
const KernelEntry *table_lds_bf16(int *n);
const KernelEntry *table_lds_f32(int *n);
}  // namespace fit

namespace {

using namespace fit;

constexpr int MAX_BPR = 64;

// Sum of a row's partials in order, scaled to the mean, NaN -> +inf, scattered.
__device__ __forceinline__ void finalize_body(const float *__restrict__ partial, int rows, int bpr,
                                              float inv_norm, const OutMap &map,
                                              float *__restrict__ out, Blk b)
{
    const int r = b.x * 256 + threadIdx.x;
    if (r >= rows) return;
    float t = 0.0f;
    for (int c = 0; c < bpr; ++c) t += partial[(size_t)r * bpr + c];
    out[map.index(r)] = canon_fitness(t * inv_norm);
}

__global__ __launch_bounds__(256) void k_fit_finalize(const float *__restrict__ partial, int rows,
                                                      int bpr, float inv_norm, OutMap map,
                                                      float *__restrict__ out)
{
    finalize_body(partial, rows, bpr, inv_norm, map, out, own_block());
}

__global__ __launch_bounds__(256) void k_fit_finalize_group(GroupTable t, int which)
{
    const int j = group_job(t, blockIdx.x);
    Blk gb;
    if (!group_block(t, j, blockIdx.x, &gb)) return;   // padding
    const FitLaunch f = t.job[j]->fit[which];
    finalize_body(f.a.partial, f.a.rows, f.a.bpr, f.inv_norm, f.map, f.out,
                  gb);
}

// Pack the problem data: X zero-padded to [S_pad][in_pad] (FP32 or bf16 RNE;
// skipped when both X destinations are null), MSE targets to [S_pad][out],
// labels to [S_pad] (-1 on padding).
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ x, const float *__restrict__ y,
                                              const int32_t *__restrict__ lab, int S, int S_pad,
                                              int in, int in_pad, int out, int bf16,
                                              float *__restrict__ Xp, uint16_t *__restrict__ Xb,
                                              float *__restrict__ Yp, int32_t *__restrict__ Lp)
{
    const size_t tid = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t nx = (size_t)S_pad * in_pad;
    if (tid < nx && (Xb || Xp)) {   // (the wide kernel packs its samples itself)
        const int s = (int)(tid / in_pad), k = (int)(tid % in_pad);
        const float v = (s < S && k < in) ? x[(size_t)s * in + k] : 0.0f;
        if (bf16) Xb[tid] = __builtin_bit_cast(uint16_t, (__bf16)v);
        else Xp[tid] = v;
    }
    if (tid < (size_t)S_pad * out && Yp) {
        const int s = (int)(tid / out);
        Yp[tid] = (s < S && y) ? y[tid] : 0.0f;
    }
    if (tid < (size_t)S_pad && Lp) Lp[tid] = (tid < (size_t)S && lab) ? lab[tid] : -1;
}

const KernelEntry *(*const kTables[])(int *) = {
    table_std,         table_l1,          table_l2,       table_l2_wide,     table_l3,
    table_l3_wide_f32, table_l3_wide_bf16, table_l4_f32,  table_l4_bf16,     table_l4_wide_f32,
    table_l4_wide_bf16, table_lds_bf16, table_lds_f32,
};

}  // namespace

int fit_max_bpr() { return MAX_BPR; }

// LDS layout of the staged weights for kernel entry e; returns the byte size.
static int lds_layout(const Net &net, const KernelEntry &e, FitPlan *p)
{
    const int es = e.bf16 ? 2 : 4;          // storage bytes per weight
    // pitch padding in elements: BF16 16 bytes; FP32 32 bytes (a pitch of 2 mod 8
    // 16-byte chunks, with the row-parity chunk swizzle of the kernel)
    const int unit = 8;
    int off = 0, boff = 0;
    for (int l = 0; l < MAXL; ++l) {
        p->lw[l] = p->lpitch[l] = p->lrows[l] = p->lcols[l] = p->lb[l] = 0;
        if (l >= net.nl) continue;
        const int rows = 16 * e.R[l];
        int cols;
        if (l == 0) cols = net.in_pad;
        else cols = e.bf16 ? 32 * ((e.R[l - 1] + 1) / 2) : 16 * e.R[l - 1];
        const int pitch = cols + unit;
        off = (off + (16 / es) - 1) / (16 / es) * (16 / es);   // 16-byte aligned layer base
        p->lw[l] = off;
        p->lpitch[l] = pitch;
        p->lrows[l] = rows;
        p->lcols[l] = cols;
        p->lb[l] = boff;
        off += rows * pitch;
        boff += rows;
    }
    p->lbias_byte = (off * es + 15) / 16 * 16;
    p->lds_bytes = p->lbias_byte + boff * 4;
    return p->lds_bytes;
}

int resident_lds_bytes(const Net &net)
{
    KernelEntry e{};
    e.bf16 = net.bf16;
    for (int l = 0; l < MAXL; ++l) {
        e.R[l] = l < net.nl ? (net.fo[l] + 15) / 16 : 0;
        if (net.bf16 && l < net.nl - 1 && (e.R[l] & 1)) e.R[l] += 1;
    }
    FitPlan p{};
    return lds_layout(net, e, &p);
}

// Whether kernel entry e covers the network; *cost is the model cost used to
// rank the entries that do.
static bool entry_fits(const Net &net, const KernelEntry &e, double *cost)
{
    int need[MAXL] = {0, 0, 0, 0};
    for (int l = 0; l < net.nl; ++l) {
        need[l] = (net.fo[l] + 15) / 16;
        // BF16 chains need even 16-row blocks for every layer that feeds another
        if (net.bf16 && l < net.nl - 1 && (need[l] & 1)) need[l] += 1;
    }
    if (e.bf16 != net.bf16) return false;
    if (e.act >= 0) {
        for (int l = 0; l < net.nl - 1; ++l)   // a fixed activation must match every hidden layer
            if (net.act[l] != e.act) return false;
    }
    double c = 0.0;
    for (int l = 0; l < MAXL; ++l) {
        const bool present = l < net.nl;
        if (present != (e.R[l] > 0) || (present && e.R[l] < need[l])) return false;
        if (present) c += (double)e.R[l] * (l == 0 ? net.in_pad : net.fo[l - 1] + 16);
    }
    if (e.wl) {
        FitPlan tmp{};
        if (lds_layout(net, e, &tmp) > net.lds_max) return false;
        c *= 0.5;                             // staged weights beat global fragment loads
    }
    if (e.act >= 0) c *= 0.9;                 // specialised activation: straight-line epilogue
    *cost = c;
    return true;
}

// Blocks per spark row by default: enough blocks to fill the chip (about 4 per
// CU) while keeping at least two slab groups per wavefront.  A launch too small
// to fill the chip even then (a few rows: the re-check of the winners, the
// guiding sparks of a small job) takes one slab group per wavefront, since its
// duration is the chain of passes a block runs one after another.
static int default_bpr(const Net &net, const KernelEntry &e, int rows)
{
    const int group = e.nw * 16 * e.P;                    // samples per block pass
    const int max_bpr = (net.S_pad + group - 1) / group;
    int bpr = (1024 + rows - 1) / (rows > 0 ? rows : 1);
    const int lim = (long)rows * max_bpr <= 1024 ? max_bpr : max_bpr / 2 > 0 ? max_bpr / 2 : 1;
    if (bpr > lim) bpr = lim;
    if (bpr > MAX_BPR) bpr = MAX_BPR;
    return bpr < 1 ? 1 : bpr;
}

// The plan for entry e with about `bpr` blocks per row (rounded to whole block passes).
static void make_plan(const Net &net, const KernelEntry &e, int rows, int bpr, FitPlan *plan)
{
    plan->kernel = e.fn;
    plan->gkernel = e.gfn;
    plan->nw = e.nw;
    plan->P = e.P;
    plan->wl = e.wl;
    plan->rows = rows;
    lds_layout(net, e, plan);
    if (!e.wl) plan->lds_bytes = 0;
    const int group = e.nw * 16 * e.P;
    int spb = (net.S_pad + bpr - 1) / bpr;
    spb = (spb + group - 1) / group * group;
    plan->bpr = (net.S_pad + spb - 1) / spb;
    plan->spb = spb;
}

bool fit_select(const Net &net, int rows, FitPlan *plan)
{
    const KernelEntry *best = nullptr;
    double best_cost = 0.0;
    for (auto table : kTables) {
        int nent = 0;
        const KernelEntry *ents = table(&nent);
        for (int ie = 0; ie < nent; ++ie) {
            double cost = 0.0;
            if (!entry_fits(net, ents[ie], &cost)) continue;
            if (!best || cost < best_cost) {
                best = &ents[ie];
                best_cost = cost;
            }
        }
    }
    if (!best) return false;
    make_plan(net, *best, rows, default_bpr(net, *best, rows), plan);
    return true;
}

int fit_candidates(const Net &net, int rows, FitPlan *out, int max_out)
{
    int n = 0;
    for (auto table : kTables) {
        int nent = 0;
        const KernelEntry *ents = table(&nent);
        for (int ie = 0; ie < nent; ++ie) {
            double cost = 0.0;
            if (!entry_fits(net, ents[ie], &cost)) continue;
            const int b0 = default_bpr(net, ents[ie], rows);
            for (int b : {b0, 2 * b0, b0 / 2, 4 * b0}) {
                if (b < 1 || b > MAX_BPR || n >= max_out) continue;
                FitPlan p{};
                make_plan(net, ents[ie], rows, b, &p);
                bool dup = false;
                for (int i = 0; i < n; ++i)
                    dup = dup || (out[i].kernel == p.kernel && out[i].bpr == p.bpr);
                if (!dup) out[n++] = p;
            }
        }
    }
    return n;
}

hipError_t fit_prepare(const FitPlan &plan)
{
    if (plan.lds_bytes <= 0) return hipSuccess;
    return hipFuncSetAttribute(plan.kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               plan.lds_bytes);
}

FitLaunch fit_launch_args(const Net &net, const FitPlan &plan, const DevState &d, const float *W,
                          size_t ld, int rows, OutMap map, float *out, const SparkRegen *rg)
{
    FitLaunch f;
    FitArgs &a = f.a;
    a.rg = rg ? *rg : SparkRegen{};
    a.W = W;
    a.ld = ld;
    a.rows = rows;
    a.X = d.Xp;
    a.Xb = d.Xb;
    a.in_pad = net.in_pad;
    a.S = net.S;
    a.S_pad = net.S_pad;
    a.nl = net.nl;
    for (int l = 0; l < MAXL; ++l) {
        a.fi[l] = net.fi[l];
        a.fo[l] = net.fo[l];
        a.woff[l] = net.woff[l];
        a.boff[l] = net.boff[l];
        a.act[l] = net.act[l];
        a.vec[l] = net.vec[l];
        a.lw[l] = plan.lw[l];
        a.lpitch[l] = plan.lpitch[l];
        a.lrows[l] = plan.lrows[l];
        a.lcols[l] = plan.lcols[l];
        a.lb[l] = plan.lb[l];
    }
    a.lbias_byte = plan.lbias_byte;
    a.loss = net.loss;
    a.Y = d.Ypad;
    a.lab = d.Lpad;
    a.bpr = plan.bpr;
    a.spb = plan.spb;
    a.partial = d.partial;
    f.inv_norm = net.inv_norm;
    f.map = map;
    f.out = out;
    return f;
}

dim3 fitness_grid(const FitLaunch &f) { return dim3((unsigned)(f.a.rows * f.a.bpr)); }
dim3 finalize_grid(const FitLaunch &f) { return dim3((unsigned)((f.a.rows + 255) / 256)); }

hipError_t launch_fitness(const Net &net, const FitPlan &plan, const DevState &d, const float *W,
                          size_t ld, int rows, OutMap map, float *out, hipStream_t st,
                          hipEvent_t mid, const SparkRegen *rg)
{
    if (rows <= 0) return hipSuccess;
    if (rg && !plan.wl) return hipErrorInvalidValue;   // only the staging regenerates
    FitLaunch f = fit_launch_args(net, plan, d, W, ld, rows, map, out, rg);
    FitArgs &a = f.a;
    void *args[] = {&a};
    hipError_t e = hipLaunchKernel(plan.kernel, dim3((unsigned)(rows * plan.bpr)),
                                   dim3(64 * plan.nw), args, (size_t)plan.lds_bytes, st);
    if (e != hipSuccess) return e;
    if (mid) {
        e = hipEventRecord(mid, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_fit_finalize, finalize_grid(f), dim3(256), 0, st, d.partial, rows,
                       plan.bpr, net.inv_norm, map, out);
    return hipGetLastError();
}

hipError_t fit_group_prepare(const void *gkernel, int lds_bytes)
{
    if (lds_bytes <= 0) return hipSuccess;
    return hipFuncSetAttribute(gkernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

hipError_t launch_fitness_group(const GroupTable &t, const void *gkernel, int nw, int lds_bytes,
                                int which, hipStream_t st)
{
    GroupTable tt = t;
    void *args[] = {&tt, &which};
    return hipLaunchKernel(gkernel, dim3((unsigned)t.start[t.njobs]), dim3(64 * nw), args,
                           (size_t)lds_bytes, st);
}

hipError_t launch_finalize_group(const GroupTable &t, int which, hipStream_t st)
{
    hipLaunchKernelGGL(k_fit_finalize_group, dim3((unsigned)t.start[t.njobs]), dim3(256), 0, st, t,
                       which);
    return hipGetLastError();
}

hipError_t launch_pack_problem(const Net &net, const float *x, const float *y,
                               const int32_t *labels, const DevState &d, hipStream_t st)
{
    const int out = net.fo[net.nl - 1];
    size_t n = (size_t)net.S_pad * net.in_pad;
    if ((size_t)net.S_pad * out > n) n = (size_t)net.S_pad * out;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_pack, dim3(blocks), dim3(256), 0, st, x, net.loss == 0 ? y : nullptr,
                       net.loss == 1 ? labels : nullptr, net.S, net.S_pad, net.fi[0], net.in_pad,
                       out, net.bf16, d.Xp, d.Xb, net.loss == 0 ? d.Ypad : nullptr,
                       net.loss == 1 ? d.Lpad : nullptr);
    return hipGetLastError();
}

}  // namespace mgfwa
