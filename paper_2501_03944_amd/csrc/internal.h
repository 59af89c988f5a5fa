// Internal interfaces between the host runtime (capi.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mgfwa.h"
#include "device_common.h"

namespace mgfwa {

constexpr int MAXL = 4;        // Linear layers per MLP
constexpr int MAXW = 256;      // widest layer output
constexpr int S_ALIGN = 256;   // sample padding of the packed problem data

// Where a row's result goes: out[(r / per) * stride + offset + r % per].
struct OutMap {
    int per, stride, offset;
    // rows from `split` on form a second segment: (r' / per2) * stride + offset2 + r' % per2
    int split = 0x7fffffff, per2 = 1, offset2 = 0;
    __host__ __device__ size_t index(int r) const
    {
        if (r < split) return (size_t)(r / per) * stride + offset + r % per;
        const int q = r - split;
        return (size_t)(q / per2) * stride + offset2 + q % per2;
    }
};

// Device pointers carved out of the caller's workspace.
struct DevState {
    float *F, *SE, *SG, *A, *Y, *Yprev, *Yc, *best_x, *best_y, *partial;
    float *Aexp;       // [B*N] amplitude the generation's sparks were exploded with
    int32_t *fresh, *top, *bottom, *tie, *cstar, *improved, *reinit, *src, *best_f, *best_gen,
        *best_upd, *ctrl;
    float *Xp;         // [S_pad][in_pad] packed inputs (FP32 precision)
    uint16_t *Xb;      // [S_pad][in_pad] packed inputs as bf16 bits (BF16 precision)
    float *Ypad;       // [S_pad][out] MSE targets (zero padded)
    int32_t *Lpad;     // [S_pad] CE labels (-1 padded)
    char *Wpack;       // packed spark rows for the wide-first-layer kernel
    char *Xw;          // [S_pad][Kp] samples with a ones column (wide kernel)
    float *lo, *hi;    // [B][Dp] population ranges (range mapping)
    float *Pnet;       // packed parameters of a fixed network (input problems)
    float *H0, *H1;    // [partial_rows][hnp] activations between layers (input problems)
    float *zero;       // 256 zero bytes (input problems)
    float *Wstar;      // [B*N][Dp] each firework's best candidate (FP32 re-check of BF16 runs)
    float *Ystar;      // [B*N] its FP32 fitness
};

// Population shape and algorithm constants as the kernels need them.
struct Shape {
    int B, N, lam, G, m, k, BN, C;     // C = lam + G candidates per firework
    int D, Dp;                         // spark length and padded row pitch (floats)
    float inv_k, boost, amp_up, amp_down, amp0;
    int T, loser_out, use_target;
    float target;
    Box box;
    uint2 key;
    int lag;                           // guiding from the previous generation's sparks
    int map_range;                     // random mapping into the population's range
    int regen;                         // the guiding and apply steps regenerate explosion
                                       // sparks instead of reading SE
    int recheck;                       // BF16 fitness: each firework's best candidate is
                                       // re-evaluated in FP32 before the selection compares it
};

// MLP problem as the fitness kernels need it.
struct Net {
    int nl;                            // layers
    int fi[MAXL], fo[MAXL];            // in/out width per layer
    int woff[MAXL], boff[MAXL];        // offsets of W_l and b_l inside a spark
    int act[MAXL];                     // activation after layer l (identity for the last)
    int vec[MAXL];                     // 1 when W_l rows allow 16-byte loads
    int loss;                          // 0 MSE, 1 CE
    int S, S_pad, in_pad;              // samples, padded samples, padded input width
    int bf16;                          // precision
    float inv_norm;                    // 1/(S*out) for MSE, 1/S for CE
    int lds_max;                       // LDS bytes a block may use (0: weights stay in global)
    int wide;                          // first layer streamed through LDS (two-layer nets)
    int num_cu;                        // compute units (persistent grid size)
};

// A fixed MLP whose input is the spark (the paper's testbed, eq. (1)), as its
// fitness kernel needs it.  Packed parameters: per layer W_l zero-padded to
// np[l] x kp[l] (row-major, output-major like nn.Linear), then b_l padded to
// np[l]; kp of a hidden layer is np of the layer before it.
constexpr int NET_MAXL = 12;
constexpr int NET_MAXW = 512;
struct InNet {
    int nl;                            // layers (the last has one output)
    int fi[NET_MAXL], fo[NET_MAXL];    // true widths
    int kp[NET_MAXL], np[NET_MAXL];    // K and N padded to 16
    int act[NET_MAXL];                 // activation after layer l (identity for the last)
    int woff[NET_MAXL], boff[NET_MAXL];// float offsets into the packed parameters
    int n_packed;                      // floats of the packed parameters
    int hs;                            // LDS row pitch (floats) of the activation tile
    int hnp;                           // widest hidden output (padded): activation row pitch
    int num_cu;                        // compute units (rows per block choice)
    int path;                          // 0 choose per launch, 1 whole-network tiles, 2 layer by
                                       // layer, 3 layer by layer with LDS-staged tiles
};

// Explosion sparks of a fitness launch that are not stored: launch row r is
// explosion row r of generation ctrl[CTRL_GEN] + 1, regenerated from its
// firework's row and amplitude (and the population range) exactly as the
// explosion kernel draws it.
struct SparkRegen {
    const float *F, *A, *lo, *hi;
    const int32_t *ctrl;
    uint2 key;
    Box box;
    int lam, N, D, Dp;
};

// Arguments of the register-chain fitness kernel (fit_kernel.h).
struct FitArgs {
    const float *W;        // spark rows
    size_t ld;             // row pitch (floats)
    int rows;
    const float *X;        // [S_pad][in_pad] (FP32 kernels)
    const uint16_t *Xb;    // [S_pad][in_pad] bf16 bits (BF16 kernels)
    int in_pad, S, S_pad;
    int nl;
    int fi[MAXL], fo[MAXL], woff[MAXL], boff[MAXL], act[MAXL], vec[MAXL];
    // LDS layout (WL kernels), per layer: weight offset and row pitch in
    // elements of the storage type, padded rows and columns, bias offset (floats)
    int lw[MAXL], lpitch[MAXL], lrows[MAXL], lcols[MAXL], lb[MAXL];
    int lbias_byte;        // start of the FP32 bias area
    int loss;
    const float *Y;        // [S_pad][out]
    const int32_t *lab;    // [S_pad]
    int bpr, spb;
    float *partial;        // [rows][bpr]
    // Explosion sparks regenerated while staging (rg.F non-null, LDS-staged
    // kernels only); W is then not read.
    SparkRegen rg;
};

// A chosen fitness kernel and its launch geometry for a given row count.
struct FitPlan {
    const void *kernel;   // __global__ function
    const void *gkernel;  // its grouped form (k_fit_group)
    int nw;               // wavefronts per block
    int P;                // 16-sample slabs per wave in flight
    int wl;               // weights staged in LDS
    int bpr;              // blocks per spark row
    int spb;              // samples per block
    int rows;
    // LDS layout of the staged weights (wl = 1)
    int lw[MAXL], lpitch[MAXL], lrows[MAXL], lcols[MAXL], lb[MAXL];
    int lbias_byte, lds_bytes;
    int net_shape = -1;   // input problems: NET_* kernel shape (-1 chosen per launch)
};

// The wide fitness kernel's packed spark rows, for the explosion kernel to
// write each spark there as well (the fitness launch then skips packing them).
// Row layout (fit_wide.hip): W1 with b1 as column `in`, K-blocked as
// [Kp/32][256][32]; W2 [16][256] (BF16: each 32-column block in MFMA lane
// order); b2 [16] FP32.  Padding stays zero from initialisation.
struct WidePack {
    char *Wp;                           // packed rows
    size_t pr;                          // row pitch (bytes)
    int in, hid, out, Kp, bf16;
    int woff1, boff1, woff2, boff2;     // parameter offsets inside a spark
};

// Byte offset of W1aug element (o, k) (b1 is column k = in) in a packed row.
__device__ __forceinline__ size_t wide_w1_offset(int o, int k, size_t es)
{
    return (((size_t)(k >> 5) * 256 + o) * 32 + (k & 31)) * es;
}

// Byte offset of spark coordinate j (< D) in its packed row; *f32 is set when
// the element is stored as FP32 whatever the precision (b2).
__device__ __forceinline__ size_t wide_pack_offset(const WidePack &p, int j, bool *f32)
{
    const size_t es = p.bf16 ? 2 : 4;
    *f32 = false;
    int o, k;
    if (j >= p.woff1 && j < p.woff1 + p.hid * p.in) {
        const int rel = j - p.woff1;
        o = rel / p.in;
        k = rel - o * p.in;
    } else if (j >= p.boff1 && j < p.boff1 + p.hid) {
        o = j - p.boff1;
        k = p.in;
    } else if (j >= p.woff2 && j < p.woff2 + p.out * p.hid) {
        const int rel = j - p.woff2, i = rel / p.hid, c = rel - i * p.hid;
        int pos = c;
        if (p.bf16) {
            const int r = c & 31;
            pos = (c & ~31) + (r < 16 ? (r >> 2) * 8 + (r & 3) : ((r - 16) >> 2) * 8 + 4 + (r & 3));
        }
        return (size_t)256 * p.Kp * es + ((size_t)i * 256 + pos) * es;
    } else {
        *f32 = true;
        return (size_t)256 * p.Kp * es + (size_t)16 * 256 * es + (size_t)(j - p.boff2) * 4;
    }
    return wide_w1_offset(o, k, es);
}

// ---- grouped launches (batched generations) --------------------------------
// A kernel body works on one block of its launch: Blk is that block's index and
// the grid of the job's own launch.  A grouped launch runs the blocks of many
// jobs' launches of one kernel as a single 1-D grid and hands every body the
// block (and the job arguments) it would have had in the job's own launch, so a
// job computes exactly what it computes alone.
struct Blk {
    int x, y, gx, gy;
};

__device__ __forceinline__ Blk own_block()
{
    return Blk{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)gridDim.y};
}

// One fitness launch of a job: the kernel's arguments and its finalisation.
struct FitLaunch {
    FitArgs a;              // a.rows sparks, a.bpr partials each
    float inv_norm;
    OutMap map;
    float *out;
};

// Per-job arguments of the grouped kernels, in device memory (the job's workspace).
struct JobDesc {
    Shape s;
    DevState d;
    FitLaunch fit[3];       // explosion sparks, guiding sparks, FP32 re-check (BF16 jobs)
};

constexpr int GROUP_MAX = 64;   // jobs per grouped launch

// Every job's range of grouped blocks starts at a multiple of 8 (padding blocks
// exit at once), so block l of a job sits on XCD l % 8 as in its own launch: a
// job's blocks are spread over the XCDs and its XCD-aware tile order holds.
constexpr int GROUP_ALIGN = 8;

struct GroupTable {
    int njobs;
    int start[GROUP_MAX + 1];          // first grouped block of job j; start[njobs] = total
    int gx[GROUP_MAX], gy[GROUP_MAX];  // the job's own grid
    const JobDesc *job[GROUP_MAX];
};

// The job owning grouped block `bid` (binary search over start[]).
__device__ __forceinline__ int group_job(const GroupTable &t, int bid)
{
    int lo = 0, hi = t.njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.start[mid] <= bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The job's own block for grouped block bid; false for a padding block.
__device__ __forceinline__ bool group_block(const GroupTable &t, int j, int bid, Blk *b)
{
    const int l = bid - t.start[j];
    if (l >= t.gx[j] * t.gy[j]) return false;
    *b = Blk{l % t.gx[j], l / t.gx[j], t.gx[j], t.gy[j]};
    return true;
}

// Host side: a grouped launch over jobs[0..n) whose own grids are grid[i].
void group_table(const JobDesc *const *jobs, const dim3 *grid, int n, GroupTable *t);

// Each kernel's own grid for a job (the solo launches use the same functions),
// and its grouped launch over a table.
dim3 pop_range_grid(const Shape &s);
dim3 explode_grid(const Shape &s);
dim3 rank_grid(const Shape &s);
dim3 guide_grid(const Shape &s);
dim3 select_grid(const Shape &s);
dim3 firework_row_grid(const Shape &s);     // apply, gather_best
hipError_t launch_pop_range_group(const GroupTable &t, hipStream_t st);
hipError_t launch_explode_group(const GroupTable &t, hipStream_t st);   // stored FP32 sparks
hipError_t launch_rank_group(const GroupTable &t, int max_lam, hipStream_t st);
hipError_t launch_guide_group(const GroupTable &t, hipStream_t st);
hipError_t launch_gather_best_group(const GroupTable &t, hipStream_t st);
hipError_t launch_select_group(const GroupTable &t, hipStream_t st);
hipError_t launch_apply_group(const GroupTable &t, hipStream_t st);
hipError_t launch_finish_group(const GroupTable &t, hipStream_t st);    // one block per job

// ---- spark.hip
hipError_t launch_init_positions(const Shape &s, const DevState &d, hipStream_t st);
hipError_t launch_pop_range(const Shape &s, const DevState &d, hipStream_t st);
// write_se false (only with wp): the FP32 spark rows are not stored.
hipError_t launch_explode(const Shape &s, const DevState &d, hipStream_t st,
                          const WidePack *wp = nullptr, bool write_se = true);

// ---- guide.hip
hipError_t launch_rank(const Shape &s, const DevState &d, hipStream_t st);
hipError_t launch_guide(const Shape &s, const DevState &d, hipStream_t st);

// ---- select.hip
// checked: the best candidate of every firework was gathered into d.Wstar and its
// FP32 fitness stored in d.Ystar (launch_gather_best); the selection compares
// that value, and the apply step copies the gathered row.
hipError_t launch_select(const Shape &s, const DevState &d, hipStream_t st, bool checked = false);
hipError_t launch_init_select(const Shape &s, const DevState &d, hipStream_t st);
hipError_t launch_apply(const Shape &s, const DevState &d, hipStream_t st, bool checked = false);
// Per firework: c* = argmin over its candidates' fitness (lower index on ties) into
// d.cstar, and the candidate's row into d.Wstar (explosion sparks regenerated when
// s.regen).
hipError_t launch_gather_best(const Shape &s, const DevState &d, hipStream_t st);
hipError_t launch_finish(const DevState &d, int advance, hipStream_t st);
// Zero the control words (generation counter, stop flags) in stream order.
hipError_t launch_clear_ctrl(int32_t *ctrl, hipStream_t st);
hipError_t launch_store_fitness(const float *src, int rows, OutMap map, float *out,
                                const int32_t *ctrl, hipStream_t st);

// ---- fitness.hip
// Choose the kernel for the network (false if the shape is not compiled in).
bool fit_select(const Net &net, int rows, FitPlan *plan);
// Every plan that covers the network for `rows` sparks: each fitting kernel
// entry with a few blocks-per-row choices; returns the count (at most max_out).
int fit_candidates(const Net &net, int rows, FitPlan *out, int max_out);
// Device-side preparation of a chosen plan (dynamic LDS limit); needs a device.
hipError_t fit_prepare(const FitPlan &plan);
// Fitness of `rows` sparks into out[map(row)]: the GEMM kernel writes one partial
// per (row, block); the finalisation sums them in order.  `mid` (optional) is
// recorded between the two launches.
// rg (LDS-staged plans only): the sparks are regenerated, W is not read.
hipError_t launch_fitness(const Net &net, const FitPlan &plan, const DevState &d,
                          const float *W, size_t ld, int rows, OutMap map, float *out,
                          hipStream_t st, hipEvent_t mid = nullptr,
                          const SparkRegen *rg = nullptr);
// The kernel arguments and finalisation of one fitness launch (what
// launch_fitness passes), for a grouped launch's job descriptor.
FitLaunch fit_launch_args(const Net &net, const FitPlan &plan, const DevState &d, const float *W,
                          size_t ld, int rows, OutMap map, float *out,
                          const SparkRegen *rg = nullptr);
// Fitness launch `which` of every job of t, all on the same kernel instance
// (gkernel, nw wavefronts, lds_bytes of dynamic LDS: the most any of them needs;
// fit_group_prepare must have allowed it).
hipError_t fit_group_prepare(const void *gkernel, int lds_bytes);
hipError_t launch_fitness_group(const GroupTable &t, const void *gkernel, int nw, int lds_bytes,
                                int which, hipStream_t st);
hipError_t launch_finalize_group(const GroupTable &t, int which, hipStream_t st);
dim3 fitness_grid(const FitLaunch &f);     // the job's own grid of the GEMM kernel
dim3 finalize_grid(const FitLaunch &f);
hipError_t launch_pack_problem(const Net &net, const float *x, const float *y,
                               const int32_t *labels, const DevState &d, hipStream_t st);
// largest partial-sum count per row any plan may use
int fit_max_bpr();
// LDS bytes the resident-weights kernel would need for this network
int resident_lds_bytes(const Net &net);

// ---- net_input.hip (input problems)
// Pack the caller's nn.Linear-layout parameters into the padded blocks.
hipError_t launch_pack_net(const InNet &net, const float *params, float *packed, hipStream_t st);
// out[map.index(r)] = f(x_r) for the rows of X (leading dimension ld >= fi[0]);
// the layer-by-layer path keeps the activations in H0/H1 ([rows][hnp] each).
// shape: 0..3 layer by layer with 64x128, 64x64, 32x32 or K-split 16x16 tiles,
// NET_WHOLE the whole-network tiles, NET_LDS / NET_LDS64 layer by layer with
// LDS-staged 64x128 / 64x64 tiles, -1 a choice from the shape and row count.
// zero: 16 zero bytes.
constexpr int NET_WHOLE = 4;
constexpr int NET_LDS = 5;
constexpr int NET_LDS64 = 6;
hipError_t launch_net_input(const InNet &net, int shape, const float *packed, const float *X,
                            size_t ld, int rows, OutMap map, float *out, float *H0, float *H1,
                            const float *zero, hipStream_t st);
size_t net_input_lds_bytes(const InNet &net);
hipError_t net_input_prepare(const InNet &net);   // raises the kernels' LDS limit

// ---- fit_wide.hip
bool wide_applicable(const Net &net);
int wide_kp(const Net &net);
size_t wide_row_bytes(const Net &net);
int wide_lds_bytes(const Net &net);
hipError_t wide_prepare(const Net &net);
hipError_t launch_pack_wide_x(const Net &net, const float *x, char *Xw, hipStream_t st);
// prepacked: the first rows are already in d.Wpack (written by the explosion)
hipError_t launch_fitness_wide(const Net &net, const DevState &d, const float *W, size_t ld,
                               int rows, OutMap map, float *out, hipStream_t st,
                               hipEvent_t mid = nullptr, hipEvent_t pre = nullptr,
                               int prepacked = 0);
WidePack wide_pack_geometry(const Net &net, const DevState &d);

// Record the message returned by mgfwa_last_error (printf format) and return code.
mgfwa_status fail(mgfwa_status code, const char *fmt, ...);

}  // namespace mgfwa
