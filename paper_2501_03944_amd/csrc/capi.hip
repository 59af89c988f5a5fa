// Host runtime and C ABI of the MGFWA library (declarations in include/mgfwa.h).
//
// A context owns no device memory: it carves the caller's workspace into the
// state arrays, validates the configuration, and enqueues the generation loop
// of Alg. 1 on the caller's stream.  Steady-state generations are captured once
// into a HIP graph (on a private capture stream) and replayed; every kernel
// reads the generation counter from device memory, so replays need no host
// parameter updates and no host synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mgfwa.h"
#include "internal.h"

using namespace mgfwa;

namespace {
thread_local char g_err[512] = "";
}  // namespace

mgfwa_status mgfwa::fail(mgfwa_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

namespace {

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(MGFWA_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

constexpr size_t ALIGN = 256;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int round_up(int v, int a) { return (v + a - 1) / a * a; }

struct Layout {
    size_t F, SE, SG, A, Aexp, Y, Yprev, fresh, Yc, top, bottom, tie, cstar, improved, reinit, src;
    size_t best_x, best_y, best_f, best_gen, best_upd, ctrl, partial, Xp, Xb, Ypad, Lpad;
    size_t Wpack, Xw, lo, hi, Pnet, H0, H1, Zero;
    size_t Wstar, Ystar, Xp32, Wpack32, Xw32;   // FP32 re-check of BF16 selection winners
    size_t desc;                                // the job's descriptor for grouped launches
    size_t total;
    int partial_rows;
};

enum Phase { PH_READY, PH_INIT_ASK, PH_INIT_TELL, PH_EXPL_TELL, PH_GUIDE_ASK, PH_GUIDE_TELL };

struct Derived {
    Shape s;
    Net net;
    Net net32;       // BF16 runs: the same network in FP32 (selection re-check)
    InNet in;        // input problems: the fixed network
    bool input;
    Layout lay;
};

bool finite(float v) { return std::isfinite(v); }

// rows per firework of the explosion-fitness launch
int expl_rows(const Shape &s) { return s.lag ? s.C : s.lam; }

mgfwa_status derive(const mgfwa_config *c, const mgfwa_problem *p, Derived *out)
{
    if (!c || !p) return fail(MGFWA_EINVAL, "config and problem are required");
    if (c->n_populations < 1 || c->n_fireworks < 1 || c->n_guiding < 1)
        return fail(MGFWA_EINVAL, "n_populations, n_fireworks and n_guiding must be >= 1");
    if (c->n_sparks < 2 || c->n_sparks % c->n_guiding != 0 || c->n_sparks / c->n_guiding < 2)
        return fail(MGFWA_EINVAL, "n_sparks must be a multiple of n_guiding with >= 2 sparks per group");
    if (c->n_sparks > 8192) return fail(MGFWA_EINVAL, "n_sparks > 8192");
    if (!(c->sigma > 0.0f && c->sigma <= 0.5f)) return fail(MGFWA_EINVAL, "sigma outside (0, 0.5]");
    if (!finite(c->lb) || !finite(c->ub) || !(c->lb < c->ub)) return fail(MGFWA_EINVAL, "need finite lb < ub");
    if (!finite(c->boost) || !finite(c->amp_up) || !finite(c->amp_down) || !finite(c->amp_init) ||
        c->amp_up <= 0.0f || c->amp_down <= 0.0f)
        return fail(MGFWA_EINVAL, "boost/amplitude parameters must be finite, factors > 0");
    if (c->max_generations < 1) return fail(MGFWA_EINVAL, "max_generations must be >= 1");
    if (c->lag_guiding && c->external_fitness)
        return fail(MGFWA_EUNSUPPORTED, "lag_guiding needs the built-in fitness");
    if (c->precision != MGFWA_FP32 && c->precision != MGFWA_BF16)
        return fail(MGFWA_EINVAL, "unknown precision %d", c->precision);
    if (c->fit_path < 0 || c->fit_path > (p->kind == MGFWA_PROBLEM_INPUT ? 3 : 2))
        return fail(MGFWA_EINVAL, "fit_path %d out of range for this problem kind", c->fit_path);
    if (p->kind != MGFWA_PROBLEM_WEIGHTS && p->kind != MGFWA_PROBLEM_INPUT)
        return fail(MGFWA_EINVAL, "unknown problem kind %d", p->kind);
    const bool input = p->kind == MGFWA_PROBLEM_INPUT;
    const int max_layers = input ? MGFWA_MAX_LAYERS : MGFWA_MAX_TRAIN_LAYERS;
    if (p->n_layers < 1 || p->n_layers > max_layers)
        return fail(MGFWA_EINVAL, "n_layers must be in [1, %d]", max_layers);
    for (int l = 0; l <= p->n_layers; ++l)
        if (p->widths[l] < 1) return fail(MGFWA_EINVAL, "width %d must be >= 1", l);
    if (p->widths[0] > 65536) return fail(MGFWA_EINVAL, "input width > 65536");
    for (int l = 0; l < p->n_layers - 1; ++l)
        if (p->hidden_act[l] < 0 || p->hidden_act[l] > MGFWA_ACT_GELU)
            return fail(MGFWA_EINVAL, "unknown activation %d", p->hidden_act[l]);
    if (input) {
        if (p->widths[p->n_layers] != 1)
            return fail(MGFWA_EINVAL, "the fixed network of an input problem has one output");
        for (int l = 1; l < p->n_layers; ++l)
            if (p->widths[l] > MGFWA_MAX_NET_WIDTH)
                return fail(MGFWA_EUNSUPPORTED, "hidden width %d > %d", p->widths[l],
                            MGFWA_MAX_NET_WIDTH);
        if (c->precision != MGFWA_FP32)
            return fail(MGFWA_EUNSUPPORTED, "input problems run in FP32");
    } else {
        for (int l = 1; l <= p->n_layers; ++l)
            if (p->widths[l] > MGFWA_MAX_WIDTH)
                return fail(MGFWA_EUNSUPPORTED, "layer width %d > %d", p->widths[l],
                            MGFWA_MAX_WIDTH);
        if (p->loss != MGFWA_LOSS_MSE && p->loss != MGFWA_LOSS_CE)
            return fail(MGFWA_EINVAL, "unknown loss %d", p->loss);
        if (p->loss == MGFWA_LOSS_CE && p->widths[p->n_layers] < 2)
            return fail(MGFWA_EINVAL, "cross-entropy needs >= 2 outputs");
    }
    const bool need_data = !c->external_fitness || (input ? p->net_dev : p->x_dev);
    if (need_data && input) {
        if (!p->net_dev) return fail(MGFWA_EINVAL, "net_dev is NULL");
    } else if (need_data) {
        if (p->n_samples < 1 || p->n_samples > (1 << 24))
            return fail(MGFWA_EINVAL, "n_samples must be in [1, 2^24]");
        if (!p->x_dev) return fail(MGFWA_EINVAL, "x_dev is NULL");
        if (p->loss == MGFWA_LOSS_MSE && !p->y_dev) return fail(MGFWA_EINVAL, "y_dev is NULL");
        if (p->loss == MGFWA_LOSS_CE && !p->labels_dev) return fail(MGFWA_EINVAL, "labels_dev is NULL");
    }

    Shape &s = out->s;
    s.B = c->n_populations;
    s.N = c->n_fireworks;
    s.lam = c->n_sparks;
    s.G = c->n_guiding;
    s.m = s.lam / s.G;
    s.k = std::max(1, (int)std::floor((double)c->sigma * (double)s.m));
    s.BN = s.B * s.N;
    s.C = s.lam + s.G;
    long D = 0;
    Net &net = out->net;
    std::memset(&net, 0, sizeof net);
    InNet &in = out->in;
    std::memset(&in, 0, sizeof in);
    out->input = input;
    if (input) {
        // the spark is the network's input; the parameters are packed once
        in.nl = p->n_layers;
        int off = 0, hmax = 0;
        for (int l = 0; l < p->n_layers; ++l) {
            in.fi[l] = p->widths[l];
            in.fo[l] = p->widths[l + 1];
            in.kp[l] = round_up(in.fi[l], 16);
            in.np[l] = round_up(in.fo[l], 16);
            in.act[l] = l < p->n_layers - 1 ? p->hidden_act[l] : MGFWA_ACT_IDENTITY;
            in.woff[l] = off;
            off += in.np[l] * in.kp[l];
            in.boff[l] = off;
            off += in.np[l];
            if (l > 0) hmax = std::max(hmax, in.kp[l]);
        }
        in.n_packed = off;
        in.hs = hmax + 4;   // 16-byte skew between the rows of the activation tile
        in.hnp = hmax;      // hidden outputs: np[l] = kp[l+1]
        // fit_path 1 / 2 / 3 forces the whole-network / layer-by-layer /
        // LDS-staged layer-by-layer kernels (before autotuning)
        in.path = c->fit_path;
        D = p->widths[0];
    } else {
        net.nl = p->n_layers;
        for (int l = 0; l < p->n_layers; ++l) {
            net.fi[l] = p->widths[l];
            net.fo[l] = p->widths[l + 1];
            net.woff[l] = (int)D;
            D += (long)net.fi[l] * net.fo[l];
            net.boff[l] = (int)D;
            D += net.fo[l];
            net.act[l] = l < p->n_layers - 1 ? p->hidden_act[l] : MGFWA_ACT_IDENTITY;
            net.vec[l] = (net.woff[l] % 4 == 0) && (net.fi[l] % 4 == 0);
        }
    }
    if (D > (1L << 26)) return fail(MGFWA_EINVAL, "spark dimension %ld too large", D);
    s.D = (int)D;
    s.Dp = round_up(s.D, 64);
    if ((long)s.BN * s.lam > (1L << 30)) return fail(MGFWA_EINVAL, "too many sparks");
    s.inv_k = (float)(1.0 / (double)s.k);
    s.boost = c->boost;
    s.amp_up = c->amp_up;
    s.amp_down = c->amp_down;
    s.box.lb = c->lb;
    s.box.ub = c->ub;
    s.box.span = c->ub - c->lb;
    s.amp0 = c->amp_init > 0.0f ? c->amp_init : s.box.span;
    s.T = c->max_generations;
    s.loser_out = c->loser_out ? 1 : 0;
    s.use_target = c->use_target ? 1 : 0;
    s.target = c->target_loss;
    s.key = make_uint2((uint32_t)c->seed, (uint32_t)(c->seed >> 32));
    s.lag = c->lag_guiding ? 1 : 0;
    s.map_range = c->map_range ? 1 : 0;

    int outw = 1;
    if (input) {
        net.loss = -1;   // no sample data, no targets
    } else {
        net.loss = p->loss;
        net.bf16 = c->precision == MGFWA_BF16;
        net.S = need_data ? p->n_samples : 0;
        net.S_pad = need_data ? round_up(p->n_samples, S_ALIGN) : 0;
        net.in_pad = round_up(net.fi[0], net.bf16 ? 32 : 16);
        outw = net.fo[net.nl - 1];
        net.inv_norm = net.loss == MGFWA_LOSS_MSE ? (float)(1.0 / ((double)net.S * outw))
                                                  : (float)(1.0 / (double)net.S);
        // Two-layer networks whose staged weights exceed the LDS stream their first
        // layer through LDS instead; fit_path 1 / 2 forces either family.
        if (c->fit_path == 2 && need_data && !wide_applicable(net))
            return fail(MGFWA_EUNSUPPORTED, "the wide fitness kernel needs a two-layer net with "
                                            "hidden width <= 256 and <= 16 outputs");
        net.wide = need_data && wide_applicable(net) &&
                   (c->fit_path == 2 ||
                    (c->fit_path == 0 && resident_lds_bytes(net) > 160 * 1024 - 512));
        if (net.wide && net.S_pad / 256 > fit_max_bpr())
            return fail(MGFWA_EUNSUPPORTED, "too many samples for the wide fitness kernel");
    }
    // The wide kernel reads the explosion's packed rows: the FP32 rows are then
    // not stored, and the guiding and apply steps regenerate the sparks they
    // need (the lag order reads the previous generation's sparks: it keeps them).
    s.regen = net.wide && !s.lag ? 1 : 0;
    // BF16 fitness ranks the candidates; the winner of each firework is
    // re-evaluated in FP32 before the selection compares it, so the firework and
    // best-so-far fitness stay FP32 (and so does the initial fitness)
    s.recheck = !input && net.bf16 && need_data ? 1 : 0;
    Net &net32 = out->net32;
    net32 = net;
    if (s.recheck) {
        net32.bf16 = 0;
        net32.in_pad = round_up(net.fi[0], 16);
    }

    Layout &L = out->lay;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, ALIGN);
        return o;
    };
    const size_t BN = s.BN, Dp = s.Dp;
    L.F = take(BN * Dp * 4);
    L.SE = take(BN * s.lam * Dp * 4);
    L.SG = take(BN * s.G * Dp * 4);
    L.A = take(BN * 4);
    L.Aexp = take(BN * 4);
    L.Y = take(BN * 4);
    L.Yprev = take(BN * 4);
    L.fresh = take(BN * 4);
    L.Yc = take(BN * s.C * 4);
    L.top = take(BN * s.G * s.k * 4);
    L.bottom = take(BN * s.G * s.k * 4);
    L.tie = take(BN * s.G * 4);
    L.cstar = take(BN * 4);
    L.improved = take(BN * 4);
    L.reinit = take(BN * 4);
    L.src = take(BN * 4);
    L.best_x = take((size_t)s.B * Dp * 4);
    L.best_y = take((size_t)s.B * 4);
    L.best_f = take((size_t)s.B * 4);
    L.best_gen = take((size_t)s.B * 4);
    L.best_upd = take((size_t)s.B * 4);
    L.ctrl = take(CTRL_WORDS * 4);
    // the lag order evaluates the explosion and guiding sparks (adjacent
    // buffers) in one launch
    L.partial_rows = (int)std::max<size_t>(BN * (s.lag ? s.C : s.lam), 1024);
    L.partial = take((size_t)L.partial_rows * fit_max_bpr() * 4);
    const size_t nx = (size_t)net.S_pad * net.in_pad;
    L.Xp = take(net.bf16 ? 0 : nx * 4);
    L.Xb = take(net.bf16 ? nx * 2 : 0);
    L.Ypad = take(net.loss == MGFWA_LOSS_MSE ? (size_t)net.S_pad * outw * 4 : 0);
    L.Lpad = take(net.loss == MGFWA_LOSS_CE ? (size_t)net.S_pad * 4 : 0);
    L.Wpack = take(net.wide ? (size_t)L.partial_rows * wide_row_bytes(net) : 0);
    L.Xw = take(net.wide ? (size_t)net.S_pad * wide_kp(net) * (net.bf16 ? 2 : 4) : 0);
    L.lo = take(s.map_range ? (size_t)s.B * Dp * 4 : 0);
    L.hi = take(s.map_range ? (size_t)s.B * Dp * 4 : 0);
    L.Pnet = take(input && need_data ? (size_t)in.n_packed * 4 : 0);
    const size_t hbytes = input && need_data ? (size_t)L.partial_rows * in.hnp * 4 : 0;
    L.H0 = take(hbytes);
    L.H1 = take(hbytes);
    L.Zero = take(input && need_data ? 256 : 0);
    L.Wstar = take(s.recheck ? BN * Dp * 4 : 0);
    L.Ystar = take(s.recheck ? BN * 4 : 0);
    L.Xp32 = take(s.recheck && !net.wide ? (size_t)net32.S_pad * net32.in_pad * 4 : 0);
    L.Wpack32 = take(s.recheck && net.wide ? BN * wide_row_bytes(net32) : 0);
    L.Xw32 = take(s.recheck && net.wide ? (size_t)net32.S_pad * wide_kp(net32) * 4 : 0);
    L.desc = take(sizeof(JobDesc));
    L.total = off;
    if (s.lag && L.SG != L.SE + BN * s.lam * Dp * 4)
        return fail(MGFWA_EINVAL, "internal: guiding sparks must follow the explosion sparks");
    return MGFWA_OK;
}

}  // namespace

struct mgfwa_ctx {
    mgfwa_config cfg;
    Shape s;
    Net net;
    Net net32;          // BF16 runs: the FP32 network of the selection re-check
    DevState d32;       // ... and its FP32 sample buffers (shares the rest of d)
    JobDesc *desc_dev = nullptr;   // descriptor for grouped (batched) launches, in the workspace
    FitPlan plan_check; // ... and its launch over the B*N gathered rows
    InNet in;
    bool input = false;
    Layout lay;
    DevState d;
    bool has_data;
    char *ws;
    hipStream_t stream;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool use_graph = true;
    bool sync_debug = false;
    FitPlan plan_init, plan_expl, plan_guide, plan_eval;
    Phase phase = PH_READY;
    int gen_host = 0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> pool;
    std::vector<std::vector<hipEvent_t>> pending;
    std::vector<double> gen_ms;
    double phase_ms[MGFWA_N_PHASES] = {0, 0, 0, 0, 0};
    double fit_kernel_ms = 0.0;
    double check_ms = 0.0;
};

namespace {

template <typename T>
T *at(char *base, size_t off) { return reinterpret_cast<T *>(base + off); }

mgfwa_status check(mgfwa_ctx *c, hipError_t e, const char *what)
{
    if (e != hipSuccess) return fail(MGFWA_EHIP, "%s: %s", what, hipGetErrorString(e));
    if (c->sync_debug) {
        hipError_t s = hipStreamSynchronize(c->stream);
        if (s != hipSuccess) return fail(MGFWA_EHIP, "%s (sync): %s", what, hipGetErrorString(s));
    }
    return MGFWA_OK;
}

#define STEP(expr, what)                                  \
    do {                                                  \
        mgfwa_status st_ = check(c, (expr), what);        \
        if (st_ != MGFWA_OK) return st_;                  \
    } while (0)

const OutMap kFlat = {1, 1, 0};
constexpr int N_EVENTS = 10;   // per timed generation (enqueue_generation)

// The explosion-fitness launch: BN*lambda explosion sparks into the first
// lambda candidate slots or, in the lag order, those followed by the BN*G
// guiding sparks into the last G slots.
OutMap expl_map(const Shape &s)
{
    OutMap m{s.lam, s.C, 0};
    if (s.lag) {
        m.split = s.BN * s.lam;
        m.per2 = s.G;
        m.offset2 = s.lam;
    }
    return m;
}

// Whether mgfwa_step leaves the explosion sparks unstored: the wide kernel reads
// the explosion's packed rows; with regen_sparks an LDS-staged register-chain
// plan regenerates them.  The lag order reads the previous generation's sparks.
bool sparks_regenerated(const mgfwa_ctx *c)
{
    if (c->s.lag || c->input || !c->has_data) return false;
    if (c->net.wide) return true;
    return c->cfg.regen_sparks && c->plan_expl.wl;
}

// The explosion-fitness launch's source when its sparks are regenerated.
SparkRegen spark_regen(const mgfwa_ctx *c)
{
    const Shape &s = c->s;
    SparkRegen g;
    g.F = c->d.F;
    g.A = c->d.A;
    g.lo = s.map_range ? c->d.lo : nullptr;
    g.hi = s.map_range ? c->d.hi : nullptr;
    g.ctrl = c->d.ctrl;
    g.key = s.key;
    g.box = s.box;
    g.lam = s.lam;
    g.N = s.N;
    g.D = s.D;
    g.Dp = s.Dp;
    return g;
}

mgfwa_status fit_rows(mgfwa_ctx *c, const FitPlan &plan, const float *W, size_t ld, int rows,
                      OutMap map, float *out, hipStream_t st, hipEvent_t mid = nullptr,
                      hipEvent_t pre = nullptr, int prepacked = 0, const SparkRegen *rg = nullptr)
{
    if (c->input) {
        STEP(launch_net_input(c->in, plan.net_shape, c->d.Pnet, W, ld, rows, map, out, c->d.H0,
                              c->d.H1, c->d.zero, st),
             "fitness_input");
        if (mid) STEP(hipEventRecord(mid, st), "event");
    } else if (c->net.wide)
        STEP(launch_fitness_wide(c->net, c->d, W, ld, rows, map, out, st, mid, pre, prepacked),
             "fitness_wide");
    else
        STEP(launch_fitness(c->net, plan, c->d, W, ld, rows, map, out, st, mid, rg), "fitness");
    return MGFWA_OK;
}

// FP32 fitness of `rows` rows of W (leading dimension Dp) into out[0..rows): the
// selection re-check of a BF16 run (the FP32 network and sample buffers).
mgfwa_status fit_check(mgfwa_ctx *c, const float *W, int rows, float *out, hipStream_t st)
{
    if (c->net32.wide)
        STEP(launch_fitness_wide(c->net32, c->d32, W, c->s.Dp, rows, kFlat, out, st),
             "fitness_check_wide");
    else
        STEP(launch_fitness(c->net32, c->plan_check, c->d32, W, c->s.Dp, rows, kFlat, out, st),
             "fitness_check");
    return MGFWA_OK;
}

hipEvent_t take_event(mgfwa_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Enqueue one generation on `st`; ev (N_EVENTS events) brackets the five phases
// when non-null, ev[6] marks the end of the explosion-fitness GEMM kernel and
// ev[7] its start (after the wide kernel's packing; ev[1] serves otherwise);
// ev[8] and ev[9] bracket the FP32 re-check launch of a BF16 run.
//
// The lag order (Alg. 1 as printed) builds the guiding sparks from the sparks
// and fitness the previous generation left in SE and Yc before exploding, then
// evaluates both kinds of spark in one launch; its explosion phase also holds
// the rank and guide kernels and its guiding-fitness phase is empty.
mgfwa_status enqueue_generation(mgfwa_ctx *c, hipStream_t st, hipEvent_t *ev)
{
    const Shape &s = c->s;
    if (ev) STEP(hipEventRecord(ev[0], st), "event");
    if (s.map_range) STEP(launch_pop_range(s, c->d, st), "pop_range");
    if (s.lag) {
        STEP(launch_rank(s, c->d, st), "rank");
        STEP(launch_guide(s, c->d, st), "guide");
    }
    // wide fitness kernel: the explosion writes the sparks' packed rows (only
    // those when they are regenerated later); regenerating register-chain plans
    // need no explosion launch at all
    const WidePack wp = c->net.wide ? wide_pack_geometry(c->net, c->d) : WidePack{};
    const bool regen_fit = s.regen && !c->net.wide;
    if (!regen_fit)
        STEP(launch_explode(s, c->d, st, c->net.wide ? &wp : nullptr, !s.regen), "explode");
    if (ev) STEP(hipEventRecord(ev[1], st), "event");
    const SparkRegen rg = spark_regen(c);
    mgfwa_status r = fit_rows(c, c->plan_expl, c->d.SE, s.Dp, s.BN * expl_rows(s), expl_map(s),
                              c->d.Yc, st, ev ? ev[6] : nullptr,
                              ev && c->net.wide ? ev[7] : nullptr, c->net.wide ? s.BN * s.lam : 0,
                              regen_fit ? &rg : nullptr);
    if (r) return r;
    if (ev) STEP(hipEventRecord(ev[2], st), "event");
    if (!s.lag) {
        STEP(launch_rank(s, c->d, st), "rank");
        STEP(launch_guide(s, c->d, st), "guide");
    }
    if (ev) STEP(hipEventRecord(ev[3], st), "event");
    if (!s.lag) {
        r = fit_rows(c, c->plan_guide, c->d.SG, s.Dp, s.BN * s.G, OutMap{s.G, s.C, s.lam},
                     c->d.Yc, st);
        if (r) return r;
    }
    if (ev) STEP(hipEventRecord(ev[4], st), "event");
    if (s.recheck) {
        // each firework's best candidate by its BF16 fitness, re-evaluated in FP32
        STEP(launch_gather_best(s, c->d, st), "gather_best");
        if (ev) STEP(hipEventRecord(ev[8], st), "event");
        r = fit_check(c, c->d.Wstar, s.BN, c->d.Ystar, st);
        if (r) return r;
        if (ev) STEP(hipEventRecord(ev[9], st), "event");
    }
    STEP(launch_select(s, c->d, st, s.recheck), "select");
    STEP(launch_apply(s, c->d, st, s.recheck), "apply");
    STEP(launch_finish(c->d, 1, st), "finish");
    if (ev) STEP(hipEventRecord(ev[5], st), "event");
    return MGFWA_OK;
}

mgfwa_status build_graph(mgfwa_ctx *c)
{
    if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    mgfwa_status r = enqueue_generation(c, c->cap, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap, &g);
    if (r != MGFWA_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return fail(MGFWA_EHIP, "graph capture: %s", hipGetErrorString(e));
    c->graph = g;
    HIP_TRY(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    return MGFWA_OK;
}

mgfwa_status reset_ctrl(mgfwa_ctx *c)
{
    // the control words start at zero (a kernel on the stream: no host wait)
    HIP_TRY(launch_clear_ctrl(c->d.ctrl, c->stream));
    return MGFWA_OK;
}

mgfwa_status finish_init(mgfwa_ctx *c)
{
    STEP(launch_init_select(c->s, c->d, c->stream), "init_select");
    STEP(launch_apply(c->s, c->d, c->stream), "apply");
    STEP(launch_finish(c->d, 0, c->stream), "finish");
    return MGFWA_OK;
}

}  // namespace

extern "C" {

size_t mgfwa_workspace_bytes(const mgfwa_config *config, const mgfwa_problem *problem)
{
    Derived dv;
    if (derive(config, problem, &dv) != MGFWA_OK) return 0;
    return dv.lay.total;
}

mgfwa_status mgfwa_init(mgfwa_ctx **out, const mgfwa_config *config, const mgfwa_problem *problem,
                        void *workspace_dev, size_t workspace_bytes, void *hip_stream)
{
    if (!out) return fail(MGFWA_EINVAL, "out is NULL");
    *out = nullptr;
    Derived dv;
    mgfwa_status r = derive(config, problem, &dv);
    if (r != MGFWA_OK) return r;
    if (!hip_stream)
        return fail(MGFWA_EINVAL, "hip_stream is NULL: pass a stream created by the caller "
                                  "(the library never uses the null stream)");
    if (!workspace_dev) return fail(MGFWA_ENOMEM, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace_dev) % ALIGN != 0)
        return fail(MGFWA_ENOMEM, "workspace must be %zu-byte aligned", ALIGN);
    if (workspace_bytes < dv.lay.total)
        return fail(MGFWA_ENOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes,
                    dv.lay.total);
    const bool has_data = !config->external_fitness ||
                          (dv.input ? (const void *)problem->net_dev : (const void *)problem->x_dev);
    FitPlan pi{}, pe{}, pg{}, pv{};
    if (has_data && !dv.input && !dv.net.wide) {
        if (!fit_select(dv.net, dv.s.BN, &pi) || !fit_select(dv.net, dv.s.BN * expl_rows(dv.s), &pe) ||
            !fit_select(dv.net, dv.s.BN * dv.s.G, &pg) ||
            !fit_select(dv.net, dv.lay.partial_rows, &pv))
            return fail(MGFWA_EUNSUPPORTED, "no compiled fitness kernel covers this MLP shape");
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int lds_max = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    dv.net.lds_max = lds_max - 256;   // leave room for the kernels' static LDS
    int num_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    dv.net.num_cu = num_cu > 0 ? num_cu : 1;
    dv.in.num_cu = dv.net.num_cu;
    if (has_data && dv.input) {
        if (net_input_lds_bytes(dv.in) > (size_t)lds_max)
            return fail(MGFWA_EUNSUPPORTED, "device LDS too small for the network's activations");
        HIP_TRY(net_input_prepare(dv.in));
    } else if (has_data && dv.net.wide) {
        if (wide_lds_bytes(dv.net) > lds_max - 64)
            return fail(MGFWA_EUNSUPPORTED, "device LDS too small for the wide fitness kernel");
        HIP_TRY(wide_prepare(dv.net));
    } else if (has_data) {
        if (!fit_select(dv.net, dv.s.BN, &pi) || !fit_select(dv.net, dv.s.BN * expl_rows(dv.s), &pe) ||
            !fit_select(dv.net, dv.s.BN * dv.s.G, &pg) ||
            !fit_select(dv.net, dv.lay.partial_rows, &pv))
            return fail(MGFWA_EUNSUPPORTED, "no compiled fitness kernel covers this MLP shape");
        for (const FitPlan *fp : {&pi, &pe, &pg, &pv}) HIP_TRY(fit_prepare(*fp));
    }
    FitPlan pc{};
    if (dv.s.recheck) {
        dv.net32.lds_max = dv.net.lds_max;
        dv.net32.num_cu = dv.net.num_cu;
        if (dv.net32.wide) {
            if (wide_lds_bytes(dv.net32) > lds_max - 64)
                return fail(MGFWA_EUNSUPPORTED, "device LDS too small for the FP32 wide kernel");
            HIP_TRY(wide_prepare(dv.net32));
        } else {
            if (!fit_select(dv.net32, dv.s.BN, &pc))
                return fail(MGFWA_EUNSUPPORTED, "no compiled FP32 fitness kernel covers this MLP "
                                                "shape (needed to re-check BF16 selections)");
            HIP_TRY(fit_prepare(pc));
        }
    }

    mgfwa_ctx *c = new mgfwa_ctx();
    c->cfg = *config;
    c->s = dv.s;
    c->net = dv.net;
    c->in = dv.in;
    c->input = dv.input;
    c->lay = dv.lay;
    c->has_data = has_data;
    c->ws = static_cast<char *>(workspace_dev);
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->plan_init = pi;
    c->plan_expl = pe;
    c->plan_guide = pg;
    c->plan_eval = pv;
    c->net32 = dv.net32;
    c->plan_check = pc;
    c->s.regen = sparks_regenerated(c) ? 1 : 0;
    const char *ev = std::getenv("MGFWA_NO_GRAPH");
    c->use_graph = !(ev && ev[0] == '1');
    ev = std::getenv("MGFWA_SYNC_DEBUG");
    c->sync_debug = ev && ev[0] == '1';
    const Layout &L = c->lay;
    DevState &d = c->d;
    char *b = c->ws;
    d.F = at<float>(b, L.F);
    d.SE = at<float>(b, L.SE);
    d.SG = at<float>(b, L.SG);
    d.A = at<float>(b, L.A);
    d.Aexp = at<float>(b, L.Aexp);
    d.Y = at<float>(b, L.Y);
    d.Yprev = at<float>(b, L.Yprev);
    d.fresh = at<int32_t>(b, L.fresh);
    d.Yc = at<float>(b, L.Yc);
    d.top = at<int32_t>(b, L.top);
    d.bottom = at<int32_t>(b, L.bottom);
    d.tie = at<int32_t>(b, L.tie);
    d.cstar = at<int32_t>(b, L.cstar);
    d.improved = at<int32_t>(b, L.improved);
    d.reinit = at<int32_t>(b, L.reinit);
    d.src = at<int32_t>(b, L.src);
    d.best_x = at<float>(b, L.best_x);
    d.best_y = at<float>(b, L.best_y);
    d.best_f = at<int32_t>(b, L.best_f);
    d.best_gen = at<int32_t>(b, L.best_gen);
    d.best_upd = at<int32_t>(b, L.best_upd);
    d.ctrl = at<int32_t>(b, L.ctrl);
    d.partial = at<float>(b, L.partial);
    d.Xp = c->net.bf16 ? nullptr : at<float>(b, L.Xp);
    d.Xb = c->net.bf16 ? at<uint16_t>(b, L.Xb) : nullptr;
    d.Ypad = c->net.loss == MGFWA_LOSS_MSE ? at<float>(b, L.Ypad) : nullptr;
    d.Lpad = c->net.loss == MGFWA_LOSS_CE ? at<int32_t>(b, L.Lpad) : nullptr;
    d.Wpack = c->net.wide ? at<char>(b, L.Wpack) : nullptr;
    d.Xw = c->net.wide ? at<char>(b, L.Xw) : nullptr;
    d.lo = c->s.map_range ? at<float>(b, L.lo) : nullptr;
    d.hi = c->s.map_range ? at<float>(b, L.hi) : nullptr;
    d.Pnet = c->input && has_data ? at<float>(b, L.Pnet) : nullptr;
    d.H0 = c->input && has_data ? at<float>(b, L.H0) : nullptr;
    d.H1 = c->input && has_data ? at<float>(b, L.H1) : nullptr;
    d.zero = c->input && has_data ? at<float>(b, L.Zero) : nullptr;
    c->desc_dev = at<JobDesc>(b, L.desc);
    d.Wstar = c->s.recheck ? at<float>(b, L.Wstar) : nullptr;
    d.Ystar = c->s.recheck ? at<float>(b, L.Ystar) : nullptr;
    // the re-check's FP32 view: its own packed samples and spark rows
    c->d32 = d;
    if (c->s.recheck) {
        c->d32.Xb = nullptr;
        c->d32.Xp = c->net32.wide ? nullptr : at<float>(b, L.Xp32);
        c->d32.Wpack = c->net32.wide ? at<char>(b, L.Wpack32) : nullptr;
        c->d32.Xw = c->net32.wide ? at<char>(b, L.Xw32) : nullptr;
    }

    auto bail = [&](mgfwa_status st) {
        mgfwa_destroy(c);
        return st;
    };
    r = reset_ctrl(c);
    if (r) return bail(r);
    if (has_data && c->input) {
        r = check(c, launch_pack_net(c->in, problem->net_dev, d.Pnet, c->stream), "pack_net");
        if (r) return bail(r);
        r = check(c, hipMemsetAsync(d.zero, 0, 256, c->stream), "zero");
        if (r) return bail(r);
    } else if (has_data) {
        r = check(c, launch_pack_problem(c->net, problem->x_dev, problem->y_dev,
                                         problem->labels_dev, d, c->stream), "pack");
        if (r) return bail(r);
        if (c->net.wide) {
            r = check(c, launch_pack_wide_x(c->net, problem->x_dev, d.Xw, c->stream), "pack_x");
            if (r) return bail(r);
            // the explosion writes only the parameters of its packed rows: the
            // padding must read as zero
            r = check(c, hipMemsetAsync(d.Wpack, 0, (size_t)L.partial_rows * wide_row_bytes(c->net),
                                        c->stream), "zero Wpack");
            if (r) return bail(r);
        }
        if (c->s.recheck) {   // FP32 samples of the selection re-check
            r = c->net32.wide
                    ? check(c, launch_pack_wide_x(c->net32, problem->x_dev, c->d32.Xw, c->stream),
                            "pack_x32")
                    : check(c, launch_pack_problem(c->net32, problem->x_dev, problem->y_dev,
                                                   problem->labels_dev, c->d32, c->stream),
                            "pack32");
            if (r) return bail(r);
        }
    }
    r = check(c, launch_init_positions(c->s, d, c->stream), "init_positions");
    if (r) return bail(r);
    if (config->external_fitness) {
        c->phase = PH_INIT_ASK;
    } else {
        // the firework fitness is FP32 in every run (BF16 runs: the re-check's launch)
        r = c->s.recheck ? fit_check(c, d.F, c->s.BN, d.Y, c->stream)
                         : fit_rows(c, c->plan_init, d.F, c->s.Dp, c->s.BN, kFlat, d.Y, c->stream);
        if (r) return bail(r);
        r = finish_init(c);
        if (r) return bail(r);
        c->phase = PH_READY;
    }
    *out = c;
    return MGFWA_OK;
}

mgfwa_status mgfwa_step(mgfwa_ctx *c, int n)
{
    if (!c) return fail(MGFWA_EINVAL, "ctx is NULL");
    if (n < 0) return fail(MGFWA_EINVAL, "n_generations < 0");
    if (c->cfg.external_fitness) return fail(MGFWA_ESTATE, "step needs the built-in fitness");
    if (c->phase != PH_READY) return fail(MGFWA_ESTATE, "an ask/tell exchange is in progress");
    for (int i = 0; i < n; ++i) {
        if (c->timing) {
            std::vector<hipEvent_t> ev(N_EVENTS);
            for (auto &e : ev) {
                e = take_event(c);
                if (!e) return fail(MGFWA_EHIP, "hipEventCreate failed");
            }
            mgfwa_status r = enqueue_generation(c, c->stream, ev.data());
            c->pending.push_back(ev);
            if (r) return r;
        } else if (c->use_graph) {
            if (!c->gexec) {
                mgfwa_status r = build_graph(c);
                if (r) return r;
            }
            HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
        } else {
            mgfwa_status r = enqueue_generation(c, c->stream, nullptr);
            if (r) return r;
        }
        c->gen_host += 1;
    }
    HIP_TRY(hipGetLastError());
    return MGFWA_OK;
}

mgfwa_status mgfwa_best_all(mgfwa_ctx *c, float *x_host, float *f_host, int32_t *gen_host)
{
    if (!c) return fail(MGFWA_EINVAL, "ctx is NULL");
    const int B = c->s.B;
    if (f_host)
        HIP_TRY(hipMemcpyAsync(f_host, c->d.best_y, B * 4, hipMemcpyDeviceToHost, c->stream));
    if (gen_host)
        HIP_TRY(hipMemcpyAsync(gen_host, c->d.best_gen, B * 4, hipMemcpyDeviceToHost, c->stream));
    if (x_host)
        HIP_TRY(hipMemcpy2DAsync(x_host, (size_t)c->s.D * 4, c->d.best_x, (size_t)c->s.Dp * 4,
                                 (size_t)c->s.D * 4, B, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MGFWA_OK;
}

mgfwa_status mgfwa_best(mgfwa_ctx *c, float *x_host, float *f_host, int *generation)
{
    if (!c) return fail(MGFWA_EINVAL, "ctx is NULL");
    const int B = c->s.B;
    std::vector<float> by(B);
    int32_t ctrl[CTRL_WORDS];
    HIP_TRY(hipMemcpyAsync(by.data(), c->d.best_y, B * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(ctrl, c->d.ctrl, sizeof ctrl, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    int pb = 0;
    for (int b = 1; b < B; ++b)
        if (by[b] < by[pb]) pb = b;
    if (f_host) *f_host = by[pb];
    if (generation) *generation = ctrl[CTRL_GEN];
    if (x_host) {
        HIP_TRY(hipMemcpyAsync(x_host, c->d.best_x + (size_t)pb * c->s.Dp, (size_t)c->s.D * 4,
                               hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return MGFWA_OK;
}

mgfwa_status mgfwa_ask(mgfwa_ctx *c, const float **sparks, int *rows, int *ld)
{
    if (!c || !sparks) return fail(MGFWA_EINVAL, "NULL argument");
    const Shape &s = c->s;
    if (s.lag) return fail(MGFWA_EUNSUPPORTED, "the lagged guiding order has no ask/tell form");
    switch (c->phase) {
    case PH_INIT_ASK:
        *sparks = c->d.F;
        if (rows) *rows = s.BN;
        c->phase = PH_INIT_TELL;
        break;
    case PH_READY:
        if (s.map_range) STEP(launch_pop_range(s, c->d, c->stream), "pop_range");
        STEP(launch_explode(s, c->d, c->stream), "explode");
        *sparks = c->d.SE;
        if (rows) *rows = s.BN * s.lam;
        c->phase = PH_EXPL_TELL;
        break;
    case PH_GUIDE_ASK:
        *sparks = c->d.SG;
        if (rows) *rows = s.BN * s.G;
        c->phase = PH_GUIDE_TELL;
        break;
    default:
        return fail(MGFWA_ESTATE, "ask while a tell is expected");
    }
    if (ld) *ld = s.Dp;
    return MGFWA_OK;
}

mgfwa_status mgfwa_tell(mgfwa_ctx *c, const float *fit)
{
    if (!c || !fit) return fail(MGFWA_EINVAL, "NULL argument");
    const Shape &s = c->s;
    switch (c->phase) {
    case PH_INIT_TELL: {
        STEP(launch_store_fitness(fit, s.BN, kFlat, c->d.Y, nullptr, c->stream), "store");
        mgfwa_status r = finish_init(c);
        if (r) return r;
        c->phase = PH_READY;
        break;
    }
    case PH_EXPL_TELL:
        STEP(launch_store_fitness(fit, s.BN * s.lam, OutMap{s.lam, s.C, 0}, c->d.Yc, c->d.ctrl,
                                  c->stream), "store");
        STEP(launch_rank(s, c->d, c->stream), "rank");
        STEP(launch_guide(s, c->d, c->stream), "guide");
        c->phase = PH_GUIDE_ASK;
        break;
    case PH_GUIDE_TELL:
        STEP(launch_store_fitness(fit, s.BN * s.G, OutMap{s.G, s.C, s.lam}, c->d.Yc, c->d.ctrl,
                                  c->stream), "store");
        STEP(launch_select(s, c->d, c->stream), "select");
        STEP(launch_apply(s, c->d, c->stream), "apply");
        STEP(launch_finish(c->d, 1, c->stream), "finish");
        c->phase = PH_READY;
        c->gen_host += 1;
        break;
    default:
        return fail(MGFWA_ESTATE, "tell without a matching ask");
    }
    return MGFWA_OK;
}

mgfwa_status mgfwa_evaluate(mgfwa_ctx *c, const float *w, int rows, int ld, float *out)
{
    if (!c) return fail(MGFWA_EINVAL, "ctx is NULL");
    if (!c->has_data) return fail(MGFWA_EINVAL, "context has no problem data to evaluate");
    if (rows < 0 || (rows > 0 && (!w || !out))) return fail(MGFWA_EINVAL, "bad rows/buffers");
    if (ld < c->s.D || ld % 4 != 0 || reinterpret_cast<uintptr_t>(w) % 16 != 0)
        return fail(MGFWA_EINVAL, "ld must be >= D and a multiple of 4; w 16-byte aligned");
    // the kernels stage per-row partial sums (weights problems) or activations
    // (input problems) in buffers of partial_rows rows
    const int chunk = c->lay.partial_rows;
    for (int r0 = 0; r0 < rows; r0 += chunk) {
        const int nr = std::min(chunk, rows - r0);
        FitPlan plan{};
        if (!c->net.wide && !c->input) {
            if (!fit_select(c->net, nr, &plan))
                return fail(MGFWA_EUNSUPPORTED, "no compiled fitness kernel covers this MLP shape");
            HIP_TRY(fit_prepare(plan));
        }
        mgfwa_status r = fit_rows(c, plan, w + (size_t)r0 * ld, (size_t)ld, nr, kFlat, out + r0,
                                  c->stream);
        if (r) return r;
    }
    return MGFWA_OK;
}

mgfwa_status mgfwa_state(const mgfwa_ctx *c, mgfwa_state_info *info)
{
    if (!c || !info) return fail(MGFWA_EINVAL, "NULL argument");
    const Layout &L = c->lay;
    info->D = c->s.D;
    info->Dp = c->s.Dp;
    info->m = c->s.m;
    info->k = c->s.k;
    info->n_candidates = c->s.C;
    info->generation = c->gen_host;
    info->F = L.F;
    info->A = L.A;
    info->Y = L.Y;
    info->Yprev = L.Yprev;
    info->fresh = L.fresh;
    info->SE = L.SE;
    info->SG = L.SG;
    info->Yc = L.Yc;
    info->top = L.top;
    info->bottom = L.bottom;
    info->tie = L.tie;
    info->cstar = L.cstar;
    info->improved = L.improved;
    info->reinit = L.reinit;
    info->best_x = L.best_x;
    info->best_y = L.best_y;
    info->best_f = L.best_f;
    info->best_gen = L.best_gen;
    info->gen = L.ctrl + CTRL_GEN * 4;
    info->done = L.ctrl + CTRL_DONE * 4;
    info->se_written = c->s.regen ? 0 : 1;
    return MGFWA_OK;
}

mgfwa_status mgfwa_set_timing(mgfwa_ctx *c, int on)
{
    if (!c) return fail(MGFWA_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto &ev : c->pending)
        for (hipEvent_t e : ev) c->pool.push_back(e);
    c->pending.clear();
    c->gen_ms.clear();
    for (double &v : c->phase_ms) v = 0.0;
    c->fit_kernel_ms = 0.0;
    c->check_ms = 0.0;
    c->timing = on != 0;
    return MGFWA_OK;
}

mgfwa_status mgfwa_timing(mgfwa_ctx *c, mgfwa_timing_info *info)
{
    if (!c || !info) return fail(MGFWA_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto &ev : c->pending) {
        float ms = 0.0f;
        for (int p = 0; p < MGFWA_N_PHASES; ++p) {
            HIP_TRY(hipEventElapsedTime(&ms, ev[p], ev[p + 1]));
            c->phase_ms[p] += ms;
        }
        HIP_TRY(hipEventElapsedTime(&ms, c->net.wide ? ev[7] : ev[1], ev[6]));
        c->fit_kernel_ms += ms;
        if (c->s.recheck) {
            HIP_TRY(hipEventElapsedTime(&ms, ev[8], ev[9]));
            c->check_ms += ms;
        }
        HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[MGFWA_N_PHASES]));
        c->gen_ms.push_back(ms);
        for (hipEvent_t e : ev) c->pool.push_back(e);
    }
    c->pending.clear();
    for (int p = 0; p < MGFWA_N_PHASES; ++p) info->ms[p] = c->phase_ms[p];
    info->fit_kernel_ms = c->fit_kernel_ms;
    info->check_fit_ms = c->check_ms;
    info->generations = (int)c->gen_ms.size();
    info->gen_ms_p50 = info->gen_ms_p99 = info->gen_ms_mean = 0.0;
    if (!c->gen_ms.empty()) {
        std::vector<double> v = c->gen_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            size_t i = (size_t)std::ceil(q * v.size()) - 1;
            return v[std::min(i, v.size() - 1)];
        };
        info->gen_ms_p50 = pct(0.50);
        info->gen_ms_p99 = pct(0.99);
        double s = 0.0;
        for (double x : v) s += x;
        info->gen_ms_mean = s / v.size();
    }
    return MGFWA_OK;
}

void mgfwa_destroy(mgfwa_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    for (auto &ev : c->pending)
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"

// ---- fitness without a workspace --------------------------------------------
namespace {

// Device scratch of mgfwa_evaluate_noalloc: a file-scope device array, so every
// device the library runs on holds its own copy until the process ends.  In host
// code its name is only a stand-in: kernels get the per-device address that
// hipGetSymbolAddress returns.
__device__ __align__(256) char scratch[MGFWA_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[MAX_DEVICES] = {};

// Address of the current device's scratch, looked up on its first use there.
mgfwa_status scratch_address(int dev, char **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(MGFWA_EHIP, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MGFWA_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch[dev] = static_cast<char *>(p);
    }
    *out = g_scratch[dev];
    return MGFWA_OK;
}

}  // namespace

extern "C" mgfwa_status mgfwa_evaluate_noalloc(const mgfwa_problem *problem, int precision,
                                               const float *w, int rows, int ld, float *out,
                                               void *hip_stream)
{
    if (!problem) return fail(MGFWA_EINVAL, "problem is NULL");
    if (!hip_stream)
        return fail(MGFWA_EINVAL, "hip_stream is NULL: pass a stream created by the caller");
    if (problem->kind != MGFWA_PROBLEM_WEIGHTS)
        return fail(MGFWA_EUNSUPPORTED, "mgfwa_evaluate_noalloc takes weights problems only");
    // the network as a context of this problem would see it (one firework)
    mgfwa_config cfg{};
    cfg.n_populations = cfg.n_fireworks = cfg.n_guiding = 1;
    cfg.n_sparks = 2;
    cfg.sigma = 0.5f;
    cfg.boost = cfg.amp_up = cfg.amp_down = 1.0f;
    cfg.lb = -1.0f;
    cfg.ub = 1.0f;
    cfg.max_generations = 1;
    cfg.precision = precision;
    Derived dv;
    mgfwa_status r = derive(&cfg, problem, &dv);
    if (r != MGFWA_OK) return r;
    const Net &n0 = dv.net;
    if (rows < 0 || (rows > 0 && (!w || !out))) return fail(MGFWA_EINVAL, "bad rows/buffers");
    if (ld < dv.s.D || ld % 4 != 0 || reinterpret_cast<uintptr_t>(w) % 16 != 0)
        return fail(MGFWA_EINVAL, "ld must be >= D and a multiple of 4; w 16-byte aligned");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int lds_max = 0, num_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    HIP_TRY(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    Net net = n0;
    net.lds_max = lds_max - 256;
    net.num_cu = num_cu > 0 ? num_cu : 1;
    // scratch layout: packed samples, targets or labels, then per chunk of rows
    // the partial sums (and the wide kernel's packed rows)
    const size_t es = net.bf16 ? 2 : 4;
    const int outw = net.fo[net.nl - 1];
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, ALIGN);
        return o;
    };
    const size_t oX = take(net.wide ? 0 : (size_t)net.S_pad * net.in_pad * es);
    const size_t oXw = take(net.wide ? (size_t)net.S_pad * wide_kp(net) * es : 0);
    const size_t oY = take(net.loss == MGFWA_LOSS_MSE ? (size_t)net.S_pad * outw * 4 : 0);
    const size_t oL = take(net.loss == MGFWA_LOSS_CE ? (size_t)net.S_pad * 4 : 0);
    const size_t fixed = off;
    const size_t per_row = net.wide ? wide_row_bytes(net) + (size_t)(net.S_pad / 256) * 4
                                    : (size_t)fit_max_bpr() * 4;
    const size_t cap = MGFWA_NOALLOC_SCRATCH_BYTES;
    if (fixed + per_row + 2 * ALIGN > cap)
        return fail(MGFWA_EINVAL, "problem too large for the %zu-byte no-allocation scratch "
                                  "(packed samples need %zu bytes, one row %zu)", cap, fixed, per_row);
    // rows per launch: what fits, and no more than mgfwa_evaluate takes at once
    const int chunk = (int)std::min<size_t>((cap - fixed - 2 * ALIGN) / per_row, 1024);
    const size_t oP = take((size_t)chunk * (net.wide ? (size_t)(net.S_pad / 256) * 4
                                                     : (size_t)fit_max_bpr() * 4));
    const size_t oW = take(net.wide ? (size_t)chunk * wide_row_bytes(net) : 0);
    if (off > cap) return fail(MGFWA_EINVAL, "internal: no-allocation scratch layout overflows");
    if (rows == 0) return MGFWA_OK;
    char *base = nullptr;
    r = scratch_address(dev, &base);
    if (r != MGFWA_OK) return r;
    if (net.wide) {
        if (wide_lds_bytes(net) > lds_max - 64)
            return fail(MGFWA_EUNSUPPORTED, "device LDS too small for the wide fitness kernel");
        HIP_TRY(wide_prepare(net));
    }
    DevState d{};
    d.Xp = !net.wide && !net.bf16 ? at<float>(base, oX) : nullptr;
    d.Xb = !net.wide && net.bf16 ? at<uint16_t>(base, oX) : nullptr;
    d.Xw = net.wide ? at<char>(base, oXw) : nullptr;
    d.Ypad = net.loss == MGFWA_LOSS_MSE ? at<float>(base, oY) : nullptr;
    d.Lpad = net.loss == MGFWA_LOSS_CE ? at<int32_t>(base, oL) : nullptr;
    d.partial = at<float>(base, oP);
    d.Wpack = net.wide ? at<char>(base, oW) : nullptr;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // the array keeps the previous call's contents: every byte a launch reads is
    // rewritten here first (samples, targets, labels and their padding by the
    // packing kernels; packed rows and partial sums by the fitness launch)
    HIP_TRY(launch_pack_problem(net, problem->x_dev, problem->y_dev, problem->labels_dev, d, st));
    if (net.wide) HIP_TRY(launch_pack_wide_x(net, problem->x_dev, d.Xw, st));
    for (int r0 = 0; r0 < rows; r0 += chunk) {
        const int nr = std::min(chunk, rows - r0);
        const float *wr = w + (size_t)r0 * ld;
        if (net.wide) {
            HIP_TRY(launch_fitness_wide(net, d, wr, (size_t)ld, nr, kFlat, out + r0, st));
        } else {
            FitPlan plan{};
            if (!fit_select(net, nr, &plan))
                return fail(MGFWA_EUNSUPPORTED, "no compiled fitness kernel covers this MLP shape");
            HIP_TRY(fit_prepare(plan));
            HIP_TRY(launch_fitness(net, plan, d, wr, (size_t)ld, nr, kFlat, out + r0, st));
        }
    }
    return MGFWA_OK;
}

// ---- autotuning ------------------------------------------------------------
namespace {

std::mutex g_tune_mu;
std::map<std::string, FitPlan> g_tune;   // shape key -> timed choice, for the process
constexpr int MAX_CANDIDATES = 64;

std::string tune_key(const Net &net, int rows)
{
    std::string k = "p" + std::to_string(net.bf16) + " S" + std::to_string(net.S) + " L" +
                    std::to_string(net.loss) + " r" + std::to_string(rows);
    for (int l = 0; l < net.nl; ++l)
        k += " " + std::to_string(net.fi[l]) + "x" + std::to_string(net.fo[l]) + "a" +
             std::to_string(net.act[l]);
    return k;
}

std::string tune_key_input(const InNet &in, int rows)
{
    std::string k = "in r" + std::to_string(rows);
    for (int l = 0; l < in.nl; ++l)
        k += " " + std::to_string(in.fi[l]) + "x" + std::to_string(in.fo[l]) + "a" +
             std::to_string(in.act[l]);
    return k;
}

// Candidate launches of a problem: the compiled fitness kernels that cover the
// weights problem's shape, or the tile shapes of the input problem's kernels.
int tune_candidates(const mgfwa_ctx *c, int rows, FitPlan *cand, int max_out)
{
    if (!c->input) return fit_candidates(c->net, rows, cand, max_out);
    int n = 0;
    for (int shape = 0; shape <= NET_LDS64 && n < max_out; ++shape) {
        cand[n] = FitPlan{};
        cand[n].rows = rows;
        cand[n].net_shape = shape;
        ++n;
    }
    return n;
}

// Sparks per launch of fitness launch `which` (0 explosion, 1 guiding sparks,
// 2 the FP32 re-check of a BF16 run's winners).
int launch_rows(const mgfwa_ctx *c, int which)
{
    return which == 0 ? c->s.BN * expl_rows(c->s) : which == 1 ? c->s.BN * c->s.G : c->s.BN;
}

// The network (precision) and the plan of fitness launch `which`.
const Net &launch_net(const mgfwa_ctx *c, int which) { return which == 2 ? c->net32 : c->net; }
FitPlan &launch_plan(mgfwa_ctx *c, int which)
{
    return which == 0 ? c->plan_expl : which == 1 ? c->plan_guide : c->plan_check;
}
const FitPlan &launch_plan(const mgfwa_ctx *c, int which)
{
    return launch_plan(const_cast<mgfwa_ctx *>(c), which);
}

// `which` names a fitness launch the context has (EINVAL / ESTATE otherwise).
mgfwa_status check_which(const mgfwa_ctx *c, int which)
{
    if (which < 0 || which > 2) return fail(MGFWA_EINVAL, "which must be 0, 1 or 2");
    if (which == 2 && !c->s.recheck)
        return fail(MGFWA_ESTATE, "no re-check launch: the context has no BF16 built-in fitness");
    return MGFWA_OK;
}

void fill_plan_info(const mgfwa_ctx *c, const FitPlan &p, int rows, mgfwa_plan_info *info,
                    int which = 0)
{
    const Net &net = launch_net(c, which);
    std::memset(info, 0, sizeof *info);
    info->wide = net.wide ? 1 : 0;
    info->rows = rows;
    info->net_kernel = c->input ? p.net_shape : -1;
    if (!net.wide && !c->input) {
        info->wavefronts = p.nw;
        info->slabs = p.P;
        info->lds_weights = p.wl;
        info->blocks_per_row = p.bpr;
        info->samples_per_block = p.spb;
        info->lds_bytes = p.lds_bytes;
        for (int l = 0; l < MAXL; ++l) info->row_blocks[l] = p.lrows[l] / 16;
    }
}

// Time every candidate plan for `rows` sparks of W on the context's stream and
// keep the fastest; a shape seen before reuses its choice without timing.
// check: the launch is the FP32 re-check of a BF16 run's winners (the FP32
// network and sample buffers, results into the re-check's output).
mgfwa_status tune_plan(mgfwa_ctx *c, int rows, const float *W, OutMap map, int reps, FitPlan *out,
                       bool check = false)
{
    const Net &net = check ? c->net32 : c->net;
    const DevState &dv = check ? c->d32 : c->d;
    float *res = check ? c->d.Ystar : c->d.Yc;
    const std::string key = c->input ? tune_key_input(c->in, rows) : tune_key(net, rows);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *out = it->second;
            HIP_TRY(fit_prepare(*out));
            return MGFWA_OK;
        }
    }
    FitPlan cand[MAX_CANDIDATES];
    const int n = check ? fit_candidates(net, rows, cand, MAX_CANDIDATES)
                        : tune_candidates(c, rows, cand, MAX_CANDIDATES);
    if (n == 0) return fail(MGFWA_EUNSUPPORTED, "no compiled fitness kernel covers this MLP shape");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int best = -1;
    float best_ms = 0.0f;
    mgfwa_status r = MGFWA_OK;
    for (int i = 0; i < n && r == MGFWA_OK; ++i) {
        hipError_t e = fit_prepare(cand[i]);
        for (int k = 0; k <= reps && e == hipSuccess; ++k) {
            if (k == 1) e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess)
                e = c->input ? launch_net_input(c->in, cand[i].net_shape, c->d.Pnet, W, c->s.Dp, rows,
                                                map, c->d.Yc, c->d.H0, c->d.H1, c->d.zero, c->stream)
                             : launch_fitness(net, cand[i], dv, W, c->s.Dp, rows, map, res, c->stream);
        }
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            r = fail(MGFWA_EHIP, "autotune: %s", hipGetErrorString(e));
            break;
        }
        if (best < 0 || ms < best_ms) {
            best = i;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != MGFWA_OK) return r;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto ins = g_tune.emplace(key, cand[best]);   // a concurrent tuner may have won
        *out = ins.first->second;
    }
    HIP_TRY(fit_prepare(*out));
    return MGFWA_OK;
}

}  // namespace

// ---- batched generations -----------------------------------------------------
struct mgfwa_batch {
    std::vector<mgfwa_ctx *> jobs;
    hipStream_t stream = nullptr;            // launch stream (caller's)
    hipStream_t cap = nullptr;               // capture origin
    std::vector<hipStream_t> branch;         // capture branches
    std::vector<hipEvent_t> ev;              // fork and joins of the capture
    std::vector<hipEvent_t> job_ev;          // per job: its own stream's queued work
    hipEvent_t done = nullptr;               // end of the last batch step
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<int> grouped, solo;          // jobs run by grouped launches / as branches
    std::vector<JobDesc> desc;               // host copies of the grouped jobs' descriptors
    std::vector<hipStream_t> fit_branch;     // capture branches of the grouped fitness launches
};

void mgfwa::group_table(const JobDesc *const *jobs, const dim3 *grid, int n, GroupTable *t)
{
    int acc = 0;
    t->njobs = n;
    for (int i = 0; i < n; ++i) {
        t->start[i] = acc;
        t->gx[i] = (int)grid[i].x;
        t->gy[i] = (int)grid[i].y;
        t->job[i] = jobs[i];
        acc += (int)((grid[i].x * grid[i].y + GROUP_ALIGN - 1) / GROUP_ALIGN * GROUP_ALIGN);
    }
    t->start[n] = acc;
}

namespace {

constexpr int MAX_BRANCHES = 16;
constexpr int MAX_FIT_BRANCHES = 8;   // parallel grouped fitness launches (kernel instances)

// Jobs whose whole generation runs as grouped launches: weights problems on the
// register-chain kernels in the default order.  (The wide kernel is persistent
// over the device already; input problems and the lag order keep their own
// sequences as graph branches.)
bool groupable(const mgfwa_ctx *c)
{
    return !c->input && c->has_data && !c->net.wide && !c->s.lag && !c->cfg.external_fitness;
}

// Fitness FLOPs of one generation of a job (every candidate over every sample).
double job_flops(const mgfwa_ctx *c)
{
    double per = 0.0;
    for (int l = 0; l < c->net.nl; ++l) per += (double)c->net.fi[l] * c->net.fo[l];
    return 2.0 * c->net.S * per * c->s.BN * (c->s.lam + c->s.G);
}

// Jobs whose generation is short enough that launches dominate it run as
// grouped launches (one launch per kernel for all of them); larger jobs keep
// their own kernel sequence on a graph branch, where the jobs' phases overlap
// instead of every job waiting for the slowest one at each phase.  Measured
// with 64 BF16 jobs of 1-142 GFLOP per generation: all grouped 6.8 ms, all on
// branches 6.1 ms, grouped up to 1 / 4 / 16 GFLOP 5.9 / 6.0 / 6.4 ms; with 64
// jobs of 10 MFLOP: grouped 0.31 ms, on branches 1.9 ms.
constexpr double GROUP_MAX_FLOPS = 1e9;

JobDesc job_desc(const mgfwa_ctx *c)
{
    JobDesc j;
    std::memset(&j, 0, sizeof j);
    const Shape &s = c->s;
    j.s = s;
    j.d = c->d;
    const SparkRegen rg = spark_regen(c);
    j.fit[0] = fit_launch_args(c->net, c->plan_expl, c->d, c->d.SE, s.Dp, s.BN * s.lam, expl_map(s),
                               c->d.Yc, s.regen ? &rg : nullptr);
    j.fit[1] = fit_launch_args(c->net, c->plan_guide, c->d, c->d.SG, s.Dp, s.BN * s.G,
                               OutMap{s.G, s.C, s.lam}, c->d.Yc);
    if (s.recheck)
        j.fit[2] = fit_launch_args(c->net32, c->plan_check, c->d32, c->d.Wstar, s.Dp, s.BN, kFlat,
                                   c->d.Ystar);
    return j;
}

const FitPlan &job_plan(const mgfwa_ctx *c, int which) { return launch_plan(c, which); }

// Sparks of fitness launch `which` of a grouped job (as in job_desc).
int job_fit_rows(const mgfwa_ctx *c, int which)
{
    return which == 0 ? c->s.BN * c->s.lam : which == 1 ? c->s.BN * c->s.G : c->s.BN;
}

// One grouped launch per GROUP_MAX jobs among the grouped jobs that `take` selects,
// each with its own grid from `grid`.
template <class Take, class Grid, class Launch>
mgfwa_status group_run(mgfwa_batch *b, Take take, Grid grid, Launch launch)
{
    std::vector<const JobDesc *> jd;
    std::vector<dim3> gr;
    for (int i : b->grouped) {
        const mgfwa_ctx *c = b->jobs[i];
        if (!take(c)) continue;
        const dim3 g = grid(c);
        if (g.x * g.y == 0) continue;
        jd.push_back(c->desc_dev);
        gr.push_back(g);
    }
    for (size_t o = 0; o < jd.size(); o += GROUP_MAX) {
        const int m = (int)std::min<size_t>(GROUP_MAX, jd.size() - o);
        GroupTable t;
        group_table(jd.data() + o, gr.data() + o, m, &t);
        const hipError_t e = launch(t);
        if (e != hipSuccess) return fail(MGFWA_EHIP, "grouped launch: %s", hipGetErrorString(e));
    }
    return MGFWA_OK;
}

hipEvent_t batch_event(mgfwa_batch *b);

// Fitness launch `which` of the grouped jobs: one grouped launch per kernel
// instance, the instances on parallel branches of the graph (they touch
// different jobs), then one grouped finalisation.
mgfwa_status group_fitness(mgfwa_batch *b, int which, bool (*take)(const mgfwa_ctx *),
                           hipStream_t st)
{
    std::vector<const void *> kernels;
    for (int i : b->grouped) {
        const mgfwa_ctx *c = b->jobs[i];
        if (!take(c)) continue;
        const void *k = job_plan(c, which).gkernel;
        if (std::find(kernels.begin(), kernels.end(), k) == kernels.end()) kernels.push_back(k);
    }
    const int nbr = std::min((int)kernels.size(), (int)b->fit_branch.size());
    hipEvent_t fork = nullptr;
    if (nbr > 1) {
        fork = batch_event(b);
        if (!fork) return fail(MGFWA_EHIP, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(fork, st));
        for (int i = 0; i < nbr; ++i) HIP_TRY(hipStreamWaitEvent(b->fit_branch[i], fork, 0));
    }
    for (size_t ik = 0; ik < kernels.size(); ++ik) {
        const void *k = kernels[ik];
        hipStream_t ks = nbr > 1 ? b->fit_branch[ik % nbr] : st;
        int lds = 0, nw = 0;
        for (int i : b->grouped) {
            const mgfwa_ctx *c = b->jobs[i];
            if (!take(c) || job_plan(c, which).gkernel != k) continue;
            lds = std::max(lds, job_plan(c, which).lds_bytes);
            nw = job_plan(c, which).nw;
        }
        mgfwa_status r = group_run(
            b, [&](const mgfwa_ctx *c) { return take(c) && job_plan(c, which).gkernel == k; },
            [&](const mgfwa_ctx *c) {
                return dim3((unsigned)(job_fit_rows(c, which) * job_plan(c, which).bpr));
            },
            [&](const GroupTable &t) { return launch_fitness_group(t, k, nw, lds, which, ks); });
        if (r) return r;
    }
    for (int i = 0; i < nbr && nbr > 1; ++i) {
        hipEvent_t join = batch_event(b);
        if (!join) return fail(MGFWA_EHIP, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(join, b->fit_branch[i]));
        HIP_TRY(hipStreamWaitEvent(st, join, 0));
    }
    return group_run(
        b, take,
        [&](const mgfwa_ctx *c) { return dim3((unsigned)((job_fit_rows(c, which) + 255) / 256)); },
        [&](const GroupTable &t) { return launch_finalize_group(t, which, st); });
}

bool take_all(const mgfwa_ctx *) { return true; }
bool take_recheck(const mgfwa_ctx *c) { return c->s.recheck != 0; }

// One generation of every grouped job as grouped launches, in the order of
// enqueue_generation (default order, register-chain kernels).
mgfwa_status enqueue_grouped(mgfwa_batch *b, hipStream_t st)
{
    mgfwa_status r = group_run(
        b, [](const mgfwa_ctx *c) { return c->s.map_range != 0; },
        [](const mgfwa_ctx *c) { return pop_range_grid(c->s); },
        [&](const GroupTable &t) { return launch_pop_range_group(t, st); });
    if (!r)
        r = group_run(
            b, [](const mgfwa_ctx *c) { return c->s.regen == 0; },
            [](const mgfwa_ctx *c) { return explode_grid(c->s); },
            [&](const GroupTable &t) { return launch_explode_group(t, st); });
    if (!r) r = group_fitness(b, 0, take_all, st);
    int max_lam = 0;
    for (int i : b->grouped) max_lam = std::max(max_lam, b->jobs[i]->s.lam);
    if (!r)
        r = group_run(
            b, [](const mgfwa_ctx *c) { return c->s.m > 64; },
            [](const mgfwa_ctx *c) { return rank_grid(c->s); },
            [&](const GroupTable &t) { return launch_rank_group(t, max_lam, st); });
    if (!r)
        r = group_run(
            b, take_all, [](const mgfwa_ctx *c) { return guide_grid(c->s); },
            [&](const GroupTable &t) { return launch_guide_group(t, st); });
    if (!r) r = group_fitness(b, 1, take_all, st);
    if (!r)
        r = group_run(
            b, take_recheck, [](const mgfwa_ctx *c) { return firework_row_grid(c->s); },
            [&](const GroupTable &t) { return launch_gather_best_group(t, st); });
    if (!r) r = group_fitness(b, 2, take_recheck, st);
    if (!r)
        r = group_run(
            b, take_all, [](const mgfwa_ctx *c) { return select_grid(c->s); },
            [&](const GroupTable &t) { return launch_select_group(t, st); });
    if (!r)
        r = group_run(
            b, take_all, [](const mgfwa_ctx *c) { return firework_row_grid(c->s); },
            [&](const GroupTable &t) { return launch_apply_group(t, st); });
    if (!r)
        r = group_run(
            b, take_all, [](const mgfwa_ctx *) { return dim3(1); },
            [&](const GroupTable &t) { return launch_finish_group(t, st); });
    return r;
}

// Descriptors of the grouped jobs written to their workspaces (on each job's
// stream, which the batch orders itself after), and the LDS limits of the
// grouped fitness kernels raised to what their jobs need.
mgfwa_status group_setup(mgfwa_batch *b)
{
    for (int i = 0; i < (int)b->jobs.size(); ++i)
        (groupable(b->jobs[i]) && job_flops(b->jobs[i]) <= GROUP_MAX_FLOPS ? b->grouped : b->solo)
            .push_back(i);
    for (int i = 0; i < MAX_FIT_BRANCHES && !b->grouped.empty(); ++i) {
        hipStream_t st = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        b->fit_branch.push_back(st);
    }
    b->desc.resize(b->grouped.size());
    for (size_t k = 0; k < b->grouped.size(); ++k) {
        mgfwa_ctx *c = b->jobs[b->grouped[k]];
        b->desc[k] = job_desc(c);
        HIP_TRY(hipMemcpyAsync(c->desc_dev, &b->desc[k], sizeof(JobDesc), hipMemcpyHostToDevice,
                               c->stream));
    }
    std::map<const void *, int> lds;   // grouped kernel -> the most LDS any of its launches takes
    for (int i : b->grouped) {
        const mgfwa_ctx *c = b->jobs[i];
        for (int which = 0; which < (c->s.recheck ? 3 : 2); ++which) {
            const FitPlan &p = job_plan(c, which);
            int &v = lds[p.gkernel];
            v = std::max(v, p.lds_bytes);
        }
    }
    for (const auto &kv : lds) HIP_TRY(fit_group_prepare(kv.first, kv.second));
    return MGFWA_OK;
}


hipEvent_t batch_event(mgfwa_batch *b)
{
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    b->ev.push_back(e);
    return e;
}

mgfwa_status batch_capture(mgfwa_batch *b)
{
    mgfwa_status r0 = group_setup(b);
    if (r0) return r0;
    const int n = (int)b->solo.size();
    const int nb = std::min(n, MAX_BRANCHES);
    HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    for (int i = 0; i < nb; ++i) {
        hipStream_t st = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        b->branch.push_back(st);
    }
    std::vector<hipEvent_t> join(nb);
    hipEvent_t fork = batch_event(b);
    for (auto &e : join) e = batch_event(b);
    if (!fork || std::find(join.begin(), join.end(), nullptr) != join.end())
        return fail(MGFWA_EHIP, "hipEventCreate failed");
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    mgfwa_status r = MGFWA_OK;
    hipError_t e = hipEventRecord(fork, b->cap);
    for (int i = 0; i < nb && e == hipSuccess; ++i) e = hipStreamWaitEvent(b->branch[i], fork, 0);
    if (e != hipSuccess) r = fail(MGFWA_EHIP, "batch capture: %s", hipGetErrorString(e));
    // branch jobs, largest first, each to the branch with the least work so far
    // (a branch runs its jobs in order); the grouped jobs' generation is one
    // sequence of grouped launches on the capture stream, beside them
    std::vector<int> order(b->solo);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return job_flops(b->jobs[x]) > job_flops(b->jobs[y]);
    });
    std::vector<double> load(nb, 0.0);
    for (size_t k = 0; k < order.size() && r == MGFWA_OK; ++k) {
        const int br = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[br] += job_flops(b->jobs[order[k]]);
        r = enqueue_generation(b->jobs[order[k]], b->branch[br], nullptr);
    }
    if (r == MGFWA_OK && !b->grouped.empty()) r = enqueue_grouped(b, b->cap);
    for (int i = 0; i < nb && r == MGFWA_OK; ++i) {
        e = hipEventRecord(join[i], b->branch[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, join[i], 0);
        if (e != hipSuccess) r = fail(MGFWA_EHIP, "batch capture: %s", hipGetErrorString(e));
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (r != MGFWA_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return fail(MGFWA_EHIP, "batch capture: %s", hipGetErrorString(e));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    return MGFWA_OK;
}

}  // namespace

extern "C" {

mgfwa_status mgfwa_autotune(mgfwa_ctx *c, int reps)
{
    if (!c) return fail(MGFWA_EINVAL, "ctx is NULL");
    if (reps < 1 || reps > 1000) return fail(MGFWA_EINVAL, "reps must be in [1, 1000]");
    if (c->cfg.external_fitness || !c->has_data)
        return fail(MGFWA_ESTATE, "autotuning needs the built-in fitness");
    if (c->phase != PH_READY || c->gen_host != 0 || c->gexec)
        return fail(MGFWA_ESTATE, "autotune before the first generation");
    if (c->net.wide) return MGFWA_OK;   // one fixed tile shape
    const Shape &s = c->s;
    mgfwa_status r = tune_plan(c, s.BN * expl_rows(s), c->d.SE, expl_map(s), reps, &c->plan_expl);
    if (r) return r;
    c->s.regen = sparks_regenerated(c) ? 1 : 0;   // the plan decides whether it can regenerate
    r = tune_plan(c, s.BN * s.G, c->d.SG, OutMap{s.G, s.C, s.lam}, reps, &c->plan_guide);
    if (r || !s.recheck || c->net32.wide) return r;
    // the FP32 re-check of the B*N winners (timed on the firework rows, whose
    // FP32 fitness the initialisation computed with the same launch)
    return tune_plan(c, s.BN, c->d.F, kFlat, reps, &c->plan_check, true);
}

mgfwa_status mgfwa_fit_plan(const mgfwa_ctx *c, int which, mgfwa_plan_info *info)
{
    if (!c || !info) return fail(MGFWA_EINVAL, "NULL argument");
    mgfwa_status r = check_which(c, which);
    if (r) return r;
    fill_plan_info(c, launch_plan(c, which), launch_rows(c, which), info,
                   which);
    return MGFWA_OK;
}

mgfwa_status mgfwa_fit_candidates(const mgfwa_ctx *c, int which, mgfwa_plan_info *out, int max_out,
                                  int *n)
{
    if (!c || !n) return fail(MGFWA_EINVAL, "NULL argument");
    if (max_out < 0 || (max_out > 0 && !out)) return fail(MGFWA_EINVAL, "bad output buffer");
    if (!c->has_data) return fail(MGFWA_ESTATE, "no built-in fitness: no fitness launches");
    mgfwa_status r = check_which(c, which);
    if (r) return r;
    const int rows = launch_rows(c, which);
    const Net &net = launch_net(c, which);
    FitPlan cand[MAX_CANDIDATES];
    const int nc = net.wide ? 1
                   : which == 2 ? fit_candidates(net, rows, cand, MAX_CANDIDATES)
                                : tune_candidates(c, rows, cand, MAX_CANDIDATES);
    if (net.wide) cand[0] = launch_plan(c, which);
    for (int i = 0; i < nc && i < max_out; ++i) fill_plan_info(c, cand[i], rows, &out[i], which);
    *n = nc;
    return MGFWA_OK;
}

mgfwa_status mgfwa_set_fit_plan(mgfwa_ctx *c, int which, int index)
{
    if (!c) return fail(MGFWA_EINVAL, "ctx is NULL");
    if (c->cfg.external_fitness || !c->has_data)
        return fail(MGFWA_ESTATE, "forcing a plan needs the built-in fitness");
    mgfwa_status r = check_which(c, which);
    if (r) return r;
    if (c->phase != PH_READY || c->gen_host != 0 || c->gexec)
        return fail(MGFWA_ESTATE, "set the fitness plan before the first generation");
    const int rows = launch_rows(c, which);
    const Net &net = launch_net(c, which);
    FitPlan cand[MAX_CANDIDATES];
    const int nc = net.wide ? 1
                   : which == 2 ? fit_candidates(net, rows, cand, MAX_CANDIDATES)
                                : tune_candidates(c, rows, cand, MAX_CANDIDATES);
    if (index < 0 || index >= nc)
        return fail(MGFWA_EINVAL, "plan index %d outside [0, %d)", index, nc);
    if (net.wide) return MGFWA_OK;   // one fixed tile shape
    HIP_TRY(fit_prepare(cand[index]));
    launch_plan(c, which) = cand[index];
    c->s.regen = sparks_regenerated(c) ? 1 : 0;
    return MGFWA_OK;
}

mgfwa_status mgfwa_batch_create(mgfwa_batch **out, mgfwa_ctx *const *ctxs, int n_jobs,
                                void *hip_stream)
{
    if (!out) return fail(MGFWA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctxs || n_jobs < 1) return fail(MGFWA_EINVAL, "no jobs");
    if (!hip_stream)
        return fail(MGFWA_EINVAL, "hip_stream is NULL: pass a stream created by the caller");
    std::vector<mgfwa_ctx *> jobs(ctxs, ctxs + n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        mgfwa_ctx *c = jobs[i];
        if (!c) return fail(MGFWA_EINVAL, "job %d is NULL", i);
        if (c->cfg.external_fitness || c->phase != PH_READY || c->timing)
            return fail(MGFWA_ESTATE, "job %d: needs the built-in fitness, no exchange in "
                                      "progress and timing off", i);
        for (int k = 0; k < i; ++k)
            if (jobs[k] == c) return fail(MGFWA_EINVAL, "job %d appears twice", i);
    }
    mgfwa_batch *b = new mgfwa_batch();
    b->jobs = jobs;
    b->stream = static_cast<hipStream_t>(hip_stream);
    mgfwa_status r = MGFWA_OK;
    for (int i = 0; i <= n_jobs && r == MGFWA_OK; ++i) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            r = fail(MGFWA_EHIP, "hipEventCreate failed");
        else if (i < n_jobs)
            b->job_ev.push_back(e);
        else
            b->done = e;
    }
    if (r == MGFWA_OK) r = batch_capture(b);
    if (r != MGFWA_OK) {
        mgfwa_batch_destroy(b);
        return r;
    }
    *out = b;
    return MGFWA_OK;
}

mgfwa_status mgfwa_batch_step(mgfwa_batch *b, int n)
{
    if (!b) return fail(MGFWA_EINVAL, "batch is NULL");
    if (n < 0) return fail(MGFWA_EINVAL, "n_generations < 0");
    if (n == 0) return MGFWA_OK;
    for (mgfwa_ctx *c : b->jobs)
        if (c->phase != PH_READY || c->timing)
            return fail(MGFWA_ESTATE, "a job of the batch is in an exchange or timing");
    // work already queued on the jobs' own streams runs first, and later work
    // on those streams waits for the batch
    for (size_t i = 0; i < b->jobs.size(); ++i) {
        HIP_TRY(hipEventRecord(b->job_ev[i], b->jobs[i]->stream));
        HIP_TRY(hipStreamWaitEvent(b->stream, b->job_ev[i], 0));
    }
    for (int i = 0; i < n; ++i) HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
    HIP_TRY(hipEventRecord(b->done, b->stream));
    for (mgfwa_ctx *c : b->jobs) {
        HIP_TRY(hipStreamWaitEvent(c->stream, b->done, 0));
        c->gen_host += n;
    }
    return MGFWA_OK;
}

void mgfwa_batch_destroy(mgfwa_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipStream_t st : b->branch) (void)hipStreamDestroy(st);
    for (hipStream_t st : b->fit_branch) (void)hipStreamDestroy(st);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->job_ev) (void)hipEventDestroy(e);
    if (b->done) (void)hipEventDestroy(b->done);
    delete b;
}

const char *mgfwa_last_error(void) { return g_err; }

const char *mgfwa_version(void) { return "mgfwa-gfx950 0.1.0"; }

}  // extern "C"
