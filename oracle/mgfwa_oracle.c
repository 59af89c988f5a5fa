/*
 * MGFWA oracle -- TEST INFRASTRUCTURE ONLY (see mgfwa_oracle.h).
 *
 * Plain CPU MGFWA for MLP weight optimisation.  The generation loop follows the
 * GPU-MGFWA paper, Sec. 3, Alg. 1: random initialisation of the fireworks of b
 * populations, explosion sparks, random mapping, multi-guiding sparks, random
 * mapping, fitness of every spark, selection of the best individual of each
 * firework, loser-out tournament, repeated until termination; the answer is the
 * best fitness and its firework position.  The operator definitions that the
 * paper names but does not print (Sec. 2.1: dynamic amplitude, guiding/elite
 * spark, multi-guiding spark, boosted guiding vector, population-based random
 * mapping, loser-out tournament) follow the build's written reading, restated
 * step by step in the comments below.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 */
#include "mgfwa_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static __thread char g_err[256];
static void set_err(const char *msg) { snprintf(g_err, sizeof g_err, "%s", msg); }
const char *orc_error(void) { return g_err; }

/* ------------------------------------------------------------------------- */
/* Counter-based random numbers: Philox4x32 with 10 rounds (Salmon, Moraes,   */
/* Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).  One     */
/* round multiplies counter words 0 and 2 by the two round multipliers, and    */
/* the new words are (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,     */
/* lo(M0*c0)); the key is bumped by the two Weyl constants between rounds.     */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter layout of a draw: (d / 4, row, generation, stream tag), key = seed
 * split into its low and high 32-bit halves; coordinate d takes word d mod 4. */
uint32_t orc_word(uint64_t seed, int tag, uint32_t row, uint32_t t, uint32_t d)
{
    uint32_t ctr[4] = { d / 4u, row, t, (uint32_t)tag };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[d % 4u];
}

float orc_u01(uint32_t r)
{
    /* 24 random bits; both the conversion and the scaling are exact. */
    return (float)(r >> 8) * 0x1p-24f;
}

static float clampf(float v, float lo, float hi)
{
    if (v < lo) return lo;
    if (v > hi) return hi;
    return v;
}

/* Uniform position in [lb, ub]: fma(u, ub - lb, lb), clamped into the closed box. */
static float uniform_in_box(const orc_config *c, float u)
{
    float span = c->ub - c->lb;
    return clampf(fmaf(u, span, c->lb), c->lb, c->ub);
}

/* ------------------------------------------------------------------------- */
/* Fitness (binary64): the loss of the MLP whose weights are the spark, or,   */
/* for the paper's testbed (Sec. 4.1, eq. (1)), the scalar output of a fixed  */
/* MLP whose input is the spark.                                              */
/* Weight layout: for every layer l in order, W_l (out x in, row-major) then  */
/* b_l (out), i.e. the nn.Linear convention.                                  */
/* ------------------------------------------------------------------------- */
int orc_n_params(const orc_problem *p)
{
    int D = 0;
    for (int l = 0; l < p->n_layers; ++l)
        D += p->widths[l] * p->widths[l + 1] + p->widths[l + 1];
    return D;
}

int orc_dim(const orc_problem *p)
{
    return p->kind == ORC_PROBLEM_INPUT ? p->widths[0] : orc_n_params(p);
}

static double act_apply(int act, double z)
{
    switch (act) {
    case ORC_ACT_RELU: return z > 0.0 ? z : 0.0;
    case ORC_ACT_TANH: return tanh(z);
    case ORC_ACT_GELU: return 0.5 * z * (1.0 + erf(z / sqrt(2.0)));
    default: return z;
    }
}

static int max_width(const orc_problem *p)
{
    int w = 0;
    for (int l = 0; l <= p->n_layers; ++l)
        if (p->widths[l] > w) w = p->widths[l];
    return w;
}

/* Forward pass of the network with parameters w at input `in` into
 * out[widths[L]]; a and b are scratch rows. */
static void forward_vec(const orc_problem *p, const float *w, const float *in, double *a,
                        double *b, double *out)
{
    const int in0 = p->widths[0];
    for (int k = 0; k < in0; ++k) a[k] = (double)in[k];
    size_t off = 0;
    for (int l = 0; l < p->n_layers; ++l) {
        const int fi = p->widths[l], fo = p->widths[l + 1];
        const float *W = w + off;
        const float *bias = w + off + (size_t)fi * fo;
        for (int o = 0; o < fo; ++o) {
            double z = 0.0;
            for (int k = 0; k < fi; ++k) z += (double)W[(size_t)o * fi + k] * a[k];
            z += (double)bias[o];
            b[o] = (l < p->n_layers - 1) ? act_apply(p->acts[l], z) : z;
        }
        off += (size_t)fi * fo + fo;
        double *tmp = a; a = b; b = tmp;
    }
    for (int o = 0; o < p->widths[p->n_layers]; ++o) out[o] = a[o];
}

/* Forward pass of sample s of the problem's data. */
static void forward_one(const orc_problem *p, const float *w, int s, double *a, double *b,
                        double *out)
{
    forward_vec(p, w, p->x + (size_t)s * p->widths[0], a, b, out);
}

double orc_net_output(const orc_problem *p, const float *x)
{
    const int mw = max_width(p);
    double *a = malloc(sizeof(double) * mw), *b = malloc(sizeof(double) * mw);
    double *z = malloc(sizeof(double) * mw);
    forward_vec(p, p->net, x, a, b, z);
    const double y = z[0];
    free(a);
    free(b);
    free(z);
    return y;
}

void orc_forward(const orc_problem *p, const float *w, int sample, double *out)
{
    int mw = max_width(p);
    double *a = malloc(sizeof(double) * mw), *b = malloc(sizeof(double) * mw);
    forward_one(p, w, sample, a, b, out);
    free(a);
    free(b);
}

/* Loss of one sample: MSE sums (z_o - y_o)^2 over outputs; CE is
 * log-sum-exp(z) - z_label with the maximum subtracted inside the exponentials. */
static double sample_loss(const orc_problem *p, const double *z, int s)
{
    const int no = p->widths[p->n_layers];
    if (p->loss == ORC_LOSS_MSE) {
        double acc = 0.0;
        for (int o = 0; o < no; ++o) {
            double e = z[o] - (double)p->y[(size_t)s * no + o];
            acc += e * e;
        }
        return acc;
    }
    double mx = z[0];
    for (int o = 1; o < no; ++o)
        if (z[o] > mx) mx = z[o];
    double se = 0.0;
    for (int o = 0; o < no; ++o) se += exp(z[o] - mx);
    return mx + log(se) - z[p->labels[s]];
}

static void per_sample_losses(const orc_problem *p, const float *w, double *ls, int parallel)
{
    const int S = p->n_samples, mw = max_width(p);
#pragma omp parallel if (parallel)
    {
        double *a = malloc(sizeof(double) * mw), *b = malloc(sizeof(double) * mw);
        double *z = malloc(sizeof(double) * mw);
#pragma omp for schedule(static)
        for (int s = 0; s < S; ++s) {
            forward_one(p, w, s, a, b, z);
            ls[s] = sample_loss(p, z, s);
        }
        free(a);
        free(b);
        free(z);
    }
}

/* Mean over samples (and outputs, for MSE), summed in sample order. */
static double reduce_losses(const orc_problem *p, const double *ls)
{
    double tot = 0.0;
    for (int s = 0; s < p->n_samples; ++s) tot += ls[s];
    double denom = (double)p->n_samples;
    if (p->loss == ORC_LOSS_MSE) denom *= (double)p->widths[p->n_layers];
    return tot / denom;
}

static double loss_impl(const orc_problem *p, const float *w, double *per_sample, int parallel)
{
    double *ls = per_sample ? per_sample : malloc(sizeof(double) * p->n_samples);
    per_sample_losses(p, w, ls, parallel);
    double r = reduce_losses(p, ls);
    if (!per_sample) free(ls);
    return r;
}

double orc_loss(const orc_problem *p, const float *w, double *per_sample)
{
    return loss_impl(p, w, per_sample, 1);
}

int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

void orc_loss_rows(const orc_problem *p, const float *w, int rows, int ld, double *out)
{
    if (p->kind == ORC_PROBLEM_INPUT) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int r = 0; r < rows; ++r) out[r] = orc_net_output(p, w + (size_t)r * ld);
        return;
    }
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    if (rows >= 2 * nthreads) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int r = 0; r < rows; ++r) out[r] = loss_impl(p, w + (size_t)r * ld, NULL, 0);
    } else {
        for (int r = 0; r < rows; ++r) out[r] = loss_impl(p, w + (size_t)r * ld, NULL, 1);
    }
}

/* ------------------------------------------------------------------------- */
/* State path (binary32).                                                     */
/* ------------------------------------------------------------------------- */
struct orc_state {
    orc_config c;
    orc_problem p;
    int has_problem;
    int D, m, k, BN, C;
    float inv_k;
    int t, done, phase;
    float *F, *A, *Y, *Yprev;
    int32_t *fresh;
    float *SE, *SG, *Yc;
    double *Yc64;
    int32_t *top, *bottom, *tie;
    int32_t *cstar, *improved, *reinit;
    int32_t *best_f, *best_gen;
    float *best_x, *best_y;
    float *lo, *hi;          /* [B][D] population ranges (map_range) */
};

enum { PH_NEW = 0, PH_NEED_INIT_FIT, PH_READY, PH_NEED_EXPL_FIT, PH_EXPL_DONE, PH_NEED_GUIDE_FIT,
       PH_GUIDE_DONE, PH_LAG_GUIDED };

/* The ranges of every population from the current fireworks (map_range). */
static void update_ranges(orc_state *st)
{
    if (!st->c.map_range) return;
    const size_t D = (size_t)st->D;
    for (int b = 0; b < st->c.B; ++b)
        orc_population_range(st->c.N, st->D, st->F + (size_t)b * st->c.N * D, st->lo + b * D,
                             st->hi + b * D);
}

static const float *range_lo(const orc_state *st, int gf)
{
    return st->c.map_range ? st->lo + (size_t)(gf / st->c.N) * st->D : NULL;
}

static const float *range_hi(const orc_state *st, int gf)
{
    return st->c.map_range ? st->hi + (size_t)(gf / st->c.N) * st->D : NULL;
}

/* A fitness value as the state path stores it: NaN becomes +inf. */
static float canon(float y) { return isnan(y) ? INFINITY : y; }
static float canon64(double y) { return isnan(y) ? INFINITY : (float)y; }

/* Initial / re-initialised position: uniform in the box, one draw per coordinate. */
void orc_init_row(const orc_config *c, int dim, uint32_t row, uint32_t t, int tag, float *x)
{
    for (int d = 0; d < dim; ++d)
        x[d] = uniform_in_box(c, orc_u01(orc_word(c->seed, tag, row, t, (uint32_t)d)));
}

/* Random mapping of one out-of-box coordinate from its draw u2: uniform in the
 * box, or (map_range) uniform in the population's range lo..hi of that
 * dimension, fma(u2, hi - lo, lo), clamped into the box. */
static float map_coordinate(const orc_config *c, float u2, const float *lo, const float *hi, int d)
{
    if (!lo) return uniform_in_box(c, u2);
    float width = hi[d] - lo[d];
    return clampf(fmaf(u2, width, lo[d]), c->lb, c->ub);
}

void orc_population_range(int n, int dim, const float *F, float *lo, float *hi)
{
    for (int d = 0; d < dim; ++d) {
        float a = F[d], b = F[d];
        for (int f = 1; f < n; ++f) {
            float v = F[(size_t)f * dim + d];
            if (v < a) a = v;
            if (v > b) b = v;
        }
        lo[d] = a;
        hi[d] = b;
    }
}

/* Explosion spark: every coordinate moves by A*(2u-1), u uniform; a coordinate
 * that leaves [lb, ub] is mapped to a fresh uniform position drawn from its own
 * stream (the reading of the random mapping; lo/hi select the range variant). */
void orc_explosion_row(const orc_config *c, int dim, const float *x, float amp, uint32_t row,
                       uint32_t t, const float *lo, const float *hi, float *s)
{
    for (int d = 0; d < dim; ++d) {
        float u = orc_u01(orc_word(c->seed, ORC_TAG_EXPL, row, t, (uint32_t)d));
        float v = 2.0f * u - 1.0f;
        float sv = fmaf(amp, v, x[d]);
        if (sv < c->lb || sv > c->ub) {
            float u2 = orc_u01(orc_word(c->seed, ORC_TAG_EXPL_MAP, row, t, (uint32_t)d));
            sv = map_coordinate(c, u2, lo, hi, d);
        }
        s[d] = sv;
    }
}

static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

orc_state *orc_create(const orc_config *c, const orc_problem *p)
{
    if (c->B < 1 || c->N < 1 || c->lambda < 1 || c->G < 1 || c->lambda % c->G != 0) {
        set_err("bad population shape");
        return NULL;
    }
    int m = c->lambda / c->G;
    if (m < 2) { set_err("need at least 2 sparks per guiding group"); return NULL; }
    if (!(c->sigma > 0.0f && c->sigma <= 0.5f)) { set_err("sigma outside (0, 0.5]"); return NULL; }
    if (!(c->lb < c->ub)) { set_err("lb >= ub"); return NULL; }
    if (!p) { set_err("problem dimension needed"); return NULL; }
    orc_state *st = calloc(1, sizeof *st);
    st->c = *c;
    st->p = *p;
    st->has_problem = p->kind == ORC_PROBLEM_INPUT ? p->net != NULL : p->x != NULL;
    if (p->kind == ORC_PROBLEM_INPUT && p->widths[p->n_layers] != 1) {
        set_err("the fixed network of an input problem has one output");
        free(st);
        return NULL;
    }
    st->D = orc_dim(p);
    st->m = m;
    int k = (int)floor((double)c->sigma * (double)m);
    st->k = k < 1 ? 1 : k;
    st->inv_k = (float)(1.0 / (double)st->k);
    st->BN = c->B * c->N;
    st->C = c->lambda + c->G;
    size_t D = (size_t)st->D, BN = (size_t)st->BN;
    st->F = xcalloc(BN * D, sizeof(float));
    st->A = xcalloc(BN, sizeof(float));
    st->Y = xcalloc(BN, sizeof(float));
    st->Yprev = xcalloc(BN, sizeof(float));
    st->fresh = xcalloc(BN, sizeof(int32_t));
    st->SE = xcalloc(BN * c->lambda * D, sizeof(float));
    st->SG = xcalloc(BN * c->G * D, sizeof(float));
    st->Yc = xcalloc(BN * st->C, sizeof(float));
    st->Yc64 = xcalloc(BN * st->C, sizeof(double));
    st->top = xcalloc(BN * c->G * st->k, sizeof(int32_t));
    st->bottom = xcalloc(BN * c->G * st->k, sizeof(int32_t));
    st->tie = xcalloc(BN * c->G, sizeof(int32_t));
    st->cstar = xcalloc(BN, sizeof(int32_t));
    st->improved = xcalloc(BN, sizeof(int32_t));
    st->reinit = xcalloc(BN, sizeof(int32_t));
    st->best_f = xcalloc(c->B, sizeof(int32_t));
    st->best_gen = xcalloc(c->B, sizeof(int32_t));
    st->best_x = xcalloc((size_t)c->B * D, sizeof(float));
    st->best_y = xcalloc(c->B, sizeof(float));
    st->lo = xcalloc((size_t)c->B * st->D, sizeof(float));
    st->hi = xcalloc((size_t)c->B * st->D, sizeof(float));
    st->phase = PH_NEW;
    return st;
}

void orc_destroy(orc_state *st)
{
    if (!st) return;
    free(st->F); free(st->A); free(st->Y); free(st->Yprev); free(st->fresh);
    free(st->SE); free(st->SG); free(st->Yc); free(st->Yc64);
    free(st->top); free(st->bottom); free(st->tie);
    free(st->cstar); free(st->improved); free(st->reinit);
    free(st->best_f); free(st->best_gen); free(st->best_x); free(st->best_y);
    free(st->lo); free(st->hi);
    free(st);
}

static int want(orc_state *st, int phase, const char *what)
{
    if (st->phase != phase) {
        char buf[200];
        snprintf(buf, sizeof buf, "%s called in phase %d (needs %d)", what, st->phase, phase);
        set_err(buf);
        return 0;
    }
    return 1;
}

/* Index of the minimum of n values, lower index on ties. */
static int argmin_first(const float *v, int n)
{
    int best = 0;
    for (int i = 1; i < n; ++i)
        if (v[i] < v[best]) best = i;
    return best;
}

/* Best firework of population b: lowest fitness, lower index on ties. */
static int population_best(orc_state *st, int b)
{
    return argmin_first(st->Y + (size_t)b * st->c.N, st->c.N);
}

static void copy_best(orc_state *st, int b, int f, int gen)
{
    size_t D = (size_t)st->D;
    int gf = b * st->c.N + f;
    memcpy(st->best_x + (size_t)b * D, st->F + (size_t)gf * D, D * sizeof(float));
    st->best_y[b] = st->Y[gf];
    st->best_f[b] = f;
    st->best_gen[b] = gen;
}

static void check_target(orc_state *st)
{
    if (!st->c.use_target) return;
    for (int b = 0; b < st->c.B; ++b)
        if (st->best_y[b] <= st->c.target_loss) st->done = 1;
}

/* Alg. 1, initialisation: fireworks uniform in the box, amplitude A0. */
int orc_init_positions(orc_state *st)
{
    if (!want(st, PH_NEW, "init_positions")) return -1;
    st->t = 0;
    for (int gf = 0; gf < st->BN; ++gf) {
        orc_init_row(&st->c, st->D, (uint32_t)gf, 0u, ORC_TAG_INIT, st->F + (size_t)gf * st->D);
        st->A[gf] = st->c.amp_init;
        st->fresh[gf] = 0;
    }
    st->phase = PH_NEED_INIT_FIT;
    return 0;
}

static void finish_init(orc_state *st)
{
    for (int gf = 0; gf < st->BN; ++gf) st->Yprev[gf] = st->Y[gf];
    for (int b = 0; b < st->c.B; ++b) copy_best(st, b, population_best(st, b), 0);
    check_target(st);
    st->phase = PH_READY;
}

int orc_tell_init(orc_state *st, const float *y)
{
    if (!want(st, PH_NEED_INIT_FIT, "tell_init")) return -1;
    for (int gf = 0; gf < st->BN; ++gf) st->Y[gf] = canon(y[gf]);
    finish_init(st);
    return 0;
}

int orc_eval_init(orc_state *st)
{
    if (!want(st, PH_NEED_INIT_FIT, "eval_init")) return -1;
    if (!st->has_problem) { set_err("no problem to evaluate"); return -1; }
    double *y = malloc(sizeof(double) * st->BN);
    orc_loss_rows(&st->p, st->F, st->BN, st->D, y);
    for (int gf = 0; gf < st->BN; ++gf) st->Y[gf] = canon64(y[gf]);
    free(y);
    finish_init(st);
    return 0;
}

/* Alg. 1, explosion sparks of every firework plus their random mapping. */
int orc_explode(orc_state *st)
{
    if (!want(st, st->c.lag_guiding ? PH_LAG_GUIDED : PH_READY, "explode")) return -1;
    const uint32_t tn = (uint32_t)(st->t + 1);
    const int lam = st->c.lambda;
    update_ranges(st);
    for (int gf = 0; gf < st->BN; ++gf)
        for (int j = 0; j < lam; ++j) {
            uint32_t row = (uint32_t)(gf * lam + j);
            orc_explosion_row(&st->c, st->D, st->F + (size_t)gf * st->D, st->A[gf], row, tn,
                              range_lo(st, gf), range_hi(st, gf), st->SE + (size_t)row * st->D);
        }
    st->phase = PH_NEED_EXPL_FIT;
    return 0;
}

static void store_fitness(orc_state *st, int first, int per, const double *y64, const float *y32)
{
    for (int gf = 0; gf < st->BN; ++gf)
        for (int j = 0; j < per; ++j) {
            size_t src = (size_t)gf * per + j;
            size_t dst = (size_t)gf * st->C + first + j;
            if (y64) {
                st->Yc64[dst] = y64[src];
                st->Yc[dst] = canon64(y64[src]);
            } else {
                st->Yc64[dst] = NAN;
                st->Yc[dst] = canon(y32[src]);
            }
        }
}

int orc_eval_explosion(orc_state *st)
{
    if (!want(st, PH_NEED_EXPL_FIT, "eval_explosion")) return -1;
    if (!st->has_problem) { set_err("no problem to evaluate"); return -1; }
    int rows = st->BN * st->c.lambda;
    double *y = malloc(sizeof(double) * rows);
    orc_loss_rows(&st->p, st->SE, rows, st->D, y);
    store_fitness(st, 0, st->c.lambda, y, NULL);
    free(y);
    st->phase = PH_EXPL_DONE;
    return 0;
}

int orc_tell_explosion(orc_state *st, const float *y)
{
    if (!want(st, PH_NEED_EXPL_FIT, "tell_explosion")) return -1;
    store_fitness(st, 0, st->c.lambda, NULL, y);
    st->phase = PH_EXPL_DONE;
    return 0;
}

/* Multi-guiding sparks.  The lambda explosion sparks of a firework form G
 * contiguous groups of m = lambda/G.  In each group the members are ranked by
 * (fitness, spark index) ascending; the first k form the top set and the last k
 * the bottom set, k = max(1, floor(sigma*m)).  The guiding vector is
 * (sum of top sparks - sum of bottom sparks) * (1/k), each sum accumulated in
 * ascending spark index, or exactly zero when every fitness in the group is
 * equal.  The guiding spark is x + boost*delta (x + delta when boost is 1),
 * followed by the same random mapping as the explosion sparks. */
void orc_guide_group(int m, int k, int dim, const float *sparks, const float *y, const float *x,
                     float boost, float inv_k, int32_t *top, int32_t *bottom, int32_t *tie,
                     float *gs)
{
    int *order = malloc(sizeof(int) * m);
    char *in_top = calloc(m, 1), *in_bot = calloc(m, 1);
    /* stable insertion sort of the members by fitness: ties keep index order */
    for (int j = 0; j < m; ++j) {
        int pos = j;
        while (pos > 0 && y[j] < y[order[pos - 1]]) {
            order[pos] = order[pos - 1];
            --pos;
        }
        order[pos] = j;
    }
    *tie = (y[order[0]] == y[order[m - 1]]);
    for (int i = 0; i < k; ++i) {
        in_top[order[i]] = 1;
        in_bot[order[m - 1 - i]] = 1;
    }
    int nt = 0, nb = 0;
    for (int j = 0; j < m; ++j) {
        if (in_top[j]) top[nt++] = j;
        if (in_bot[j]) bottom[nb++] = j;
    }
    for (int d = 0; d < dim; ++d) {
        float delta = 0.0f;
        if (!*tie) {
            float sum_top = 0.0f, sum_bot = 0.0f;
            for (int i = 0; i < k; ++i) {
                sum_top = sum_top + sparks[(size_t)top[i] * dim + d];
                sum_bot = sum_bot + sparks[(size_t)bottom[i] * dim + d];
            }
            delta = (sum_top - sum_bot) * inv_k;
        }
        gs[d] = (boost == 1.0f) ? x[d] + delta : fmaf(boost, delta, x[d]);
    }
    free(order);
    free(in_top);
    free(in_bot);
}

int orc_guide(orc_state *st)
{
    const int lag = st->c.lag_guiding;
    if (!want(st, lag ? PH_READY : PH_EXPL_DONE, "guide")) return -1;
    const int G = st->c.G, m = st->m, k = st->k, lam = st->c.lambda;
    const size_t D = (size_t)st->D;
    const uint32_t tn = (uint32_t)(st->t + 1);
    update_ranges(st);
    /* lag: the explosion sparks and fitness in SE / Yc are the previous
     * generation's; before the first generation there are none, and every
     * guiding vector is zero (the group counts as tied) */
    const int none_yet = lag && st->t == 0;
    for (int gf = 0; gf < st->BN; ++gf) {
        for (int g = 0; g < G; ++g) {
            const size_t gidx = (size_t)gf * G + g;
            const size_t first = (size_t)gf * lam + (size_t)g * m;
            int32_t *top = st->top + gidx * k, *bot = st->bottom + gidx * k;
            float *gs = st->SG + gidx * D;
            if (none_yet) {
                for (int i = 0; i < k; ++i) {
                    top[i] = i;
                    bot[i] = m - k + i;
                }
                st->tie[gidx] = 1;
                memcpy(gs, st->F + (size_t)gf * D, D * sizeof(float));
            } else {
                orc_guide_group(m, k, st->D, st->SE + first * D,
                                st->Yc + (size_t)gf * st->C + g * m, st->F + (size_t)gf * D,
                                st->c.boost, st->inv_k, top, bot, st->tie + gidx, gs);
            }
            for (int i = 0; i < k; ++i) {   /* report spark indices within the firework */
                top[i] += g * m;
                bot[i] += g * m;
            }
            for (size_t d = 0; d < D; ++d) {
                float v = gs[d];
                if (v < st->c.lb || v > st->c.ub) {
                    float u2 = orc_u01(orc_word(st->c.seed, ORC_TAG_GUIDE_MAP, (uint32_t)gidx, tn,
                                                (uint32_t)d));
                    gs[d] = map_coordinate(&st->c, u2, range_lo(st, gf), range_hi(st, gf), (int)d);
                }
            }
        }
    }
    st->phase = lag ? PH_LAG_GUIDED : PH_NEED_GUIDE_FIT;
    return 0;
}

int orc_eval_guiding(orc_state *st)
{
    if (!want(st, st->c.lag_guiding ? PH_EXPL_DONE : PH_NEED_GUIDE_FIT, "eval_guiding")) return -1;
    if (!st->has_problem) { set_err("no problem to evaluate"); return -1; }
    int rows = st->BN * st->c.G;
    double *y = malloc(sizeof(double) * rows);
    orc_loss_rows(&st->p, st->SG, rows, st->D, y);
    store_fitness(st, st->c.lambda, st->c.G, y, NULL);
    free(y);
    st->phase = PH_GUIDE_DONE;
    return 0;
}

int orc_tell_guiding(orc_state *st, const float *y)
{
    if (!want(st, st->c.lag_guiding ? PH_EXPL_DONE : PH_NEED_GUIDE_FIT, "tell_guiding")) return -1;
    store_fitness(st, st->c.lambda, st->c.G, NULL, y);
    st->phase = PH_GUIDE_DONE;
    return 0;
}

/* Selection of each firework's best individual, dynamic amplitude, loser-out
 * tournament and best-so-far, for generation t+1.
 *  - Yprev <- Y.  c* = argmin over the lambda+G candidates (lower index on
 *    ties).  If Y[c*] < Y (strict) the firework moves to that candidate and
 *    A <- A*amp_up, else A <- A*amp_down.
 *  - b = the population's best firework.  Every other firework that was not
 *    re-initialised in the previous generation is a loser when
 *    fma(-(Yprev - Y), T - t, Y) > Y_b, i.e. when its improvement rate would not
 *    reach the best fitness by the end of the budget (T - t clamps at 0); a loser
 *    restarts uniformly in the box with A = A0 and fitness +inf.
 *  - The population best is copied when it improves on the best so far. */
int orc_select(orc_state *st)
{
    if (!want(st, PH_GUIDE_DONE, "select")) return -1;
    const int N = st->c.N, lam = st->c.lambda;
    const size_t D = (size_t)st->D;
    st->t += 1;
    const int t = st->t;
    for (int gf = 0; gf < st->BN; ++gf) {
        const float *yc = st->Yc + (size_t)gf * st->C;
        st->Yprev[gf] = st->Y[gf];
        int cs = argmin_first(yc, st->C);
        st->cstar[gf] = cs;
        if (yc[cs] < st->Y[gf]) {
            const float *src = cs < lam ? st->SE + ((size_t)gf * lam + cs) * D
                                        : st->SG + ((size_t)gf * st->c.G + (cs - lam)) * D;
            memcpy(st->F + (size_t)gf * D, src, D * sizeof(float));
            st->Y[gf] = yc[cs];
            st->A[gf] = st->A[gf] * st->c.amp_up;
            st->improved[gf] = 1;
        } else {
            st->A[gf] = st->A[gf] * st->c.amp_down;
            st->improved[gf] = 0;
        }
        st->reinit[gf] = 0;
    }
    const float remaining = (float)(t < st->c.T ? st->c.T - t : 0);
    for (int b = 0; b < st->c.B; ++b) {
        const int fb = population_best(st, b);
        const float yb = st->Y[b * N + fb];
        for (int f = 0; f < N; ++f) {
            const int gf = b * N + f;
            const int was_fresh = st->fresh[gf];
            st->fresh[gf] = 0;
            if (!st->c.loser_out || f == fb || was_fresh) continue;
            float improvement = st->Yprev[gf] - st->Y[gf];
            float predicted = fmaf(-improvement, remaining, st->Y[gf]);
            if (predicted > yb) {
                orc_init_row(&st->c, st->D, (uint32_t)gf, (uint32_t)t, ORC_TAG_REINIT,
                             st->F + (size_t)gf * D);
                st->A[gf] = st->c.amp_init;
                st->Y[gf] = INFINITY;
                st->fresh[gf] = 1;
                st->reinit[gf] = 1;
            }
        }
        if (yb < st->best_y[b]) copy_best(st, b, fb, t);
    }
    check_target(st);
    st->phase = PH_READY;
    return 0;
}

int orc_run(orc_state *st, int n)
{
    if (st->phase == PH_NEW) {
        if (orc_init_positions(st) || orc_eval_init(st)) return -1;
    }
    for (int i = 0; i < n && !st->done; ++i) {
        if (st->c.lag_guiding) {
            if (orc_guide(st) || orc_explode(st) || orc_eval_explosion(st) ||
                orc_eval_guiding(st) || orc_select(st))
                return -1;
        } else if (orc_explode(st) || orc_eval_explosion(st) || orc_guide(st) ||
                   orc_eval_guiding(st) || orc_select(st)) {
            return -1;
        }
    }
    return 0;
}

void orc_get_view(orc_state *st, orc_view *v)
{
    v->D = st->D; v->m = st->m; v->k = st->k; v->t = st->t; v->done = st->done;
    v->inv_k = st->inv_k;
    v->F = st->F; v->A = st->A; v->Y = st->Y; v->Yprev = st->Yprev; v->fresh = st->fresh;
    v->SE = st->SE; v->SG = st->SG; v->Yc = st->Yc; v->Yc64 = st->Yc64;
    v->top = st->top; v->bottom = st->bottom; v->tie = st->tie;
    v->cstar = st->cstar; v->improved = st->improved; v->reinit = st->reinit;
    v->best_f = st->best_f; v->best_x = st->best_x; v->best_y = st->best_y;
    v->best_gen = st->best_gen;
}
