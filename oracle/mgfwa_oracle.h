/*
 * MGFWA oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-file CPU implementation of one MGFWA run (multi-guiding
 * spark fireworks algorithm, GPU-MGFWA paper Alg. 1) applied to MLP weight
 * optimisation, or to the paper's own testbed (Sec. 4.1, eq. (1)): the input
 * of a fixed MLP that minimises the network's scalar output.  It exists to check the HIP library; only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * Precision: every fitness is computed in binary64 with naive loops and rounded
 * once to binary32; every state update (random draws, sparks, guiding vectors,
 * amplitudes, selection, loser-out) runs in binary32 with the operation order
 * written out in mgfwa_oracle.c.  Decisions (ranking, argmin, comparisons) are
 * taken on the binary32 fitness values, the precision the GPU path decides in.
 */
#ifndef MGFWA_ORACLE_H
#define MGFWA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LAYERS 12

enum { ORC_ACT_IDENTITY = 0, ORC_ACT_RELU = 1, ORC_ACT_TANH = 2, ORC_ACT_GELU = 3 };
enum { ORC_LOSS_MSE = 0, ORC_LOSS_CE = 1 };
/* What a spark is: the MLP's parameters (fitness = loss over the samples), or
 * the input of a fixed MLP (Sec. 4.1, eq. (1); fitness = its output). */
enum { ORC_PROBLEM_TRAIN = 0, ORC_PROBLEM_INPUT = 1 };
/* Philox counter word 3: which random stream a draw belongs to. */
enum { ORC_TAG_INIT = 0, ORC_TAG_EXPL = 1, ORC_TAG_EXPL_MAP = 2, ORC_TAG_GUIDE_MAP = 3,
       ORC_TAG_REINIT = 4 };

typedef struct {
    int n_layers;            /* number of Linear layers, 1..ORC_MAX_LAYERS */
    int widths[ORC_MAX_LAYERS + 1];
    int acts[ORC_MAX_LAYERS];/* activation after hidden layer l (l < n_layers-1) */
    int loss;                /* ORC_LOSS_* */
    int n_samples;
    const float *x;          /* [S][widths[0]] */
    const float *y;          /* MSE: [S][widths[n_layers]] */
    const int32_t *labels;   /* CE: [S] */
    int kind;                /* ORC_PROBLEM_*; INPUT ignores loss and the samples */
    const float *net;        /* INPUT: the fixed parameters, in the weight layout below,
                                with widths[n_layers] == 1 */
} orc_problem;

typedef struct {
    int B, N, lambda, G;     /* populations, fireworks, explosion sparks, guiding sparks */
    float sigma, boost, amp_up, amp_down, amp_init, lb, ub;
    int T;                   /* generation budget used by the loser-out prediction */
    uint64_t seed;
    int loser_out;
    int use_target;
    float target_loss;
    /* Variants of Alg. 1 (0 = the default readings):
     *  lag_guiding: guiding sparks of generation t come from generation t-1's
     *    explosion sparks and fitness (Alg. 1 taken literally: guide, explode,
     *    then one evaluation of both), the first generation's guiding vectors
     *    being zero;
     *  map_range: an out-of-box coordinate is mapped uniformly into the
     *    population's current range in that dimension (min..max over its
     *    fireworks) instead of the whole box. */
    int lag_guiding;
    int map_range;
} orc_config;

typedef struct orc_state orc_state;

/* Philox4x32-10 block function: 4 output words from a 128-bit counter and 64-bit key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Random word number (d mod 4) of block (d/4, row, t, tag) under key(seed). */
uint32_t orc_word(uint64_t seed, int tag, uint32_t row, uint32_t t, uint32_t d);
/* Top 24 bits of r scaled by 2^-24: a float in [0, 1 - 2^-24]. */
float orc_u01(uint32_t r);

/* Spark dimension: the parameter count (TRAIN) or the input width (INPUT). */
int orc_dim(const orc_problem *p);
/* Parameter count of the problem's network, sum of fi*fo + fo over layers. */
int orc_n_params(const orc_problem *p);
/* Fitness of one weight vector (binary64, TRAIN).  per_sample may be NULL. */
double orc_loss(const orc_problem *p, const float *w, double *per_sample);
/* Output of the fixed network at input x (binary64, INPUT, eq. (1)). */
double orc_net_output(const orc_problem *p, const float *x);
/* Fitness of rows sparks with leading dimension ld (binary64 results): the loss
 * (TRAIN) or the fixed network's output (INPUT). */
void orc_loss_rows(const orc_problem *p, const float *w, int rows, int ld, double *out);
/* Threads the fitness loops use: n > 0 sets the count; returns the count in force. */
int orc_threads(int n);
/* Forward pass of one sample: writes the widths[n_layers] outputs (binary64). */
void orc_forward(const orc_problem *p, const float *w, int sample, double *out);

/* Single-row helpers of the state path (all binary32). */
void orc_init_row(const orc_config *c, int dim, uint32_t row, uint32_t t, int tag, float *x);
/* lo, hi: the population's per-dimension range for map_range (NULL: the box). */
void orc_explosion_row(const orc_config *c, int dim, const float *x, float amp,
                       uint32_t row, uint32_t t, const float *lo, const float *hi, float *s);
/* Per-dimension minimum and maximum over the n rows of F ([n][dim]). */
void orc_population_range(int n, int dim, const float *F, float *lo, float *hi);

/* One guiding group of m explosion sparks ([m][dim], fitness y[m]) around the
 * firework x: writes the top and bottom member lists (ascending index), the
 * all-tie flag and the unmapped guiding spark gs[dim] = x + boost*delta. */
void orc_guide_group(int m, int k, int dim, const float *sparks, const float *y, const float *x,
                     float boost, float inv_k, int32_t *top, int32_t *bottom, int32_t *tie,
                     float *gs);

orc_state *orc_create(const orc_config *c, const orc_problem *p /* may be NULL */);
void orc_destroy(orc_state *st);
const char *orc_error(void);

/* Phases of one generation.  Fitness comes from the problem (orc_eval_*) or from
 * the caller (orc_tell_*).  Return 0 on success, -1 on misuse.  Default order:
 * explode, explosion fitness, guide, guiding fitness, select.  With lag_guiding:
 * guide, explode, explosion fitness, guiding fitness, select. */
int orc_init_positions(orc_state *st);
int orc_eval_init(orc_state *st);
int orc_tell_init(orc_state *st, const float *y);
int orc_explode(orc_state *st);
int orc_eval_explosion(orc_state *st);
int orc_tell_explosion(orc_state *st, const float *y);
int orc_guide(orc_state *st);
int orc_eval_guiding(orc_state *st);
int orc_tell_guiding(orc_state *st, const float *y);
int orc_select(orc_state *st);
/* init (when needed) then n full generations with problem fitness. */
int orc_run(orc_state *st, int n);

/* Views of the state (owned by st; valid until orc_destroy). */
typedef struct {
    int D, m, k, t, done;
    float inv_k;
    float *F, *A, *Y, *Yprev;        /* [B*N][D], [B*N] ... */
    int32_t *fresh;                  /* [B*N] */
    float *SE;                       /* [B*N*lambda][D] */
    float *SG;                       /* [B*N*G][D] */
    float *Yc;                       /* [B*N][lambda+G] binary32 fitness of candidates */
    double *Yc64;                    /* [B*N][lambda+G] binary64 fitness (NaN if told) */
    int32_t *top, *bottom;           /* [B*N*G][k] members, ascending spark index */
    int32_t *tie;                    /* [B*N*G] */
    int32_t *cstar, *improved, *reinit; /* [B*N] decisions of the last selection */
    int32_t *best_f;                 /* [B] firework holding the population best */
    float *best_x;                   /* [B][D] */
    float *best_y;                   /* [B] */
    int32_t *best_gen;               /* [B] */
} orc_view;
void orc_get_view(orc_state *st, orc_view *v);

#ifdef __cplusplus
}
#endif
#endif
