/*
 * Plain CPU oracle for the parallel tabu search of Bukata, Sucha & Hanzalek
 * (RCPSP on CUDA).  TEST INFRASTRUCTURE ONLY: it exists so that tests, the
 * smoke check and the benchmark's CPU baseline can check the GPU library
 * against an independent, obviously correct implementation.  The product
 * library never links, loads or calls it, and it shares no code with it.
 *
 * All arithmetic is integer.  Every function names the passage of the paper
 * it follows.  Orders are int arrays of activity ids (w_0 .. w_{N-1}).
 */
#ifndef RCPSP_ORACLE_H
#define RCPSP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_inst orc_inst;

/* Build from the problem statement data (Section 2).  request is N*M
 * row-major (i*M+k); successors are CSR (succ_off[N+1], succ).  Returns NULL
 * on allocation failure or a graph that is not a DAG. */
orc_inst *orc_create(int n, int m, const int *duration, const int *capacity,
                     const int *request, const int *succ_off, const int *succ);
void orc_free(orc_inst *inst);

int orc_n(const orc_inst *inst);
int orc_horizon(const orc_inst *inst);          /* UB = sum of durations (Section 5.2.1) */
int orc_critical_path(const orc_inst *inst);    /* longest 0 -> N-1 path, arcs (i,j) weighted d_i (Section 2) */
int orc_levels(const orc_inst *inst, int *level); /* unit-weight longest distance from 0 (Section 4.1); returns l_max */

/* Decoders (Section 5).  Each fills start[N] (may be NULL) and returns C_max.
 *  time:      serial SGS, each activity at the earliest t >= es_prec such that
 *             the per-time-unit capacity constraint (eq. 4) holds over [t, t+d)
 *  time_alg5: Alg. 5 (earliest start) + Alg. 6 (update) taken step by step,
 *             over all M resources
 *  capacity:  eq. 7 (earliest resource start) + Alg. 4 (update)            */
int orc_decode_time(const orc_inst *inst, const int *order, int *start);
int orc_decode_time_alg5(const orc_inst *inst, const int *order, int *start);
int orc_decode_capacity(const orc_inst *inst, const int *order, int *start);
/* decoder: 1 = time-indexed, 2 = capacity-indexed */
int orc_decode(const orc_inst *inst, int decoder, const int *order, int *start);

/* Alg. 4 on one resource array c[R] (non-increasing).  was must hold R ints.
 * Returns the residual required effort when the loop ends (0 when the effort
 * was fully placed). */
int orc_capacity_update(int R, int *c, int r, int d, int s, int *was);

/* Work counters of the last decode on this thread (instrumentation for the
 * algorithmic work model): profile slots scanned, slots updated, Alg. 4 loop
 * steps, predecessor reads. */
void orc_work_counters(int64_t out[4]);
void orc_work_reset(void);

/* Swap neighbourhood (Sections 4.2-4.4). */
int orc_count_potential(int n, int delta);      /* |{(u,v): 1<=u<v<=N-2, v-u<=delta}| */
int orc_is_feasible_order(const orc_inst *inst, const int *order); /* permutation, w_0=0, w_{N-1}=N-1, no precedence violated */
int orc_move_feasible(const orc_inst *inst, const int *order, int u, int v); /* eqs. 5 and 6 */

/* Evaluate the reduced neighbourhood of order (canonical order u asc, v asc).
 * makespan[P] receives C_max of every potential move, -1 if infeasible.
 * tabu: NULL or N*N bytes (tabu[u*N+v] != 0 means the move is tabu).
 * best[4] = (u, v, C_max, n_feasible) of the lexicographically smallest
 * (C_max, u, v) among admissible moves (not tabu, or C_max < aspiration);
 * if none is admissible, among all feasible moves; (0,0,-1,0) if none. */
void orc_evaluate_neighbourhood(const orc_inst *inst, int decoder, const int *order, int delta,
                                const uint8_t *tabu, int aspiration, int *makespan, int best[4]);

/* Simple Tabu List + Tabu Cache (Algs. 2 and 3) on caller-owned storage:
 * ring_u/ring_v[len] (empty entry = (0,0)), *widx, cache[N*N]. */
void orc_stl_add(int len, int *ring_u, int *ring_v, int *widx, uint8_t *cache, int n, int u, int v);
int orc_stl_check(const uint8_t *cache, int n, int u, int v);

/* Counter-based SplitMix64 (Steele, Lea & Flood 2014):
 * key = mix64(seed + (stream+1)*GAMMA); x_i = mix64(key + (i+1)*GAMMA). */
uint64_t orc_mix64(uint64_t z);   /* SplitMix64 output function */
uint64_t orc_rng(uint64_t seed, uint64_t stream, uint64_t i);
uint32_t orc_rng_below(uint64_t seed, uint64_t stream, uint64_t i, uint32_t n);

/* Initial order (Section 4.1): levels concatenated, ids ascending inside a
 * level, then each level shuffled (Fisher-Yates, levels in ascending order)
 * with the stream (seed, stream). */
void orc_initial_order(const orc_inst *inst, uint64_t seed, uint64_t stream, int *order);

/* Decay table for eq. 8: E[0] = 2^24, E[j] = floor(E[j-1]*K / 2^32),
 * K = 4278222805 = round(2^32 * exp(-1/256)).  Returns the table length
 * (first j with E[j] == 0); fills at most cap entries. */
int orc_decay_table(uint32_t *out, int cap);
/* eq. 8 read as floor(I_block * (4 E[a] + E[b]) / (25 * 2^24)), clamped >= 1,
 * a = floor(25600 (C_k - C*) / C*), b = floor(1024 IC_k / I_block). */
int orc_iterations_assigned(int i_block, int c_k, int c_star, int ic_k);

typedef struct {
    int delta;        /* swap range */
    int tabu_len;     /* |tabuList| */
    int iterations;   /* I_block: iterations per search */
    int searches;     /* B */
    int elite;        /* |F|; 0 = independent searches, no working set */
    int phi_max;      /* diversify when a record was read more than phi_max times */
    int phi_steps;    /* random feasible swaps per diversification */
    int decoder;      /* 1 time-indexed, 2 capacity-indexed */
    uint64_t seed;
    int i_block;      /* I_block of eq. 8 when the search is cut short (a time
                         budget) before its iteration allowance; 0 = iterations */
    int fbi;          /* 1 = forward-backward improvement of every second
                         initial solution (odd stream index) */
    const int *decoder_of_iteration;  /* [iterations] or NULL: the decoder of
                         every decode of iteration it (its neighbourhood, and
                         the diversification of a read that an exchange round
                         gave it), the periodic re-selection of the
                         experimental set-up (Section 7); set-up decodes
                         (initial orders, records, the first reads) keep
                         `decoder` */
    int exchange_every;  /* iterations between exchange rounds (0 or 1: after
                            every iteration, as in the paper); the exchange
                            conditions only grow while a read is held, so a
                            search whose condition fired at any iteration of
                            the block takes part in the round after it */
    int *round_log;      /* NULL, or room for round_log_cap rounds of
                            ORC_ROUND_LOG_INTS(N, elite, searches) ints: the
                            state after every exchange round (the first one
                            included), written for the tests: per record
                            k = 0..elite-1: C, IC, reads, W[N]; then per search
                            b: slot, I_assigned, C_read, C_cur, C_best */
    int round_log_cap;
} orc_params;

#define ORC_ROUND_LOG_INTS(n, elite, searches) ((elite) * (3 + (n)) + 5 * (searches))

typedef struct {
    int *best_makespan;      /* [B] */
    int *best_order;         /* [B*N] */
    int *iterations_done;    /* [B] */
    int64_t *evaluations;    /* [B] */
    int *trajectory;         /* [B*iterations*4] (u, v, C_after, C_best) or NULL; unused entries -1 */
    int *elite_makespan;     /* [elite] or NULL */
    int *elite_order;        /* [elite*N] or NULL */
} orc_results;

/* Forward-backward improvement of an activity list with the given decoder
 * (in place); returns the makespan of the result.  Reading in the source. */
int orc_fbi(const orc_inst *inst, int decoder, int *order);

/* Tabu search (Sections 3, 4, 6; working set of Section 6.1).  Returns the
 * number of exchange rounds run (0 without a working set). */
int orc_tabu_search(const orc_inst *inst, const orc_params *p, orc_results *res);

#ifdef __cplusplus
}
#endif
#endif
