/*
 * rcpsp.h -- C ABI of the MI355X (gfx950) tabu-search library for the
 * Resource Constrained Project Scheduling Problem, after Bukata, Sucha and
 * Hanzalek, "Solving the RCPSP using the parallel Tabu Search designed for the
 * CUDA platform" (JPDC 77, 2015).
 *
 * Conventions
 *  - All integers are int32 unless stated; arrays are row-major.
 *  - Host arrays passed to the library are copied; the caller keeps ownership.
 *  - Outputs go to caller-allocated buffers.
 *  - Every entry point returns an rcpsp_status; nothing throws across the ABI.
 *    rcpsp_last_error() returns a thread-local message for the last failure.
 *  - hip_stream is a hipStream_t (NULL = the null stream).  Entry points that
 *    say "asynchronous" only enqueue work on it.
 *  - Instances are immutable after creation and may be shared between threads;
 *    a search or batch object must not be used by two threads at once.
 */
#ifndef RCPSP_H
#define RCPSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RCPSP_OK = 0,
    RCPSP_E_ARG = -1,        /* null pointer, size or parameter out of range */
    RCPSP_E_CYCLE = -2,      /* the precedence graph is not acyclic (Section 2) */
    RCPSP_E_REQUEST = -3,    /* r_ik < 0 or r_ik > R_k, or R_k < 0 (Section 2) */
    RCPSP_E_DUMMY = -4,      /* d_0 or d_{N-1} != 0, dummy requests, an activity
                                without predecessor lacks the arc 0->i, or one
                                without successor lacks i->N-1 (Section 2) */
    RCPSP_E_ORDER = -5,      /* not a precedence-feasible permutation with
                                w_0 = 0 and w_{N-1} = N-1 (Sections 2, 4.2) */
    RCPSP_E_BUFFER = -6,     /* caller buffer too small */
    RCPSP_E_NOMEM = -7,      /* host or device allocation failed */
    RCPSP_E_DEVICE = -8,     /* a HIP call failed */
    RCPSP_E_TOO_LARGE = -9   /* beyond the kernels' limits (N, M, horizon, LDS) */
} rcpsp_status;

/* Resource evaluation algorithm used by the schedule decoder (Section 5). */
typedef enum {
    RCPSP_EVAL_AUTO = 0,      /* chosen per instance before the search (Section 5.4) */
    RCPSP_EVAL_TIME = 1,      /* time-indexed: Algs. 5 and 6 */
    RCPSP_EVAL_CAPACITY = 2   /* capacity-indexed: eq. 7 and Alg. 4 */
} rcpsp_eval;

typedef struct rcpsp_instance rcpsp_instance;

/*
 * Create a project instance (problem statement, Section 2).
 *   n          N, number of activities including the dummies 0 and N-1 (3..2048)
 *   m          M, number of renewable resources (1..16)
 *   duration   [N]    d_i >= 0, d_0 = d_{N-1} = 0; sum d_i <= 32767
 *   capacity   [M]    R_k >= 0 (<= 32767)
 *   request    [N*M]  r_{i,k} at i*M+k, 0 <= r_ik <= R_k
 *   succ_off   [N+1]  successor lists in CSR form (Table 1 "Successors")
 *   succ       [succ_off[N]] successor ids
 *   eval       decoder; AUTO resolves it from the instance attributes of
 *              Table tab:attr (see rcpsp_instance_info); a search may
 *              override it (rcpsp_search_params.eval, rcpsp_autotune)
 *   out        receives the instance (library-owned; free with
 *              rcpsp_destroy_instance)
 * The instance is validated (errors above), derived data is computed on the
 * host (predecessor lists, critical path, horizon) and a packed copy is
 * uploaded to the current device.  Synchronous.
 */
rcpsp_status rcpsp_create_instance(int32_t n, int32_t m, const int32_t *duration,
                                   const int32_t *capacity, const int32_t *request,
                                   const int32_t *succ_off, const int32_t *succ,
                                   rcpsp_eval eval, rcpsp_instance **out);

typedef struct {
    int32_t n, m, n_arcs;
    int32_t horizon;          /* UB = sum of d_i (Section 5.2.1) */
    int32_t critical_path;    /* longest 0 -> N-1 path, arc (i,j) weighted d_i (Section 2) */
    int32_t eval;             /* resolved decoder: 1 time-indexed, 2 capacity-indexed */
    int32_t min_capacity, max_capacity;
    int32_t sum_capacity;     /* sum of R_k (capacity-indexed state size) */
    int32_t field_bits;       /* 8 or 16: per-resource field width of the packed time-indexed profile */
    int32_t avg_capacity_x1000, avg_duration_x1000, branch_factor_x1000; /* Table tab:attr */
} rcpsp_info;

rcpsp_status rcpsp_instance_info(const rcpsp_instance *inst, rcpsp_info *out);
void rcpsp_destroy_instance(rcpsp_instance *inst);

/* Evaluation of one neighbourhood (Sections 4.2-4.5, 5).
 * Moves are swap(u,v) with 1 <= u < v <= N-2 and v-u <= swap_range, in the
 * canonical order u ascending then v ascending; P is their number.
 * A move is feasible under eqs. 5 and 6; every feasible move is decoded with
 * the serial schedule generation scheme (Alg. 7) and the instance's decoder.
 * A move is admissible if it is not tabu or its makespan is below
 * `aspiration`; `best` is the lexicographically smallest (C_max, u, v) among
 * admissible moves, or among all feasible moves if none is admissible.   */
typedef struct {
    int32_t u, v, makespan;   /* (0, 0, -1) when no move is feasible */
    int32_t n_feasible;       /* number of feasible moves; RCPSP_E_ORDER (<0) if
                                 the device variant was given an invalid order */
} rcpsp_move;

/* Host variant, synchronous on hip_stream.
 *   order      [N] host, a precedence-feasible activity list
 *   swap_range delta >= 1
 *   tabu       NULL or [N*N] host bytes, tabu[u*N+v] != 0 marks swap(u,v) tabu
 *   aspiration INT32_MAX for none
 *   makespan   [cap] host: C_max per potential move, -1 if infeasible;
 *              RCPSP_E_BUFFER if cap < P (P is still written to *n_potential)
 *   n_potential receives P (may be NULL)
 *   best       host, may be NULL                                            */
rcpsp_status rcpsp_evaluate_neighbourhood(const rcpsp_instance *inst, const int32_t *order,
                                          int32_t swap_range, const uint8_t *tabu,
                                          int32_t aspiration, int32_t *makespan, int32_t cap,
                                          int32_t *n_potential, rcpsp_move *best,
                                          void *hip_stream);

/* Device variant, asynchronous: order [N] int32, tabu [N*N] uint8 or NULL,
 * makespan [P] int32 and best (one rcpsp_move) are device pointers.  The
 * kernel checks the order itself; an invalid order writes
 * best->n_feasible = RCPSP_E_ORDER and leaves makespan untouched.          */
rcpsp_status rcpsp_evaluate_neighbourhood_device(const rcpsp_instance *inst, const int32_t *order,
                                                 int32_t swap_range, const uint8_t *tabu,
                                                 int32_t aspiration, int32_t *makespan,
                                                 rcpsp_move *best, void *hip_stream);

/* The host variant above without any device allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and errors as rcpsp_evaluate_neighbourhood.  The order, the tabu matrix,
 * the makespans and the best move are staged through one fixed scratch
 * array of RCPSP_NOALLOC_SCRATCH_BYTES in device memory per GPU, reserved
 * when the library is loaded and held until the process ends; every call
 * overwrites what the previous one left there (nothing in it has to start
 * at zero).  A call needs 4N + 4P + 16 bytes, plus N*N with a tabu matrix,
 * each part rounded up to 256 bytes; beyond RCPSP_NOALLOC_SCRATCH_BYTES it
 * returns RCPSP_E_TOO_LARGE.  Calls that overlap on one GPU (from several
 * host threads, or on several streams) race on the array: the caller
 * serialises them.  Synchronous on hip_stream. */
#define RCPSP_NOALLOC_SCRATCH_BYTES (1u << 20)
rcpsp_status rcpsp_evaluate_neighbourhood_noalloc(const rcpsp_instance *inst, const int32_t *order,
                                                  int32_t swap_range, const uint8_t *tabu,
                                                  int32_t aspiration, int32_t *makespan, int32_t cap,
                                                  int32_t *n_potential, rcpsp_move *best,
                                                  void *hip_stream);

/* Number of potential swap moves P for (N, swap_range). */
int32_t rcpsp_potential_moves(int32_t n, int32_t swap_range);

/* Tabu search parameters (Sections 3, 4, 6; Table tab:params). */
typedef struct {
    int32_t swap_range;       /* delta (1..64) */
    int32_t tabu_len;         /* |tabuList| (>= 1) */
    int32_t iterations;       /* I_block: iterations per search (>= 0) */
    int32_t searches;         /* B: number of concurrent searches (>= 1) */
    int32_t elite;            /* |F|: working-set size; 0 = independent searches */
    int32_t phi_max;          /* diversify when a record was read more than phi_max times */
    int32_t phi_steps;        /* random feasible swaps per diversification */
    int32_t threads;          /* threads per search: 0 = auto, else 64, 128, 256,
                                 192 (time-indexed, one candidate per lane) or
                                 512 (one candidate per wave, lanes = 64, or 8
                                 lanes per capacity-indexed candidate) */
    int32_t profile_len;      /* time-indexed LDS profile slots per lane, 0 = auto
                                 (about 1.4 x critical path, stretched while the
                                 workgroups per CU stay the same, never below
                                 1.25 x critical path + longest duration) */
    int32_t record_trajectory;/* 1 = keep (u, v, C_after, C_best) per iteration on the device */
    int32_t count_work;       /* 1 = also count the decodes' algorithmic operations
                                 (instrumented kernels; for measurement runs) */
    int32_t full_decode;      /* 1 = decode every candidate from its first position
                                 instead of continuing from the schedule prefix it
                                 shares with the current order (same results) */
    int32_t eval;             /* decoder for this search: 0 = the instance's,
                                 or capacity-indexed when the instance's is
                                 time-indexed and its LDS profile (at least
                                 1.25 x critical path + longest duration
                                 slots) does not fit; 1 time-indexed, 2 capacity-indexed.
                                 The resolved decoder is reported by
                                 rcpsp_search_get_config and decides results. */
    int32_t lanes;            /* lanes per candidate decode: 0 = auto (1, or
                                 when a per-lane state does not fit: one
                                 candidate per wave / 16 lanes time-indexed,
                                 8 lanes capacity-indexed), 1, 16
                                 (time-indexed only: 16 lanes test 16 time
                                 units per step), 8 (capacity-indexed only:
                                 a lane per resource, eq. 7 and Alg. 4 of the
                                 resources side by side) or 64 (time-indexed
                                 only, 512 threads: one candidate per wave,
                                 its profile of 2048 / words-per-unit time
                                 units in registers, a lane per unit of a
                                 64-unit chunk); same results */
    uint64_t seed;            /* seeds the initial orders and diversification */
    int32_t fbi;              /* 1 = forward-backward improvement of every second
                                 initial solution (odd search index, or odd
                                 working-set record index): backward serial
                                 SGS on the reversed project over activities by
                                 decreasing finish time, forward serial SGS by
                                 decreasing backward finish (ties: later list
                                 position first), repeated while the makespan
                                 strictly decreases, with the search's decoder.
                                 Search plans only (batches and servers reject
                                 it).  0 = off */
    int32_t exchange_every;   /* iterations between working-set exchange rounds
                                 (Section 6.1): 0 or 1 = after every iteration,
                                 as in the paper; k > 1 = after iterations
                                 k, 2k, ... (a search whose exchange condition
                                 fired at any iteration of the block takes part;
                                 the conditions only grow while a read is held).
                                 Search plans only (batches, servers and
                                 re-selecting searches take 0 or 1) */
    int32_t time_budget_us;   /* wall-time budget of a run in microseconds,
                                 counted on the device clock from the start of
                                 the run's first kernel; 0 = none.  Checked at
                                 iteration boundaries: with a working set the
                                 exchange round after an iteration ends the run
                                 when the budget has passed (no round, no further
                                 iteration); independent searches each stop at
                                 their first iteration boundary past it.  The
                                 results equal those of a run of that many
                                 iterations whose eq. 8 still takes `iterations`
                                 as I_block (iterations_done tells how many).
                                 Search plans only (batches reject it; servers
                                 take it as the request's budget when submit's
                                 budget_us is 0) */
    int32_t lane_profile;     /* where a one-candidate-per-lane time-indexed decode
                                 keeps its resource profile: 0 = automatic (LDS),
                                 1 = LDS (profile_len units per lane), 2 = registers
                                 (160 time units of one dword, for instances whose
                                 time unit packs into one dword, i.e. up to four
                                 resources of capacity <= 127 or two of <= 32767;
                                 256 threads per search; schedules past 160 take
                                 the long-profile path).  Same results */
} rcpsp_search_params;

/* Results; every pointer may be NULL (not copied).  Sizes in parentheses. */
typedef struct {
    int32_t *best_makespan;   /* [B] best makespan reached by each search */
    int32_t *best_order;      /* [B*N] the corresponding activity lists */
    int32_t *iterations_done; /* [B] */
    int64_t *evaluations;     /* [B] decoded feasible candidates */
    int32_t *trajectory;      /* [B*iterations*4] (u, v, C_after, C_best); -1 when not done */
    int32_t *elite_makespan;  /* [elite] final working set */
    int32_t *elite_order;     /* [elite*N] */
    int32_t global_best;      /* out: minimum over searches and working set */
    int64_t total_evaluations;/* out */
    int32_t overflow_decodes; /* out: candidates that needed the long-profile path */
    int64_t total_work;       /* out: algorithmic operations of the decodes the run
                                 made (count_work plans only): time-indexed:
                                 activities + predecessor reads + time units
                                 examined by Alg. 5 + time units updated by Alg. 6;
                                 capacity-indexed: activities + predecessor reads +
                                 eq. 7 lookups + Alg. 4 loop steps.  With
                                 full_decode every candidate is decoded from its
                                 first position (the method's work per
                                 evaluation); without it, the shared schedule
                                 prefixes are decoded once per wave or group and
                                 every candidate from its first swapped position
                                 on (the work the run did) */
    int64_t total_cells;      /* out: the resource-state cells among total_work
                                 (time units examined or updated; eq. 7 lookups and
                                 Alg. 4 steps) */
} rcpsp_search_result;

typedef struct rcpsp_search rcpsp_search;

/* Build a search plan: device state, initial orders (Section 4.1) and, for a
 * working set, the captured graph of iteration and exchange kernels.
 * Synchronous. */
rcpsp_status rcpsp_search_create(const rcpsp_instance *inst, const rcpsp_search_params *params,
                                 void *hip_stream, rcpsp_search **out);
/* Run the whole search from its initial state on the device (homogeneous
 * model: no host traffic).  Asynchronous; may be called repeatedly and
 * gives the same results each time. */
rcpsp_status rcpsp_search_run(rcpsp_search *s, void *hip_stream);
/* Same launches as rcpsp_search_run, issued one by one on hip_stream with
 * HIP events around each iteration-kernel and exchange-round launch; waits
 * for completion and reports the summed device milliseconds of each kind and
 * of the whole run (any pointer may be NULL).  Synchronous. */
rcpsp_status rcpsp_search_run_timed(rcpsp_search *s, void *hip_stream, double *iteration_ms,
                                    double *round_ms, double *total_ms);
/* Wait for hip_stream and copy the results to the host buffers. */
rcpsp_status rcpsp_search_results(rcpsp_search *s, rcpsp_search_result *res, void *hip_stream);
void rcpsp_search_destroy(rcpsp_search *s);

/* create + run + results + destroy. */
rcpsp_status rcpsp_tabu_search(const rcpsp_instance *inst, const rcpsp_search_params *params,
                               rcpsp_search_result *res, void *hip_stream);

/* The same independent searches in the heterogeneous model (the CPU-driven
 * alternative the paper compares its homogeneous model with, Section 1): the
 * host runs each search's loop (move application, Alg. 3 tabu list, best and
 * stop updates) and every iteration's neighbourhood is evaluated on the
 * device by rcpsp_evaluate_neighbourhood_device, one launch and one
 * read-back per iteration, searches one after another.  Initial orders come
 * from the reset kernel, so the results equal those of rcpsp_tabu_search
 * with the same parameters.  Synchronous on hip_stream.
 *   params  elite must be 0 (independent searches), count_work 0, eval 0 or
 *           the instance's decoder; threads, profile_len and lanes are
 *           ignored (the evaluation entry point chooses its own shape)
 *   res     as for rcpsp_search_results (elite outputs untouched,
 *           overflow_decodes and total_work 0)
 * Errors: RCPSP_E_ARG for the parameters above; errors of the evaluation
 * entry point. */
rcpsp_status rcpsp_tabu_search_hosted(const rcpsp_instance *inst, const rcpsp_search_params *params,
                                      rcpsp_search_result *res, void *hip_stream);

/* Periodic decoder re-selection: the paper's sequential CPU version picks
 * the faster decoder by timing both every 1000 iterations instead of the
 * Section 5.4 rules (Section 7, experimental set-up).  The searches run on
 * the device as for rcpsp_tabu_search; at the start of every period of
 * `period` iterations each decoder whose lane layout fits runs `probe`
 * iterations (time-indexed first), timed with HIP events around its
 * iteration-kernel launches, and the faster one per iteration runs the rest
 * of the period.  When only one decoder fits, it runs every period without
 * probes.  The two decoders are different serial schedules (the
 * time-indexed one back-fills), so the choice changes the search: every
 * decode of iteration it (its neighbourhood, and with a working set the
 * diversification of a read given by the exchange round before it) uses the
 * decoder of the logged segment holding it; set-up decodes (initial orders,
 * working-set records, forward-backward improvement, the first reads) use
 * the instance's decoder.  With the log, the run is reproducible exactly
 * (a search with that per-iteration decoder schedule).  Synchronous on
 * hip_stream.
 *   params   as for rcpsp_search_create, eval must be 0; threads and lanes
 *            apply to the time-indexed decoder (the capacity-indexed one
 *            takes its automatic shape where they name 192 threads or 16
 *            lanes)
 *   period   iterations per period, >= 2 * probe
 *   probe    iterations each decoder runs at the start of a period, >= 1
 *   res      as for rcpsp_search_results
 *   log      [log_cap] segments in run order: first iteration, iterations,
 *            decoder, probe (1) or chosen run (0), measured milliseconds per
 *            iteration launch (per iteration with a working set, per launch
 *            of all the segment's iterations without one, divided by its
 *            iterations); may be NULL when log_cap is 0
 *   n_log    out: segments run (also when more than log_cap)
 * Errors: RCPSP_E_ARG for the parameters above; RCPSP_E_BUFFER when the
 * log is too short (res and n_log are complete); errors of
 * rcpsp_search_create. */
typedef struct {
    int32_t first_iteration, iterations;
    int32_t eval;               /* RCPSP_EVAL_TIME or RCPSP_EVAL_CAPACITY */
    int32_t probe;              /* 1 timing probe, 0 chosen decoder */
    float ms_per_iteration;
} rcpsp_decoder_segment;
rcpsp_status rcpsp_tabu_search_reselect(const rcpsp_instance *inst, const rcpsp_search_params *params,
                                        int32_t period, int32_t probe, rcpsp_search_result *res,
                                        rcpsp_decoder_segment *log, int32_t log_cap, int32_t *n_log,
                                        void *hip_stream);

/* Kernel names and per-launch statistics of the last run of a search plan:
 * launches of the iteration kernel and the number of candidate decodes. */
typedef struct {
    int32_t threads, profile_len, lds_bytes, eval;
    int32_t iteration_launches, round_launches;
    int32_t lanes;            /* lanes per candidate */
    int32_t finish_bits;      /* bits per finish time in the lane states (8 or 16) */
    int32_t register_profile; /* 1 when the lane profiles live in registers */
} rcpsp_search_config;
rcpsp_status rcpsp_search_get_config(const rcpsp_search *s, rcpsp_search_config *out);

/* Batches (many instances, possibly of different sizes, in one run).
 * Each instance i gets its own search (params[i]); its results equal those of
 * rcpsp_tabu_search with the same instance and params (the plan's
 * profile_len and threads do not change results).  Instances are grouped
 * by decoder, profile width, threads per search and workgroups per CU; each
 * group is one persistent launch whose workgroups take tasks from a queue:
 * one set-up task per instance, then, iteration by iteration, one task per
 * (instance, search).  A search task waits for its instance's previous
 * exchange round, which the task finishing the instance's last search of an
 * iteration runs.  The groups' launches run side by side in one captured
 * graph.
 *   inst    [count] instances (must outlive the batch)
 *   params  [count] search parameters (threads 0 = 64; a member whose
 *           workgroup does not fit with the given threads takes fewer)
 * Errors: RCPSP_E_TOO_LARGE when an instance's workgroup does not fit a CU;
 * RCPSP_E_DEVICE from run_timed or results when a run ended early because
 * one wait inside the kernel exceeded its limit (20 s), which leaves the
 * results undefined. */
typedef struct rcpsp_batch rcpsp_batch;
rcpsp_status rcpsp_batch_create(const rcpsp_instance *const *inst, int32_t count,
                                const rcpsp_search_params *params, void *hip_stream, rcpsp_batch **out);
/* Run every instance's search from its initial state.  Asynchronous. */
rcpsp_status rcpsp_batch_run(rcpsp_batch *b, void *hip_stream);
/* Same, bracketed by HIP events; waits and reports device milliseconds. */
rcpsp_status rcpsp_batch_run_timed(rcpsp_batch *b, void *hip_stream, double *total_ms);
/* Results of instance `index` (waits for hip_stream; checks the run ended normally). */
rcpsp_status rcpsp_batch_results(rcpsp_batch *b, int32_t index, rcpsp_search_result *res, void *hip_stream);
typedef struct {
    int32_t instances, classes;
    /* first 8 classes: decoder, threads per search, members, workgroups, LDS bytes */
    int32_t class_eval[8], class_threads[8], class_instances[8], class_workgroups[8], class_lds_bytes[8];
} rcpsp_batch_info;
rcpsp_status rcpsp_batch_get_info(const rcpsp_batch *b, rcpsp_batch_info *out);
void rcpsp_batch_destroy(rcpsp_batch *b);

/* create + run + results + destroy of a batch: count instances, instance i
 * searched with per_inst[i] (its own searches, working set and seed; the
 * results equal rcpsp_tabu_search's for that instance and parameters);
 * out[i] receives its results as rcpsp_search_results would (each out[i]
 * with its own caller buffers, any of them NULL).  Synchronous on
 * hip_stream.  Errors: those of rcpsp_batch_create, rcpsp_batch_run and
 * rcpsp_batch_results (the first failing instance's). */
rcpsp_status rcpsp_tabu_search_batch(const rcpsp_instance *const *inst, int32_t count,
                                     const rcpsp_search_params *per_inst, rcpsp_search_result *out,
                                     void *hip_stream);

/* Decoder and launch shape for one instance and search configuration.
 * Section 5.4 fixes the resource evaluation algorithm per instance before the
 * search, with rules that were learnt by timing both algorithms for a few
 * iterations; this entry point does that timing directly: it runs the search
 * described by params for trial_iterations iterations with every candidate
 * (decoder x lanes per candidate x threads per search x profile length) and
 * keeps the one with the least device time per evaluation.  *out receives
 * params with eval, threads, profile_len, lanes and lane_profile filled in;
 * *info (may be NULL) the choice and its cost.
 * The decoder changes the schedules and so the search, so the choice is made
 * once, before the search, and is part of the result's identity.
 * Synchronous; allocates and frees its own trial plans. */
typedef struct {
    int32_t eval, threads, profile_len;
    int32_t trials;           /* candidates timed */
    int32_t lanes;            /* lanes per candidate */
    double ns_per_evaluation; /* of the chosen candidate */
    int32_t register_profile; /* 1 when the chosen lane profile is in registers
                                 (out->lane_profile = 2) */
} rcpsp_tuning;
rcpsp_status rcpsp_autotune(const rcpsp_instance *inst, const rcpsp_search_params *params,
                            int32_t trial_iterations, void *hip_stream, rcpsp_search_params *out,
                            rcpsp_tuning *info);

/* Serving (requests admitted as they arrive).  A server owns a device arena
 * for search state and a host thread that runs the device in time slices:
 * at each slice boundary it admits queued requests while the arena has room
 * for their state — one queue per launch class (decoder, profile width,
 * threads per search, lanes per candidate), each in arrival order, each
 * class holding at most an equal share of max_active resident slots among
 * the classes with work, so long requests of one class do not block the
 * others.  Each class runs its own slices: a persistent kernel on the
 * class's stream (its grid an equal share of the CUs among the classes with
 * running requests) sets up the new requests and advances every resident
 * request of the class iteration by iteration, each at its own pace; when a
 * slice ends the host takes the finished requests and starts the next.  A
 * request ends at the first iteration boundary where its iteration
 * allowance is used up, its time budget (counted from admission) has passed,
 * every search has stopped, the working set reached the critical path, or
 * it was cancelled; a request whose budget has passed (or that was
 * cancelled) by the end of its set-up runs no iteration and ends with its
 * initial solutions (status iterations = 0).  Its results equal those of a
 * plain run with
 * iterations = the request's `iterations` status field, except that eq. 8
 * keeps the full allowance (params.iterations) as I_block.  State stays
 * resident until rcpsp_server_release.  All entry points are thread-safe.
 * Errors: RCPSP_E_TOO_LARGE (submit) for a request whose state or
 * workgroup can never fit; RCPSP_E_DEVICE when a slice failed, after which
 * the server accepts nothing more. */
typedef struct rcpsp_server rcpsp_server;
typedef struct {
    int32_t max_active;     /* resident requests at most (0 = 256) */
    int32_t slice_us;       /* device time between admission points (0 = 2000) */
    int64_t arena_bytes;    /* device memory for search state (0 = 2 GiB) */
} rcpsp_server_params;
enum { RCPSP_REQ_QUEUED = 0, RCPSP_REQ_RUNNING = 1, RCPSP_REQ_DONE = 2, RCPSP_REQ_FAILED = 3 };
typedef struct {
    int32_t state;            /* RCPSP_REQ_* */
    int32_t best_makespan;    /* done: minimum over searches and working set */
    int32_t iterations;       /* done: search steps per search (see above) */
    int32_t error;            /* failed: status */
    int64_t evaluations;      /* done */
    int64_t submit_ns, admit_ns, done_ns;  /* rcpsp_server_now_ns clock; done_ns = end
                                              of the iteration that ended the search */
    int64_t seen_ns;          /* when the host loop saw the end (result available) */
} rcpsp_request_status;
typedef struct {
    int64_t submitted, admitted, completed, slices;
    double busy_ms;           /* summed wall time of slices */
    int64_t evaluations;      /* of completed requests */
    int32_t resident, queued;
    int64_t arena_used, arena_bytes;
    double device_clock_mhz;  /* measured rate of the device wall clock the deadlines use */
} rcpsp_server_stats;
rcpsp_status rcpsp_server_create(const rcpsp_server_params *params, rcpsp_server **out);
/* Queue a solve (non-blocking).  params: as for a search plan
 * (record_trajectory allowed; count_work, threads and profile_len as
 * usual); budget_us: wall-time budget from admission (0 = none).
 * The instance must outlive the request. */
rcpsp_status rcpsp_server_submit(rcpsp_server *s, const rcpsp_instance *inst, const rcpsp_search_params *params,
                                 int64_t budget_us, int64_t *ticket);
rcpsp_status rcpsp_server_poll(rcpsp_server *s, int64_t ticket, rcpsp_request_status *out);
/* Full results of a finished request (as rcpsp_search_results). */
rcpsp_status rcpsp_server_results(rcpsp_server *s, int64_t ticket, rcpsp_search_result *res);
/* Cancel: a queued request is dropped (state FAILED, error RCPSP_E_ARG); a
 * running one ends at its next iteration boundary. */
rcpsp_status rcpsp_server_cancel(rcpsp_server *s, int64_t ticket);
/* Free a finished or failed request's state and forget its ticket. */
rcpsp_status rcpsp_server_release(rcpsp_server *s, int64_t ticket);
/* Block until no request is queued or running; RCPSP_E_DEVICE if a slice
 * failed, RCPSP_E_ARG if timeout_ms (> 0) passed first. */
rcpsp_status rcpsp_server_drain(rcpsp_server *s, int64_t timeout_ms);
/* Tickets of requests that finished (done or failed) since the last call,
 * in the order the host loop saw them end; at most cap, *n set to the count. */
rcpsp_status rcpsp_server_take_finished(rcpsp_server *s, int64_t *tickets, int32_t cap, int32_t *n);
rcpsp_status rcpsp_server_get_stats(rcpsp_server *s, rcpsp_server_stats *out);
int64_t rcpsp_server_now_ns(void);
/* Stops the host thread after the running slice; requests still queued or
 * running are dropped. */
void rcpsp_server_destroy(rcpsp_server *s);

/* Decoder and threads per search for every instance of a batch (the batch
 * counterpart of rcpsp_autotune).  Instances are grouped by (N, M and the
 * dwords a time-indexed unit takes, which decides whether register profiles
 * are possible); for each
 * group, up to `sample` evenly spaced members run as a batch of
 * trial_iterations iterations under every candidate (decoder time- or
 * capacity-indexed where the instance allows it, threads 64/128/192/256,
 * lanes per candidate 1/16 and one candidate per wave (512 threads) for the
 * time-indexed decoder, 1/8 (8 also at 512 threads) for the
 * capacity-indexed one, profiles in LDS or registers; a nonzero eval,
 * threads or
 * lanes in params fixes that choice), and the candidate
 * with the most evaluations per device second is written to every member of
 * the group.  Results never depend on the choice of threads; the decoder is
 * part of the result (the two decoders are different functions).
 *   out   [count] params[i] with eval, threads and lanes filled in
 *   info  optional: the first 8 groups and their choices
 * Errors: RCPSP_E_TOO_LARGE when no candidate fits a group. */
typedef struct {
    int32_t groups, trials;
    int32_t group_n[8], group_m[8], group_members[8], group_eval[8], group_threads[8], group_lanes[8];
    double group_evals_per_s[8];
    int32_t group_register[8];   /* 1: lane profiles in registers (lane_profile 2) */
} rcpsp_batch_tuning;
rcpsp_status rcpsp_batch_autotune(const rcpsp_instance *const *inst, int32_t count,
                                  const rcpsp_search_params *params, int32_t trial_iterations, int32_t sample,
                                  void *hip_stream, rcpsp_search_params *out, rcpsp_batch_tuning *info);

const char *rcpsp_last_error(void);
const char *rcpsp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RCPSP_H */
