/*
 * Plain CPU oracle (test infrastructure only; see rcpsp_oracle.h).
 *
 * Deliberately simple: arrays, loops, no blocking or incremental tricks.
 * Where the paper is silent or garbled, the reading taken is stated at the
 * function.
 */
#include "rcpsp_oracle.h"

#include <limits.h>
#include <stdlib.h>
#include <string.h>

struct orc_inst {
    int n, m;
    int *d;          /* [N] */
    int *R;          /* [M] */
    int *r;          /* [N*M] */
    int *succ_off, *succ;
    int *pred_off, *pred;   /* predecessors, ascending id */
    uint8_t *adj;           /* adj[i*N+j] = 1 iff (i,j) in E */
    int *topo;              /* a topological order of V */
    int H, cp, rmax;
};

static _Thread_local int64_t g_work[4];

void orc_work_counters(int64_t out[4]) { memcpy(out, g_work, sizeof(g_work)); }
void orc_work_reset(void) { memset(g_work, 0, sizeof(g_work)); }

static int imax(int a, int b) { return a > b ? a : b; }

orc_inst *orc_create(int n, int m, const int *duration, const int *capacity,
                     const int *request, const int *succ_off, const int *succ) {
    if (n < 2 || m < 0) return NULL;
    orc_inst *I = (orc_inst *)calloc(1, sizeof(orc_inst));
    I->n = n; I->m = m;
    I->d = (int *)malloc(sizeof(int) * n);
    I->R = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
    I->r = (int *)malloc(sizeof(int) * (n * m > 0 ? n * m : 1));
    memcpy(I->d, duration, sizeof(int) * n);
    if (m) memcpy(I->R, capacity, sizeof(int) * m);
    if (m) memcpy(I->r, request, sizeof(int) * n * m);
    int ne = succ_off[n];
    I->succ_off = (int *)malloc(sizeof(int) * (n + 1));
    I->succ = (int *)malloc(sizeof(int) * (ne > 0 ? ne : 1));
    memcpy(I->succ_off, succ_off, sizeof(int) * (n + 1));
    if (ne) memcpy(I->succ, succ, sizeof(int) * ne);
    I->adj = (uint8_t *)calloc((size_t)n * n, 1);
    for (int i = 0; i < n; i++)
        for (int e = succ_off[i]; e < succ_off[i + 1]; e++) I->adj[(size_t)i * n + succ[e]] = 1;
    /* predecessor lists, ascending id */
    I->pred_off = (int *)calloc(n + 1, sizeof(int));
    I->pred = (int *)malloc(sizeof(int) * (ne > 0 ? ne : 1));
    for (int j = 0; j < n; j++) {
        I->pred_off[j + 1] = I->pred_off[j];
        for (int i = 0; i < n; i++)
            if (I->adj[(size_t)i * n + j]) I->pred[I->pred_off[j + 1]++] = i;
    }
    /* topological order (Kahn) */
    I->topo = (int *)malloc(sizeof(int) * n);
    int *indeg = (int *)calloc(n, sizeof(int));
    for (int j = 0; j < n; j++) indeg[j] = I->pred_off[j + 1] - I->pred_off[j];
    int head = 0, tail = 0;
    for (int j = 0; j < n; j++) if (!indeg[j]) I->topo[tail++] = j;
    while (head < tail) {
        int i = I->topo[head++];
        for (int e = succ_off[i]; e < succ_off[i + 1]; e++)
            if (--indeg[succ[e]] == 0) I->topo[tail++] = succ[e];
    }
    free(indeg);
    if (tail != n) { orc_free(I); return NULL; }
    I->H = 0;
    for (int i = 0; i < n; i++) I->H += I->d[i];
    /* critical path: longest path from 0 with arc (i,j) weighted d_i */
    int *est = (int *)calloc(n, sizeof(int));
    for (int t = 0; t < n; t++) {
        int i = I->topo[t];
        for (int e = succ_off[i]; e < succ_off[i + 1]; e++)
            est[succ[e]] = imax(est[succ[e]], est[i] + I->d[i]);
    }
    I->cp = est[n - 1];
    free(est);
    I->rmax = 0;
    for (int k = 0; k < m; k++) I->rmax = imax(I->rmax, I->R[k]);
    return I;
}

void orc_free(orc_inst *I) {
    if (!I) return;
    free(I->d); free(I->R); free(I->r); free(I->succ_off); free(I->succ);
    free(I->pred_off); free(I->pred); free(I->adj); free(I->topo);
    free(I);
}

int orc_n(const orc_inst *I) { return I->n; }
int orc_horizon(const orc_inst *I) { return I->H; }
int orc_critical_path(const orc_inst *I) { return I->cp; }

/* Section 4.1: longest paths from 0 with unit arc weights; level = distance. */
int orc_levels(const orc_inst *I, int *level) {
    for (int i = 0; i < I->n; i++) level[i] = 0;
    for (int t = 0; t < I->n; t++) {
        int i = I->topo[t];
        for (int e = I->succ_off[i]; e < I->succ_off[i + 1]; e++) {
            int j = I->succ[e];
            if (level[i] + 1 > level[j]) level[j] = level[i] + 1;
        }
    }
    int lmax = 0;
    for (int i = 0; i < I->n; i++) lmax = imax(lmax, level[i]);
    return lmax;
}

/* Precedence earliest start (Section 5): max over predecessors j of s_j + d_j. */
static int es_prec(const orc_inst *I, int a, const int *start) {
    int es = 0;
    for (int e = I->pred_off[a]; e < I->pred_off[a + 1]; e++) {
        int j = I->pred[e];
        es = imax(es, start[j] + I->d[j]);
        g_work[3]++;
    }
    return es;
}

/* Serial SGS with a per-time-unit usage table: the earliest t >= es_prec at
 * which adding activity a keeps every resource within capacity at every time
 * unit of [t, t+d_a) (eq. 4).  The horizon UB = sum d_i is never exceeded:
 * placing a at the latest finish time of the already placed activities is
 * always resource feasible, and that time is at most the sum of their
 * durations. */
int orc_decode_time(const orc_inst *I, const int *order, int *start) {
    int n = I->n, m = I->m, H = I->H;
    int *used = (int *)calloc((size_t)(H + 1) * (m > 0 ? m : 1), sizeof(int));
    int *s = (int *)malloc(sizeof(int) * n);
    int cmax = 0;
    for (int u = 0; u < n; u++) {
        int a = order[u];
        int t = es_prec(I, a, s);
        for (;;) {
            int fits = 1;
            for (int tau = t; tau < t + I->d[a] && fits; tau++)
                for (int k = 0; k < m; k++)
                    if (used[(size_t)tau * m + k] + I->r[a * m + k] > I->R[k]) { fits = 0; break; }
            g_work[0]++;
            if (fits) break;
            t++;
        }
        if (t + I->d[a] > H) abort(); /* impossible, see above */
        s[a] = t;
        for (int tau = t; tau < t + I->d[a]; tau++) {
            for (int k = 0; k < m; k++) used[(size_t)tau * m + k] += I->r[a * m + k];
            g_work[1]++;
        }
        cmax = imax(cmax, t + I->d[a]);
    }
    if (start) memcpy(start, s, sizeof(int) * n);
    free(used); free(s);
    return cmax;
}

/* Algs. 5 and 6 as the paper gives them, over all M resources (the printed
 * resource loops stop one short; eq. 4 constrains every resource).
 * Alg. 5: starting at the precedence earliest start, walk the time units
 * below UB and keep the length of the current run of units on which every
 * resource still has the activity's request free; a unit short on any
 * resource ends the run; the walk stops once the run is d long, and the
 * activity starts where that run began.  Alg. 6: take the request off every
 * resource on each unit of [start, start + d).  The free capacities are
 * kept per unit and resource, starting at R_k. */
int orc_decode_time_alg5(const orc_inst *I, const int *order, int *start) {
    const int n = I->n, m = I->m, ub = I->H;
    int *avail = (int *)malloc(sizeof(int) * (size_t)(ub + 1) * (m > 0 ? m : 1));
    for (int t = 0; t <= ub; t++)
        for (int k = 0; k < m; k++) avail[(size_t)t * m + k] = I->R[k];
    int *st = (int *)malloc(sizeof(int) * n);
    int cmax = 0;
    for (int pos = 0; pos < n; pos++) {
        const int a = order[pos], d = I->d[a];
        const int *need = I->r + (size_t)a * m;
        const int lo = es_prec(I, a, st);
        int t = lo, run = 0;
        while (run < d && t < ub) {
            int fits = 1;
            for (int k = 0; k < m; k++) fits = fits && avail[(size_t)t * m + k] >= need[k];
            run = fits ? run + 1 : 0;
            t++;
        }
        const int begin = imax(lo, t - run);
        for (int x = begin; x < begin + d; x++)
            for (int k = 0; k < m; k++) avail[(size_t)x * m + k] -= need[k];
        st[a] = begin;
        cmax = imax(cmax, begin + d);
    }
    if (start) memcpy(start, st, sizeof(int) * n);
    free(avail); free(st);
    return cmax;
}

/* Section 5.1: the capacity array of one resource after an activity takes
 * r units for d time units from s (what Alg. 4 computes, restated).
 * c[0..R) holds for every unit of the resource the time from which it is
 * free, non-increasing, so c[R-r] is the earliest time at which r units are
 * free (eq. 7).  The activity's effort r*d is charged to the units in array
 * order.  A unit is charged only while its time is below the bound, which
 * is the finish s+d until a unit has been raised and then the time the
 * last raised unit was given.  The first r charged units are raised to
 * s+d; from then on each charged unit is raised to the time that the unit
 * charged r charges earlier had before its own raise (the array shifted by
 * r places; `was` keeps those earlier times).  A raise of a unit from c to
 * t costs t - max(c, s) of the effort; the unit whose raise would cost all
 * the effort left, or more, only gets max(c, s) plus what is left, and the
 * update ends there.  Returns the effort left when the array runs out (0
 * whenever s is at least eq. 7's resource earliest start). */
int orc_capacity_update(int R, int *c, int r, int d, int s, int *was) {
    int left = r * d;
    int raised = 0;
    int bound = s + d;
    for (int j = 0; j < R && left > 0; j++) {
        g_work[2]++;
        if (c[j] >= bound) continue;
        if (raised >= r) bound = was[raised - r];
        const int from = imax(c[j], s);
        if (bound - from >= left) {
            c[j] = from + left;
            left = 0;
        } else {
            left -= bound - from;
            was[raised++] = c[j];
            c[j] = bound;
        }
    }
    return left;
}

/* Capacity-indexed SSGS: eq. 7 for the resource earliest start, Alg. 4 for
 * the update, Alg. 7 for the loop.  c_k starts at all zeros. */
int orc_decode_capacity(const orc_inst *I, const int *order, int *start) {
    int n = I->n, m = I->m;
    int **c = (int **)malloc(sizeof(int *) * (m > 0 ? m : 1));
    for (int k = 0; k < m; k++) c[k] = (int *)calloc(I->R[k] > 0 ? I->R[k] : 1, sizeof(int));
    int *copy = (int *)malloc(sizeof(int) * (I->rmax > 0 ? I->rmax : 1));
    int *s = (int *)malloc(sizeof(int) * n);
    int cmax = 0;
    for (int u = 0; u < n; u++) {
        int a = order[u];
        int esp = es_prec(I, a, s);
        int esr = 0;
        for (int k = 0; k < m; k++) {
            int rk = I->r[a * m + k];
            if (rk > 0) esr = imax(esr, c[k][I->R[k] - rk]);
        }
        int sa = imax(esp, esr);
        for (int k = 0; k < m; k++) orc_capacity_update(I->R[k], c[k], I->r[a * m + k], I->d[a], sa, copy);
        s[a] = sa;
        cmax = imax(cmax, sa + I->d[a]);
    }
    if (start) memcpy(start, s, sizeof(int) * n);
    for (int k = 0; k < m; k++) free(c[k]);
    free(c); free(copy); free(s);
    return cmax;
}

int orc_decode(const orc_inst *I, int decoder, const int *order, int *start) {
    return decoder == 2 ? orc_decode_capacity(I, order, start) : orc_decode_time(I, order, start);
}

/* ------------------------------------------------------------------------ */
/* Neighbourhood (Sections 4.2 - 4.4)                                        */

int orc_count_potential(int n, int delta) {
    int c = 0;
    for (int u = 1; u <= n - 2; u++)
        for (int v = u + 1; v <= n - 2 && v - u <= delta; v++) c++;
    return c;
}

int orc_is_feasible_order(const orc_inst *I, const int *order) {
    int n = I->n;
    if (order[0] != 0 || order[n - 1] != n - 1) return 0;
    int *pos = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; i++) pos[i] = -1;
    for (int u = 0; u < n; u++) {
        if (order[u] < 0 || order[u] >= n || pos[order[u]] != -1) { free(pos); return 0; }
        pos[order[u]] = u;
    }
    for (int i = 0; i < n; i++)
        for (int e = I->succ_off[i]; e < I->succ_off[i + 1]; e++)
            if (pos[i] >= pos[I->succ[e]]) { free(pos); return 0; }
    free(pos);
    return 1;
}

/* eq. 5: no arc (w_u, w_x) for x in u+1..v;  eq. 6: no arc (w_x, w_v) for x in u..v-1. */
int orc_move_feasible(const orc_inst *I, const int *order, int u, int v) {
    int n = I->n;
    for (int x = u + 1; x <= v; x++)
        if (I->adj[(size_t)order[u] * n + order[x]]) return 0;
    for (int x = u; x <= v - 1; x++)
        if (I->adj[(size_t)order[x] * n + order[v]]) return 0;
    return 1;
}

static int lex_less(int c1, int u1, int v1, int c2, int u2, int v2) {
    if (c1 != c2) return c1 < c2;
    if (u1 != u2) return u1 < u2;
    return v1 < v2;
}

void orc_evaluate_neighbourhood(const orc_inst *I, int decoder, const int *order, int delta,
                                const uint8_t *tabu, int aspiration, int *makespan, int best[4]) {
    int n = I->n;
    int *w = (int *)malloc(sizeof(int) * n);
    int idx = 0, nfeas = 0;
    int ba_c = INT_MAX, ba_u = 0, ba_v = 0;   /* best admissible */
    int bf_c = INT_MAX, bf_u = 0, bf_v = 0;   /* best feasible */
    for (int u = 1; u <= n - 2; u++) {
        for (int v = u + 1; v <= n - 2 && v - u <= delta; v++, idx++) {
            if (!orc_move_feasible(I, order, u, v)) { makespan[idx] = -1; continue; }
            memcpy(w, order, sizeof(int) * n);
            w[u] = order[v]; w[v] = order[u];
            int c = orc_decode(I, decoder, w, NULL);
            makespan[idx] = c;
            nfeas++;
            int is_tabu = tabu ? tabu[(size_t)u * n + v] != 0 : 0;
            int adm = !is_tabu || c < aspiration;
            if (adm && lex_less(c, u, v, ba_c, ba_u, ba_v)) { ba_c = c; ba_u = u; ba_v = v; }
            if (lex_less(c, u, v, bf_c, bf_u, bf_v)) { bf_c = c; bf_u = u; bf_v = v; }
        }
    }
    free(w);
    if (nfeas == 0) { best[0] = 0; best[1] = 0; best[2] = -1; best[3] = 0; return; }
    if (ba_c != INT_MAX) { best[0] = ba_u; best[1] = ba_v; best[2] = ba_c; }
    else { best[0] = bf_u; best[1] = bf_v; best[2] = bf_c; }
    best[3] = nfeas;
}

/* ------------------------------------------------------------------------ */
/* Simple Tabu List + Tabu Cache (Section 4.5, Algs. 2 and 3)                */

void orc_stl_add(int len, int *ring_u, int *ring_v, int *widx, uint8_t *cache, int n, int u, int v) {
    int uo = ring_u[*widx], vo = ring_v[*widx];
    cache[(size_t)uo * n + vo] = 0;
    ring_u[*widx] = u; ring_v[*widx] = v;
    cache[(size_t)u * n + v] = 1;
    *widx = (*widx + 1) % len;
}

int orc_stl_check(const uint8_t *cache, int n, int u, int v) { return cache[(size_t)u * n + v]; }

/* ------------------------------------------------------------------------ */
/* Random numbers and initial orders                                         */

static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_mix64(uint64_t z) { return mix64(z); }

uint64_t orc_rng(uint64_t seed, uint64_t stream, uint64_t i) {
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    uint64_t key = mix64(seed + (stream + 1) * G);
    return mix64(key + (i + 1) * G);
}

uint32_t orc_rng_below(uint64_t seed, uint64_t stream, uint64_t i, uint32_t n) {
    return (uint32_t)(((orc_rng(seed, stream, i) >> 32) * (uint64_t)n) >> 32);
}

void orc_initial_order(const orc_inst *I, uint64_t seed, uint64_t stream, int *order) {
    int n = I->n;
    int *level = (int *)malloc(sizeof(int) * n);
    int lmax = orc_levels(I, level);
    int pos = 0;
    uint64_t ctr = 0;
    for (int l = 0; l <= lmax; l++) {
        int begin = pos;
        for (int i = 0; i < n; i++) if (level[i] == l) order[pos++] = i;
        for (int i = pos - begin - 1; i >= 1; i--) {
            int j = (int)orc_rng_below(seed, stream, ctr++, (uint32_t)(i + 1));
            int t = order[begin + i]; order[begin + i] = order[begin + j]; order[begin + j] = t;
        }
    }
    free(level);
}

/* ------------------------------------------------------------------------ */
/* eq. 8 (iteration balancing)                                               */

#define DECAY_K 4278222805ULL

int orc_decay_table(uint32_t *out, int cap) {
    uint64_t e = 1ULL << 24;
    int j = 0;
    while (e > 0) {
        if (j < cap) out[j] = (uint32_t)e;
        j++;
        e = (e * DECAY_K) >> 32;
    }
    return j;
}

static uint32_t *g_decay = NULL;
static int g_decay_len = 0;

static uint32_t decay(int64_t j) {
    if (!g_decay) {
        int len = orc_decay_table(NULL, 0);
        uint32_t *t = (uint32_t *)malloc(sizeof(uint32_t) * len);
        orc_decay_table(t, len);
        g_decay_len = len;
        g_decay = t;
    }
    if (j < 0) j = 0;
    return j < g_decay_len ? g_decay[j] : 0;
}

/* The printed quantity factor (1/5)(I_block / I_total) equals 1/(5B) because
 * I_total = I_block * B, which would assign no iterations at all; it is read
 * as I_block / 5, the maximum that guarantees at least five reads per block. */
int orc_iterations_assigned(int i_block, int c_k, int c_star, int ic_k) {
    int64_t a = c_star > 0 ? (25600LL * (c_k - c_star)) / c_star : 0;
    int64_t b = i_block > 0 ? (1024LL * ic_k) / i_block : 0;
    int64_t num = (int64_t)i_block * (4 * (int64_t)decay(a) + (int64_t)decay(b));
    int64_t ia = num / (25LL << 24);
    return ia < 1 ? 1 : (int)ia;
}

/* ------------------------------------------------------------------------ */
/* Tabu search                                                               */

typedef struct {
    int *W_cur, *W_imp, *W_best;
    int C_cur, C_imp, C_best, C_read;
    int *ring_u, *ring_v, widx;
    uint8_t *tc;
    int slot, it_read, I_assigned, fired, stopped, it_done;
    int64_t evals;
    uint64_t rng_ctr;
} search_t;

typedef struct {
    int *W, C;
    int *ring_u, *ring_v, widx;
    uint8_t *tc;
    int IC, reads;
} record_t;

/* Forward-backward improvement (the improvement the paper applies to every
 * second initial solution, defined there only by citation of Li and Willis;
 * also known as double justification).  Reading taken:
 *   - backward pass: the serial SGS on the instance with every arc reversed,
 *     over the activities in decreasing order of their finish times (ties:
 *     the later list position first, which keeps successors first); its
 *     finish times g are times measured back from the end, so the activities
 *     sorted by decreasing g (ties: the later backward-list position first)
 *     are in increasing order of their right-justified start times;
 *   - forward pass: the serial SGS over that list;
 *   - repeat while the forward makespan strictly decreases; the last list
 *     that decreased it is the result;
 *   - both passes use the search's decoder.
 * Returns the makespan of the resulting order (written to `order`). */
static orc_inst *reversed_instance(const orc_inst *I) {
    int n = I->n, ne = I->succ_off[n];
    int *off = (int *)calloc(n + 1, sizeof(int));
    int *lst = (int *)malloc(sizeof(int) * (ne > 0 ? ne : 1));
    for (int j = 0; j < n; j++) {
        off[j + 1] = off[j];
        for (int e = I->pred_off[j]; e < I->pred_off[j + 1]; e++) lst[off[j + 1]++] = I->pred[e];
    }
    orc_inst *R = orc_create(n, I->m, I->d, I->R, I->r, off, lst);
    free(off); free(lst);
    return R;
}

static _Thread_local const int *g_sort_key, *g_sort_pos;
static int by_key_desc(const void *x, const void *y) {
    int a = *(const int *)x, b = *(const int *)y;
    if (g_sort_key[a] != g_sort_key[b]) return g_sort_key[a] > g_sort_key[b] ? -1 : 1;
    return g_sort_pos[a] > g_sort_pos[b] ? -1 : 1;
}

/* the activities by decreasing key, ties by decreasing position in `order` */
static void sort_desc(int n, const int *key, const int *order, int *out) {
    int *pos = (int *)malloc(sizeof(int) * n);
    for (int p = 0; p < n; p++) pos[order[p]] = p;
    for (int a = 0; a < n; a++) out[a] = a;
    g_sort_key = key; g_sort_pos = pos;
    qsort(out, n, sizeof(int), by_key_desc);
    free(pos);
}

int orc_fbi(const orc_inst *I, int decoder, int *order) {
    int n = I->n;
    orc_inst *R = reversed_instance(I);
    int *s = (int *)malloc(sizeof(int) * n), *f = (int *)malloc(sizeof(int) * n);
    int *g = (int *)malloc(sizeof(int) * n), *B = (int *)malloc(sizeof(int) * n);
    int *Wn = (int *)malloc(sizeof(int) * n);
    int C = orc_decode(I, decoder, order, s);
    for (int a = 0; a < n; a++) f[a] = s[a] + I->d[a];
    for (;;) {
        sort_desc(n, f, order, B);
        orc_decode(R, decoder, B, s);
        for (int a = 0; a < n; a++) g[a] = s[a] + I->d[a];
        sort_desc(n, g, B, Wn);
        int C2 = orc_decode(I, decoder, Wn, s);
        if (C2 >= C) break;
        C = C2;
        memcpy(order, Wn, sizeof(int) * n);
        for (int a = 0; a < n; a++) f[a] = s[a] + I->d[a];
    }
    free(s); free(f); free(g); free(B); free(Wn);
    orc_free(R);
    return C;
}

#define STREAM_INIT 0ULL
#define STREAM_DIVERSIFY (1ULL << 32)

static void copy_stl(int len, int n, int *du, int *dv, int *dw, uint8_t *dtc,
                     const int *su, const int *sv, int sw, const uint8_t *stc) {
    memcpy(du, su, sizeof(int) * len);
    memcpy(dv, sv, sizeof(int) * len);
    *dw = sw;
    memcpy(dtc, stc, (size_t)n * n);
}

/* Diversification (Section 6.1): phi_steps random feasible swaps; each step
 * enumerates the feasible moves of the current order in canonical order and
 * applies the one at a uniform index.  The tabu list is left unchanged. */
static void diversify(const orc_inst *I, const orc_params *p, int b, search_t *S) {
    int n = I->n;
    int P = orc_count_potential(n, p->delta);
    int *fu = (int *)malloc(sizeof(int) * (P > 0 ? P : 1));
    int *fv = (int *)malloc(sizeof(int) * (P > 0 ? P : 1));
    for (int step = 0; step < p->phi_steps; step++) {
        int cnt = 0;
        for (int u = 1; u <= n - 2; u++)
            for (int v = u + 1; v <= n - 2 && v - u <= p->delta; v++)
                if (orc_move_feasible(I, S->W_cur, u, v)) { fu[cnt] = u; fv[cnt] = v; cnt++; }
        if (cnt == 0) break;
        int j = (int)orc_rng_below(p->seed, STREAM_DIVERSIFY + (uint64_t)b, S->rng_ctr++, (uint32_t)cnt);
        int t = S->W_cur[fu[j]]; S->W_cur[fu[j]] = S->W_cur[fv[j]]; S->W_cur[fv[j]] = t;
    }
    free(fu); free(fv);
}

static int elite_min(const record_t *F, int nf) {
    int c = INT_MAX;
    for (int k = 0; k < nf; k++) if (F[k].C < c) c = F[k].C;
    return c;
}

/* Read record k into search b (Section 6.1). */
static void read_record(const orc_inst *I, const orc_params *p, int dec, int b, search_t *S, record_t *F,
                        int k) {
    int n = I->n;
    record_t *R = &F[k];
    R->reads += 1;
    memcpy(S->W_cur, R->W, sizeof(int) * n);
    S->C_cur = R->C;
    copy_stl(p->tabu_len, n, S->ring_u, S->ring_v, &S->widx, S->tc, R->ring_u, R->ring_v, R->widx, R->tc);
    S->C_read = R->C;
    if (R->reads > p->phi_max) {
        diversify(I, p, b, S);
        S->C_cur = orc_decode(I, dec, S->W_cur, NULL);
    }
    memcpy(S->W_imp, S->W_cur, sizeof(int) * n);
    S->C_imp = S->C_cur;
    if (S->C_cur < S->C_best) { S->C_best = S->C_cur; memcpy(S->W_best, S->W_cur, sizeof(int) * n); }
    S->it_read = 0;
    S->I_assigned = orc_iterations_assigned(p->i_block > 0 ? p->i_block : p->iterations, R->C,
                                            elite_min(F, p->elite), R->IC);
    S->slot = k;
}

/* One exchange round: fired searches in ascending id write (if they improved
 * the record they read and beat its current content) then read the next
 * record; a diversified read is decoded with `dec`. */
static void exchange_round(const orc_inst *I, const orc_params *p, int dec, search_t *S, record_t *F) {
    int n = I->n;
    for (int b = 0; b < p->searches; b++) {
        search_t *s = &S[b];
        /* a search that stopped (no feasible move) takes part in no round */
        if (!s->fired || s->stopped) continue;
        s->fired = 0;
        int k = s->slot;
        record_t *R = &F[k];
        R->IC += s->it_read;
        if (s->C_imp < s->C_read && s->C_imp < R->C) {
            memcpy(R->W, s->W_imp, sizeof(int) * n);
            R->C = s->C_imp;
            copy_stl(p->tabu_len, n, R->ring_u, R->ring_v, &R->widx, R->tc, s->ring_u, s->ring_v, s->widx, s->tc);
            R->IC = 0;
            R->reads = 0;
        }
        read_record(I, p, dec, b, s, F, (k + 1) % p->elite);
    }
}

/* The state after an exchange round, for the tests (orc_params.round_log). */
static void log_round(const orc_params *p, int n, const search_t *S, const record_t *F, int round) {
    if (!p->round_log || round >= p->round_log_cap) return;
    int *o = p->round_log + (size_t)round * ORC_ROUND_LOG_INTS(n, p->elite, p->searches);
    for (int k = 0; k < p->elite; k++) {
        *o++ = F[k].C; *o++ = F[k].IC; *o++ = F[k].reads;
        memcpy(o, F[k].W, sizeof(int) * n);
        o += n;
    }
    for (int b = 0; b < p->searches; b++) {
        *o++ = S[b].slot; *o++ = S[b].I_assigned; *o++ = S[b].C_read; *o++ = S[b].C_cur; *o++ = S[b].C_best;
    }
}

int orc_tabu_search(const orc_inst *I, const orc_params *p, orc_results *res) {
    int n = I->n, B = p->searches, NF = p->elite, TL = p->tabu_len, IT = p->iterations;
    int P = orc_count_potential(n, p->delta);
    const int every = p->exchange_every > 1 ? p->exchange_every : 1;
    int rounds = 0;
    search_t *S = (search_t *)calloc(B, sizeof(search_t));
    for (int b = 0; b < B; b++) {
        S[b].W_cur = (int *)malloc(sizeof(int) * n);
        S[b].W_imp = (int *)malloc(sizeof(int) * n);
        S[b].W_best = (int *)malloc(sizeof(int) * n);
        S[b].ring_u = (int *)calloc(TL, sizeof(int));
        S[b].ring_v = (int *)calloc(TL, sizeof(int));
        S[b].tc = (uint8_t *)calloc((size_t)n * n, 1);
        S[b].C_best = INT_MAX;
    }
    record_t *F = NF > 0 ? (record_t *)calloc(NF, sizeof(record_t)) : NULL;
    for (int k = 0; k < NF; k++) {
        F[k].W = (int *)malloc(sizeof(int) * n);
        F[k].ring_u = (int *)calloc(TL, sizeof(int));
        F[k].ring_v = (int *)calloc(TL, sizeof(int));
        F[k].tc = (uint8_t *)calloc((size_t)n * n, 1);
        orc_initial_order(I, p->seed, STREAM_INIT + (uint64_t)k, F[k].W);
        if (p->fbi && (k & 1)) orc_fbi(I, p->decoder, F[k].W);
        F[k].C = orc_decode(I, p->decoder, F[k].W, NULL);
    }
    if (res->trajectory)
        for (size_t i = 0; i < (size_t)B * IT * 4; i++) res->trajectory[i] = -1;

    if (NF == 0) {
        for (int b = 0; b < B; b++) {
            orc_initial_order(I, p->seed, STREAM_INIT + (uint64_t)b, S[b].W_cur);
            if (p->fbi && (b & 1)) orc_fbi(I, p->decoder, S[b].W_cur);
            S[b].C_cur = orc_decode(I, p->decoder, S[b].W_cur, NULL);
            S[b].C_best = S[b].C_cur;
            memcpy(S[b].W_best, S[b].W_cur, sizeof(int) * n);
        }
    } else {
        /* initial read: search b takes record b mod |F| (ascending b) */
        for (int b = 0; b < B; b++) {
            S[b].slot = (b + NF - 1) % NF;
            S[b].fired = 1;
            S[b].it_read = 0;
            S[b].C_imp = S[b].C_read = INT_MAX;
        }
        exchange_round(I, p, p->decoder, S, F);
        log_round(p, n, S, F, rounds++);
    }

    int cp = I->cp;
    int gstop = NF > 0 && elite_min(F, NF) == cp;
    int *mk = (int *)malloc(sizeof(int) * (P > 0 ? P : 1));
    int *w = (int *)malloc(sizeof(int) * n);
    for (int it = 0; it < IT && !gstop; it++) {
        const int dec = p->decoder_of_iteration ? p->decoder_of_iteration[it] : p->decoder;
        int c_star = NF > 0 ? elite_min(F, NF) : INT_MAX;
        for (int b = 0; b < B; b++) {
            search_t *s = &S[b];
            if (s->stopped) continue;
            if (NF == 0 && s->C_best == cp) { s->stopped = 1; continue; }
            int asp = s->C_best < c_star ? s->C_best : c_star;
            /* neighbourhood evaluation: every feasible move decoded (Alg. 7) */
            int bu = 0, bv = 0, bc = INT_MAX, fu = 0, fv = 0, fc = INT_MAX, nfeas = 0;
            for (int u = 1; u <= n - 2; u++) {
                for (int v = u + 1; v <= n - 2 && v - u <= p->delta; v++) {
                    if (!orc_move_feasible(I, s->W_cur, u, v)) continue;
                    memcpy(w, s->W_cur, sizeof(int) * n);
                    w[u] = s->W_cur[v]; w[v] = s->W_cur[u];
                    int c = orc_decode(I, dec, w, NULL);
                    nfeas++;
                    int adm = !orc_stl_check(s->tc, n, u, v) || c < asp;
                    if (adm && lex_less(c, u, v, bc, bu, bv)) { bc = c; bu = u; bv = v; }
                    if (lex_less(c, u, v, fc, fu, fv)) { fc = c; fu = u; fv = v; }
                }
            }
            if (nfeas == 0) { s->stopped = 1; continue; }
            if (bc == INT_MAX) { bc = fc; bu = fu; bv = fv; }
            s->evals += nfeas;
            /* apply the selected move, add it to the STL */
            int t = s->W_cur[bu]; s->W_cur[bu] = s->W_cur[bv]; s->W_cur[bv] = t;
            orc_stl_add(TL, s->ring_u, s->ring_v, &s->widx, s->tc, n, bu, bv);
            s->C_cur = bc;
            if (bc < s->C_best) { s->C_best = bc; memcpy(s->W_best, s->W_cur, sizeof(int) * n); }
            if (res->trajectory) {
                int *rec = res->trajectory + ((size_t)b * IT + it) * 4;
                rec[0] = bu; rec[1] = bv; rec[2] = bc; rec[3] = s->C_best;
            }
            s->it_done++;
            if (NF > 0) {
                s->it_read++;
                if (s->C_cur < s->C_imp) { s->C_imp = s->C_cur; memcpy(s->W_imp, s->W_cur, sizeof(int) * n); }
                s->fired = (s->C_imp < s->C_read) || (s->it_read > s->I_assigned);
            }
        }
        if (NF > 0 && it < IT - 1 && (it + 1) % every == 0) {
            /* the reads of this round are completed by iteration it + 1 */
            exchange_round(I, p, p->decoder_of_iteration ? p->decoder_of_iteration[it + 1] : p->decoder, S, F);
            log_round(p, n, S, F, rounds++);
            if (elite_min(F, NF) == cp) gstop = 1;
        }
    }
    free(mk); free(w);

    for (int b = 0; b < B; b++) {
        if (res->best_makespan) res->best_makespan[b] = S[b].C_best;
        if (res->best_order) memcpy(res->best_order + (size_t)b * n, S[b].W_best, sizeof(int) * n);
        if (res->iterations_done) res->iterations_done[b] = S[b].it_done;
        if (res->evaluations) res->evaluations[b] = S[b].evals;
    }
    for (int k = 0; k < NF; k++) {
        if (res->elite_makespan) res->elite_makespan[k] = F[k].C;
        if (res->elite_order) memcpy(res->elite_order + (size_t)k * n, F[k].W, sizeof(int) * n);
    }
    for (int b = 0; b < B; b++) {
        free(S[b].W_cur); free(S[b].W_imp); free(S[b].W_best);
        free(S[b].ring_u); free(S[b].ring_v); free(S[b].tc);
    }
    free(S);
    for (int k = 0; k < NF; k++) { free(F[k].W); free(F[k].ring_u); free(F[k].ring_v); free(F[k].tc); }
    free(F);
    return rounds;
}
