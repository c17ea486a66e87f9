/*
 * CPU oracle for the enhanced discrete PSO of "Enhanced Discrete Particle Swarm
 * Optimization Path Planning for UAV Vision-based Surface Inspection"
 * (Phung, Quach, Dinh, Ha; arXiv 1706.04399).
 *
 * TEST INFRASTRUCTURE. This file defines what the swarm computes, as plainly as
 * possible, so that the HIP library can be checked against it. Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it. It
 * shares no code, header, table or helper with the HIP library.
 *
 * Arithmetic: distances are int32 millimetres, costs int64, labels 0..n-1
 * (the paper's nodes 1..N). Coefficients are Q16 fixed point. Every tie is
 * broken by the smallest index. Randomness is Philox4x64-10 keyed by
 * (seed, instance) with the counter (block, particle, generation, purpose).
 *
 * Parallelism: OpenMP over particles only inside phases whose particles are
 * independent (move, reshuffle, edge exchange); every reduction runs
 * sequentially in index order, so results do not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OR_D_INF 268435455 /* 2^28 - 1: cost of a blocked pair (Sect. 2.3) */

enum { OR_OK = 0, OR_EINVAL = -1, OR_ERANGE = -2, OR_ENOMEM = -3 };
enum { PURPOSE_INIT = 0, PURPOSE_VEL = 1, PURPOSE_MUT = 2 };
enum { EE_OFF = 0, EE_ON_STALL = 1, EE_ALWAYS = 2 };
enum { NB_TWO_OPT = 0, NB_NODE_SWAP = 1 };

typedef struct {
    int32_t swarm_size, max_generations;
    uint32_t w_q16, phi1_q16, phi2_q16;
    int32_t mutation_period, ee_trigger, ee_max_moves, stall_limit, det_permille;
    uint64_t seed, instance;
    int32_t ee_neighbourhood; /* NB_TWO_OPT (segment reversal) or NB_NODE_SWAP   */
    int32_t mutation_swaps;   /* 0: reshuffle; k > 0: k random position exchanges */
    int32_t velocity_cap;     /* 0: v <- y - x; c > 0: v <- the concatenation of
                                 the three prefixes, its first c transpositions */
} or_params;

typedef struct {
    int32_t n, S;
    int32_t *X;      /* [S][n] current tours                          */
    int32_t *P;      /* [S][n] personal-best tours                    */
    int32_t *V;      /* [S][n][2] velocity: label transpositions      */
    int32_t *VL;     /* [S] velocity lengths                          */
    int64_t *F;      /* [S] cost of X                                 */
    int64_t *FP;     /* [S] cost of P                                 */
    int32_t *G;      /* [n] global-best tour                          */
    int64_t *trace;  /* [trace_cap] F_G after each generation (0=init)*/
    int32_t trace_cap;
    int32_t t, stall, done;
    int64_t FG;
    int64_t n_sweeps, n_moves, n_reshuffled; /* work counters             */
} or_state;

/* ---------------------------------------------------------------------------
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): ten rounds of two 64x64->128 multiplications,
 * with the key bumped by the Weyl constants before every round but the first.
 * ------------------------------------------------------------------------- */
static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mul128(M0, c0, &hi0, &lo0);
        mul128(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A stream of 32-bit draws for one (particle, generation, purpose): block b
 * has counter (b, p, t, purpose); its four words are split low half first. */
typedef struct {
    uint64_t key[2], p, t, purpose, block;
    int used;
    uint32_t d[8];
} or_stream;

static void stream_open(or_stream *s, uint64_t seed, uint64_t inst, uint64_t p,
                        uint64_t t, uint64_t purpose)
{
    s->key[0] = seed; s->key[1] = inst;
    s->p = p; s->t = t; s->purpose = purpose;
    s->block = 0; s->used = 8;
}

static uint32_t stream_next(or_stream *s)
{
    if (s->used == 8) {
        uint64_t ctr[4] = { s->block, s->p, s->t, s->purpose }, w[4];
        or_philox4x64_10(ctr, s->key, w);
        for (int m = 0; m < 4; m++) {
            s->d[2 * m] = (uint32_t)w[m];
            s->d[2 * m + 1] = (uint32_t)(w[m] >> 32);
        }
        s->block++;
        s->used = 0;
    }
    return s->d[s->used++];
}

/* Integer in [0, m): the high word of d*m. */
static uint32_t uniform_below(uint32_t d, uint32_t m)
{
    return (uint32_t)(((uint64_t)d * m) >> 32);
}

/* First `count` draws of a stream (for pinning the stream layout). */
void or_draws(uint64_t seed, uint64_t inst, uint64_t p, uint64_t t, uint64_t purpose,
              int32_t count, uint32_t *out)
{
    or_stream s;
    stream_open(&s, seed, inst, p, t, purpose);
    for (int32_t i = 0; i < count; i++) out[i] = stream_next(&s);
}

/* ---------------------------------------------------------------------------
 * Objective (Sect. 2.3, eq. min): a tour visits every node once and returns
 * to its first node; its cost is the sum of the costs of its n edges.
 * ------------------------------------------------------------------------- */
int64_t or_tour_cost(const int32_t *D, int32_t n, const int32_t *x)
{
    int64_t c = 0;
    for (int32_t k = 0; k < n; k++)
        c += D[(int64_t)x[k] * n + x[(k + 1) % n]];
    return c;
}

/* The matrix contract the swarm relies on (Sect. 2: a symmetric travelling
 * cost between every pair of viewpoints, none from a viewpoint to itself; a
 * blocked pair costs the very large OR_D_INF, Sect. 2.3): D[i][i] = 0,
 * D[i][j] = D[j][i] and 0 <= D[i][j] <= OR_D_INF. Returns the row-major index
 * i * n + j of the first entry that breaks it, or -1. */
int64_t or_check_dist(const int32_t *D, int32_t n)
{
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < n; j++) {
            int32_t v = D[i * n + j];
            if (v < 0 || v > OR_D_INF) return i * n + j;
            if (i == j && v != 0) return i * n + j;
            if (v != D[j * n + i]) return i * n + j;
        }
    return -1;
}

/* ---------------------------------------------------------------------------
 * Velocity operators (Sect. 3.1).
 * A transposition (a, b) exchanges the places of the LABELS a and b in the
 * tour, as in the paper's worked example of position + velocity.
 * ------------------------------------------------------------------------- */
static void swap_labels(int32_t *x, int32_t *pos, int32_t a, int32_t b)
{
    int32_t i = pos[a], j = pos[b];
    x[i] = b; x[j] = a;
    pos[b] = i; pos[a] = j;
}

/* x + (first k transpositions of v), applied in order. */
void or_apply_swaps(int32_t *x, int32_t n, const int32_t *pairs, int32_t k)
{
    int32_t *pos = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; i++) pos[x[i]] = i;
    for (int32_t s = 0; s < k; s++) swap_labels(x, pos, pairs[2 * s], pairs[2 * s + 1]);
    free(pos);
}

/* T - x: a velocity v with x + v = T. Scanning positions left to right, each
 * position holding the wrong label gets the right one by one transposition.
 * Returns the length (n minus the number of cycles of the permutation that
 * carries x to T); pairs[] receives the transpositions. */
int32_t or_bss(const int32_t *x, const int32_t *T, int32_t n, int32_t *pairs)
{
    int32_t *cur = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *pos = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t len = 0;
    memcpy(cur, x, sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; i++) pos[cur[i]] = i;
    for (int32_t q = 0; q < n; q++) {
        if (cur[q] != T[q]) {
            int32_t a = cur[q], b = T[q];
            pairs[2 * len] = a; pairs[2 * len + 1] = b;
            len++;
            swap_labels(cur, pos, a, b);
        }
    }
    free(cur); free(pos);
    return len;
}

/* c.v keeps the first c*|v| transpositions (0 <= c <= 1). The coefficients
 * are Q16; r1, r2 keep the top 16 bits of their 32-bit draws; the products
 * are floored and a coefficient above one is clamped to the whole list.
 * out = {k_w, k_1, k_2}. */
void or_truncate_counts(int32_t lv, int32_t lb, int32_t lc, uint32_t w_q16,
                        uint32_t phi1_q16, uint32_t phi2_q16, uint32_t u1, uint32_t u2,
                        int32_t out[3])
{
    uint64_t kw = ((uint64_t)w_q16 * (uint64_t)lv) >> 16;
    uint64_t k1 = ((uint64_t)phi1_q16 * (uint64_t)(u1 >> 16) * (uint64_t)lb) >> 32;
    uint64_t k2 = ((uint64_t)phi2_q16 * (uint64_t)(u2 >> 16) * (uint64_t)lc) >> 32;
    out[0] = kw < (uint64_t)lv ? (int32_t)kw : lv;
    out[1] = k1 < (uint64_t)lb ? (int32_t)k1 : lb;
    out[2] = k2 < (uint64_t)lc ? (int32_t)k2 : lc;
}

/* ---------------------------------------------------------------------------
 * Initial tours (Sect. 3.2.1 and the initialisation of the pseudo code).
 * ------------------------------------------------------------------------- */

/* Nearest neighbour from `start`: always go to the closest unvisited node,
 * the smallest label on ties. */
void or_nn_tour(const int32_t *D, int32_t n, int32_t start, int32_t *out)
{
    char *seen = calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t cur = start;
    out[0] = start;
    seen[start] = 1;
    for (int32_t s = 1; s < n; s++) {
        int32_t best = -1;
        for (int32_t k = 0; k < n; k++)
            if (!seen[k] && (best < 0 || D[(int64_t)cur * n + k] < D[(int64_t)cur * n + best]))
                best = k;
        out[s] = best;
        seen[best] = 1;
        cur = best;
    }
    free(seen);
}

/* Fisher-Yates shuffle of the identity: for i = n-1 down to 1, exchange
 * places i and uniform(i+1). */
void or_fisher_yates(int32_t n, uint64_t seed, uint64_t inst, uint64_t p, uint64_t t,
                     uint64_t purpose, int32_t *out)
{
    or_stream s;
    stream_open(&s, seed, inst, p, t, purpose);
    for (int32_t i = 0; i < n; i++) out[i] = i;
    for (int32_t i = n - 1; i >= 1; i--) {
        int32_t j = (int32_t)uniform_below(stream_next(&s), (uint32_t)(i + 1));
        int32_t tmp = out[i]; out[i] = out[j]; out[j] = tmp;
    }
}

/* ---------------------------------------------------------------------------
 * Edge exchange (Sect. 3.2.3): a complete 2-opt search. Removing edges
 * (x_i, x_i+1) and (x_j, x_j+1) and reconnecting by reversing x[i+1..j]
 * changes the cost by
 *   delta = D[x_i][x_j] + D[x_i+1][x_j+1] - D[x_i][x_i+1] - D[x_j][x_j+1]
 * (indices mod n). Every pair of non-adjacent edges is tried: 0 <= i,
 * i+2 <= j <= n-1, except (0, n-1). The most improving exchange wins; ties go
 * to the smallest i, then the smallest j.
 * ------------------------------------------------------------------------- */
int64_t or_best_2opt(const int32_t *D, int32_t n, const int32_t *x, int32_t *bi, int32_t *bj)
{
    int64_t best = 0;
    *bi = -1; *bj = -1;
    for (int32_t i = 0; i + 2 < n; i++) {
        for (int32_t j = i + 2; j < n; j++) {
            if (i == 0 && j == n - 1) continue;
            int32_t a = x[i], b = x[i + 1], c = x[j], d = x[(j + 1) % n];
            int64_t delta = (int64_t)D[(int64_t)a * n + c] + D[(int64_t)b * n + d]
                          - D[(int64_t)a * n + b] - D[(int64_t)c * n + d];
            if (*bi < 0 || delta < best) { best = delta; *bi = i; *bj = j; }
        }
    }
    return best;
}

/* Apply best exchanges while they improve; stop after max_moves applied
 * moves when max_moves > 0. Returns the number of applied moves. *sweeps
 * counts complete neighbourhood searches. */
int32_t or_edge_exchange(const int32_t *D, int32_t n, int32_t *x, int64_t *F, int32_t max_moves,
                         int64_t *sweeps)
{
    int32_t moves = 0;
    for (;;) {
        int32_t i, j;
        int64_t delta = or_best_2opt(D, n, x, &i, &j);
        if (sweeps) (*sweeps)++;
        if (i < 0 || delta >= 0) break;
        for (int32_t lo = i + 1, hi = j; lo < hi; lo++, hi--) {
            int32_t tmp = x[lo]; x[lo] = x[hi]; x[hi] = tmp;
        }
        *F += delta;
        moves++;
        if (max_moves > 0 && moves >= max_moves) break;
    }
    return moves;
}

/* ---------------------------------------------------------------------------
 * Node-swap neighbourhood (the edge-exchange kernel and pseudo code of Sect.
 * 3.3 exchange the nodes at two positions and keep the best): exchanging the
 * labels at positions i < j changes only the closing edges k -> k+1 (mod n)
 * that touch i or j, so the cost changes by the sum over those distinct edge
 * indices {i-1, i, j-1, j} (mod n) of new minus old edge cost. This is
 * C(swapped) - C(x) exactly, adjacent and wrapping pairs included.
 * ------------------------------------------------------------------------- */
int64_t or_swap_delta(const int32_t *D, int32_t n, const int32_t *x, int32_t i, int32_t j)
{
    int32_t edges[4] = {(i + n - 1) % n, i, (j + n - 1) % n, j}, m = 0;
    int32_t uniq[4];
    for (int32_t a = 0; a < 4; a++) {
        int32_t seen = 0;
        for (int32_t b = 0; b < m; b++) seen |= uniq[b] == edges[a];
        if (!seen) uniq[m++] = edges[a];
    }
    int64_t delta = 0;
    for (int32_t a = 0; a < m; a++) {
        int32_t k = uniq[a], k1 = (k + 1) % n;
        int32_t u = x[k], v = x[k1];                      /* before */
        int32_t u2 = k == i ? x[j] : k == j ? x[i] : u;   /* after  */
        int32_t v2 = k1 == i ? x[j] : k1 == j ? x[i] : v;
        delta += (int64_t)D[(int64_t)u2 * n + v2] - D[(int64_t)u * n + v];
    }
    return delta;
}

/* Best exchange of two positions: minimum delta over 0 <= i < j < n, ties to
 * the smallest i, then j. *bi = -1 when n < 2. */
int64_t or_best_swap(const int32_t *D, int32_t n, const int32_t *x, int32_t *bi, int32_t *bj)
{
    int64_t best = 0;
    *bi = -1; *bj = -1;
    for (int32_t i = 0; i + 1 < n; i++)
        for (int32_t j = i + 1; j < n; j++) {
            int64_t delta = or_swap_delta(D, n, x, i, j);
            if (*bi < 0 || delta < best) { best = delta; *bi = i; *bj = j; }
        }
    return best;
}

/* or_edge_exchange with the node-swap neighbourhood. */
int32_t or_node_exchange(const int32_t *D, int32_t n, int32_t *x, int64_t *F, int32_t max_moves,
                         int64_t *sweeps)
{
    int32_t moves = 0;
    for (;;) {
        int32_t i, j;
        int64_t delta = or_best_swap(D, n, x, &i, &j);
        if (sweeps) (*sweeps)++;
        if (i < 0 || delta >= 0) break;
        int32_t tmp = x[i]; x[i] = x[j]; x[j] = tmp;
        *F += delta;
        moves++;
        if (max_moves > 0 && moves >= max_moves) break;
    }
    return moves;
}

/* Disturbance of a tour in randomly chosen dimensions (the reading of the
 * mutation text of Sect. 3.2.2 as an alternative to a reshuffle): k
 * exchanges of positions (uniform(n), uniform(n)), drawn in that order from
 * the stream (p, t, purpose), applied one after another. */
void or_disturb(int32_t n, int32_t k, uint64_t seed, uint64_t inst, uint64_t p, uint64_t t,
                uint64_t purpose, int32_t *x)
{
    or_stream s;
    stream_open(&s, seed, inst, p, t, purpose);
    for (int32_t a = 0; a < k; a++) {
        int32_t i = (int32_t)uniform_below(stream_next(&s), (uint32_t)n);
        int32_t j = (int32_t)uniform_below(stream_next(&s), (uint32_t)n);
        int32_t tmp = x[i]; x[i] = x[j]; x[j] = tmp;
    }
}

/* ---------------------------------------------------------------------------
 * Swarm phases (pseudo code of the enhanced DPSO, Sect. 3.3).
 * ------------------------------------------------------------------------- */
static int32_t *row32(int32_t *a, int32_t n, int32_t p) { return a + (int64_t)p * n; }

static void pbest_rule(or_state *st, int32_t p)
{
    if (st->F[p] < st->FP[p]) {
        memcpy(row32(st->P, st->n, p), row32(st->X, st->n, p), sizeof(int32_t) * (size_t)st->n);
        st->FP[p] = st->F[p];
    }
}

/* Global best: the particle with the lowest personal-best cost (lowest index
 * on ties) replaces G only if it is strictly better. Returns 1 if G moved. */
int32_t or_update_gbest(or_state *st)
{
    int32_t g = 0;
    for (int32_t p = 1; p < st->S; p++)
        if (st->FP[p] < st->FP[g]) g = p;
    if (st->FP[g] < st->FG) {
        memcpy(st->G, row32(st->P, st->n, g), sizeof(int32_t) * (size_t)st->n);
        st->FG = st->FP[g];
        return 1;
    }
    return 0;
}

int32_t or_check_params(const or_params *prm, int32_t n)
{
    if (!prm || n < 1 || n > 65535) return OR_EINVAL;
    if (prm->swarm_size < 1 || prm->swarm_size > 65536 || prm->max_generations < 0) return OR_EINVAL;
    if (prm->w_q16 > 131072 || prm->phi1_q16 > 131072 || prm->phi2_q16 > 131072) return OR_EINVAL;
    if (prm->mutation_period < 0 || prm->ee_trigger < 0 || prm->ee_trigger > 2) return OR_EINVAL;
    if (prm->ee_max_moves < 0 || prm->stall_limit < 0) return OR_EINVAL;
    if (prm->det_permille < 0 || prm->det_permille > 1000) return OR_EINVAL;
    if (prm->ee_neighbourhood < NB_TWO_OPT || prm->ee_neighbourhood > NB_NODE_SWAP) return OR_EINVAL;
    if (prm->mutation_swaps < 0 || prm->mutation_swaps > 65536) return OR_EINVAL;
    if (prm->velocity_cap < 0 || prm->velocity_cap > n) return OR_EINVAL;
    return OR_OK;
}

/* Initialisation: ceil(S * det_permille / 1000) particles start from
 * nearest-neighbour tours (starts spread evenly over the labels), the rest
 * from random shuffles; velocities are empty, personal bests are the
 * particles themselves and G is the best of them. */
int32_t or_init(const int32_t *D, const or_params *prm, or_state *st)
{
    int32_t n = st->n, S = st->S;
    if (or_check_params(prm, n) || S != prm->swarm_size || st->trace_cap < 1) return OR_EINVAL;
    int64_t m = ((int64_t)S * prm->det_permille + 999) / 1000;
    if (m > S) m = S;
    #pragma omp parallel for schedule(dynamic)
    for (int32_t p = 0; p < S; p++) {
        int32_t *x = row32(st->X, n, p);
        if (p < m)
            or_nn_tour(D, n, (int32_t)((int64_t)p * n / m), x);
        else
            or_fisher_yates(n, prm->seed, prm->instance, (uint64_t)p, 0, PURPOSE_INIT, x);
        st->VL[p] = 0;
        st->F[p] = or_tour_cost(D, n, x);
        memcpy(row32(st->P, n, p), x, sizeof(int32_t) * (size_t)n);
        st->FP[p] = st->F[p];
    }
    int32_t g = 0;
    for (int32_t p = 1; p < S; p++)
        if (st->FP[p] < st->FP[g]) g = p;
    memcpy(st->G, row32(st->P, n, g), sizeof(int32_t) * (size_t)n);
    st->FG = st->FP[g];
    st->t = 0; st->stall = 0;
    st->done = prm->max_generations == 0;
    st->trace[0] = st->FG;
    st->n_sweeps = st->n_moves = st->n_reshuffled = 0;
    return OR_OK;
}

/* Move of one particle (eq. velocity and eq. position), with the two
 * uniform draws given:
 *   b = P - x, c = G - x (both from the current x),
 *   y = x + w.v + phi1 r1.b + phi2 r2.c, the three prefixes applied in this
 *   order, then v <- y - x.
 * v holds lv transpositions on entry and the new velocity on exit; y
 * receives the new position. Returns the new velocity length. */
int32_t or_move_core(const int32_t *x, const int32_t *Pp, const int32_t *G, int32_t *v, int32_t lv,
                     int32_t n, uint32_t w_q16, uint32_t phi1_q16, uint32_t phi2_q16, uint32_t u1,
                     uint32_t u2, int32_t *y)
{
    int32_t *b = malloc(sizeof(int32_t) * 2 * (size_t)(n > 0 ? n : 1));
    int32_t *c = malloc(sizeof(int32_t) * 2 * (size_t)(n > 0 ? n : 1));
    int32_t lb = or_bss(x, Pp, n, b);
    int32_t lc = or_bss(x, G, n, c);
    int32_t k[3];
    or_truncate_counts(lv, lb, lc, w_q16, phi1_q16, phi2_q16, u1, u2, k);
    memcpy(y, x, sizeof(int32_t) * (size_t)n);
    or_apply_swaps(y, n, v, k[0]);
    or_apply_swaps(y, n, b, k[1]);
    or_apply_swaps(y, n, c, k[2]);
    int32_t lnew = or_bss(x, y, n, v);
    free(b); free(c);
    return lnew;
}

/* The same move with the velocity of eq. velocity kept as the raw
 * concatenation w.v (+) phi1 r1.b (+) phi2 r2.c of the three applied prefixes
 * (the operator (+) of Sect. 3.1) instead of being renormalised, truncated to
 * its first `cap` transpositions (cap <= n, so v holds it). */
int32_t or_move_core_raw(const int32_t *x, const int32_t *Pp, const int32_t *G, int32_t *v, int32_t lv,
                         int32_t n, uint32_t w_q16, uint32_t phi1_q16, uint32_t phi2_q16, uint32_t u1,
                         uint32_t u2, int32_t cap, int32_t *y)
{
    int32_t *b = malloc(sizeof(int32_t) * 2 * (size_t)(n > 0 ? n : 1));
    int32_t *c = malloc(sizeof(int32_t) * 2 * (size_t)(n > 0 ? n : 1));
    int32_t lb = or_bss(x, Pp, n, b);
    int32_t lc = or_bss(x, G, n, c);
    int32_t k[3];
    or_truncate_counts(lv, lb, lc, w_q16, phi1_q16, phi2_q16, u1, u2, k);
    memcpy(y, x, sizeof(int32_t) * (size_t)n);
    or_apply_swaps(y, n, v, k[0]);
    or_apply_swaps(y, n, b, k[1]);
    or_apply_swaps(y, n, c, k[2]);
    int32_t len = k[0] < cap ? k[0] : cap;   /* v already starts with its own prefix */
    for (int32_t a = 0; a < k[1] && len < cap; a++, len++) { v[2 * len] = b[2 * a]; v[2 * len + 1] = b[2 * a + 1]; }
    for (int32_t a = 0; a < k[2] && len < cap; a++, len++) { v[2 * len] = c[2 * a]; v[2 * len + 1] = c[2 * a + 1]; }
    free(b); free(c);
    return len;
}

/* Move of particle p at generation t: r1, r2 are the first two draws of the
 * particle's velocity stream for generation t; the personal best follows
 * when the new cost is strictly lower. */
void or_move_particle(const int32_t *D, const or_params *prm, or_state *st, int32_t p, int32_t t)
{
    int32_t n = st->n;
    int32_t *x = row32(st->X, n, p);
    int32_t *y = malloc(sizeof(int32_t) * (size_t)n);
    or_stream s;
    stream_open(&s, prm->seed, prm->instance, (uint64_t)p, (uint64_t)t, PURPOSE_VEL);
    uint32_t u1 = stream_next(&s), u2 = stream_next(&s);
    int32_t *v = st->V + (int64_t)p * n * 2;
    if (prm->velocity_cap > 0)
        st->VL[p] = or_move_core_raw(x, row32(st->P, n, p), st->G, v, st->VL[p], n, prm->w_q16,
                                     prm->phi1_q16, prm->phi2_q16, u1, u2, prm->velocity_cap, y);
    else
        st->VL[p] = or_move_core(x, row32(st->P, n, p), st->G, v, st->VL[p], n, prm->w_q16,
                                 prm->phi1_q16, prm->phi2_q16, u1, u2, y);
    memcpy(x, y, sizeof(int32_t) * (size_t)n);
    st->F[p] = or_tour_cost(D, n, x);
    pbest_rule(st, p);
    free(y);
}

static int32_t tours_equal(const int32_t *a, const int32_t *b, int32_t n)
{
    return memcmp(a, b, sizeof(int32_t) * (size_t)n) == 0;
}

static const int64_t *g_sort_F; /* sort key for mutation_order */
static int cmp_by_cost(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    if (g_sort_F[a] != g_sort_F[b]) return g_sort_F[a] < g_sort_F[b] ? -1 : 1;
    return (a > b) - (a < b);
}

/* Random mutation at generation t (Sect. 3.2.2; the pseudo code randomises the
 * worst two thirds): particles are ordered by (cost, index); a particle whose
 * tour equals that of an earlier particle of equal cost is a duplicate; the
 * first ceil(S/3) non-duplicates are kept and every other particle restarts
 * from a fresh shuffle (or, with mutation_swaps = k > 0, is disturbed by k
 * random position exchanges) with an empty velocity (its personal best is
 * kept and updated if the new tour is strictly better). kept[p] (optional)
 * receives 1 for kept particles. Returns the number of mutated particles. */
int32_t or_mutation(const int32_t *D, const or_params *prm, or_state *st, int32_t t, int32_t *kept)
{
    int32_t n = st->n, S = st->S;
    int32_t *order = malloc(sizeof(int32_t) * (size_t)S);
    char *dup = calloc((size_t)S, 1), *keep = calloc((size_t)S, 1);
    for (int32_t p = 0; p < S; p++) order[p] = p;
    g_sort_F = st->F;
    qsort(order, (size_t)S, sizeof(int32_t), cmp_by_cost);
    for (int32_t r = 1; r < S; r++) {
        int32_t p = order[r];
        for (int32_t r2 = r - 1; r2 >= 0 && st->F[order[r2]] == st->F[p]; r2--)
            if (tours_equal(row32(st->X, n, order[r2]), row32(st->X, n, p), n)) { dup[p] = 1; break; }
    }
    int32_t K = (S + 2) / 3, taken = 0;
    for (int32_t r = 0; r < S && taken < K; r++)
        if (!dup[order[r]]) { keep[order[r]] = 1; taken++; }
    int32_t reshuffled = 0;
    #pragma omp parallel for schedule(dynamic) reduction(+ : reshuffled)
    for (int32_t p = 0; p < S; p++) {
        if (keep[p]) continue;
        int32_t *x = row32(st->X, n, p);
        if (prm->mutation_swaps > 0)
            or_disturb(n, prm->mutation_swaps, prm->seed, prm->instance, (uint64_t)p, (uint64_t)t,
                       PURPOSE_MUT, x);
        else
            or_fisher_yates(n, prm->seed, prm->instance, (uint64_t)p, (uint64_t)t, PURPOSE_MUT, x);
        st->VL[p] = 0;
        st->F[p] = or_tour_cost(D, n, x);
        pbest_rule(st, p);
        reshuffled++;
    }
    if (kept)
        for (int32_t p = 0; p < S; p++) kept[p] = keep[p];
    free(order); free(dup); free(keep);
    return reshuffled;
}

/* One generation of the pseudo code: move every particle, mutate on every
 * mutation_period-th generation, update G, run the edge exchange when the
 * trigger asks for it (always, or when G did not improve), and count
 * generations without improvement. Returns 1 if G improved. */
int32_t or_generation(const int32_t *D, const or_params *prm, or_state *st)
{
    if (st->done) return 0;
    int32_t n = st->n, S = st->S, t = st->t + 1;
    if (t >= st->trace_cap) return OR_EINVAL;
    #pragma omp parallel for schedule(dynamic)
    for (int32_t p = 0; p < S; p++) or_move_particle(D, prm, st, p, t);
    if (prm->mutation_period > 0 && t % prm->mutation_period == 0)
        st->n_reshuffled += or_mutation(D, prm, st, t, NULL);
    int32_t improved = or_update_gbest(st);
    if (prm->ee_trigger == EE_ALWAYS || (prm->ee_trigger == EE_ON_STALL && !improved)) {
        int64_t sweeps = 0, moves = 0;
        #pragma omp parallel for schedule(dynamic) reduction(+ : sweeps, moves)
        for (int32_t p = 0; p < S; p++) {
            int64_t sw = 0;
            int32_t *x = row32(st->X, n, p);
            moves += prm->ee_neighbourhood == NB_NODE_SWAP
                         ? or_node_exchange(D, n, x, &st->F[p], prm->ee_max_moves, &sw)
                         : or_edge_exchange(D, n, x, &st->F[p], prm->ee_max_moves, &sw);
            sweeps += sw;
            pbest_rule(st, p);
        }
        st->n_sweeps += sweeps;
        st->n_moves += moves;
        improved |= or_update_gbest(st);
    }
    st->stall = improved ? 0 : st->stall + 1;
    st->t = t;
    st->trace[t] = st->FG;
    if (t >= prm->max_generations || (prm->stall_limit > 0 && st->stall >= prm->stall_limit))
        st->done = 1;
    return improved;
}

int32_t or_run(const int32_t *D, const or_params *prm, or_state *st, int32_t generations)
{
    if (or_check_params(prm, st->n) || st->S != prm->swarm_size) return OR_EINVAL;
    for (int32_t g = 0; g < generations && !st->done; g++) {
        int32_t r = or_generation(D, prm, st);
        if (r < 0) return r;
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Travelling costs between viewpoints (Sect. 2.2 and 2.3).
 * The UAV is kept clear of each box by inflating it by the clearance. A
 * straight flight between two points is allowed iff it misses the open
 * interior of every inflated box (touching a face, edge or corner is
 * allowed). The graph joins every pair of mutually visible nodes among the
 * viewpoints and the corners of the inflated boxes; an edge costs its
 * Euclidean length in mm rounded half up. The cost between two viewpoints is
 * the shortest path in this graph; an unreachable pair gets the very large
 * cost OR_D_INF.
 * ------------------------------------------------------------------------- */

/* Largest r with r*r <= s. */
static uint64_t isqrt_floor(uint64_t s)
{
    uint64_t r = (uint64_t)sqrt((double)s);
    while (r > 0 && r * r > s) r--;
    while ((r + 1) * (r + 1) <= s) r++;
    return r;
}

/* Euclidean length of (dx, dy, dz) rounded half up: r + 1 iff
 * sqrt(s) >= r + 1/2, i.e. 4s >= (2r + 1)^2. */
int64_t or_round_len(int64_t dx, int64_t dy, int64_t dz)
{
    uint64_t s = (uint64_t)(dx * dx) + (uint64_t)(dy * dy) + (uint64_t)(dz * dz);
    uint64_t r = isqrt_floor(s);
    if (4 * s >= (2 * r + 1) * (2 * r + 1)) r++;
    return (int64_t)r;
}

/* p/q < r/s for q, s > 0 */
static int frac_lt(int64_t p, int64_t q, int64_t r, int64_t s) { return p * s < r * q; }

/* Does the closed segment A->B meet the open box (L, H)? Points of the
 * segment are A + t (B - A), 0 <= t <= 1; per axis the open box admits an
 * open interval of t; the segment meets the box iff the intersection of the
 * three intervals with [0, 1] is not empty. */
int32_t or_segment_hits_box(const int64_t A[3], const int64_t B[3], const int64_t L[3],
                            const int64_t H[3])
{
    int64_t lo_p = -1, lo_q = 1, hi_p = 2, hi_q = 1; /* start from (-1, 2) */
    for (int a = 0; a < 3; a++) {
        int64_t d = B[a] - A[a];
        if (d == 0) {
            if (!(L[a] < A[a] && A[a] < H[a])) return 0;
            continue;
        }
        int64_t ep, eq, fp, fq; /* entry and exit parameters ep/eq, fp/fq */
        if (d > 0) { ep = L[a] - A[a]; fp = H[a] - A[a]; eq = fq = d; }
        else       { ep = A[a] - H[a]; fp = A[a] - L[a]; eq = fq = -d; }
        if (frac_lt(lo_p, lo_q, ep, eq)) { lo_p = ep; lo_q = eq; }
        if (frac_lt(fp, fq, hi_p, hi_q)) { hi_p = fp; hi_q = fq; }
    }
    return frac_lt(lo_p, lo_q, hi_p, hi_q) && lo_p < lo_q && hi_p > 0;
}

/* ---------------------------------------------------------------------------
 * Voxel-grid planner (Sect. 2.2): the workspace is divided into voxels of
 * edge s; a voxel is occupied when its centre lies in the open interior of a
 * box, and every voxel whose centre is within the UAV's size (the clearance)
 * of an occupied centre is marked occupied too. A path moves between the 26
 * neighbouring voxels; a step (alpha, beta, gamma) in {-1, 0, 1}^3 costs
 * L = a1 alpha^2 + a2 beta^2 + a3 gamma^2 (eq. cost). It passes through free
 * voxels only; its two end voxels (the viewpoints') may be occupied. The
 * travelling cost of a pair is s times the least total step cost (the
 * shortest path the A* search of the paper looks for); OR_D_INF when there is
 * none.
 *
 * Grid: origin = (smallest coordinate of the viewpoints and box corners) - s
 * per axis, dims = (largest - origin) / s + 2, voxel i covers
 * [origin + i s, origin + (i+1) s).
 * ------------------------------------------------------------------------- */
int32_t or_voxel_grid(const int32_t *vp, int32_t n, const int32_t *boxes, int32_t nb, int32_t clearance,
                      int32_t s, int32_t *dims, int64_t *origin, uint8_t *occ)
{
    if (n < 1 || nb < 0 || clearance < 0 || s < 1 || !vp || (nb > 0 && !boxes)) return OR_EINVAL;
    int64_t lo[3], hi[3];
    for (int a = 0; a < 3; a++) lo[a] = hi[a] = vp[a];
    for (int32_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            if (vp[3 * i + a] < lo[a]) lo[a] = vp[3 * i + a];
            if (vp[3 * i + a] > hi[a]) hi[a] = vp[3 * i + a];
        }
    for (int32_t b = 0; b < nb; b++)
        for (int a = 0; a < 3; a++) {
            if (boxes[6 * b + a] > boxes[6 * b + 3 + a]) return OR_EINVAL;
            if (boxes[6 * b + a] < lo[a]) lo[a] = boxes[6 * b + a];
            if (boxes[6 * b + 3 + a] > hi[a]) hi[a] = boxes[6 * b + 3 + a];
        }
    int64_t G = 1;
    for (int a = 0; a < 3; a++) {
        origin[a] = lo[a] - s;
        int64_t d = (hi[a] - origin[a]) / s + 2;
        if (d > (1 << 20)) return OR_ERANGE;
        dims[a] = (int32_t)d;
        G *= d;
    }
    if (G > ((int64_t)1 << 26)) return OR_ERANGE;
    if (!occ) return OR_OK;
    uint8_t *core = calloc((size_t)G, 1);
    if (!core) return OR_ENOMEM;
    for (int64_t v = 0; v < G; v++) {
        int64_t idx[3] = {v % dims[0], (v / dims[0]) % dims[1], v / ((int64_t)dims[0] * dims[1])};
        for (int32_t b = 0; b < nb && !core[v]; b++) {
            int inside = 1;
            for (int a = 0; a < 3; a++) {
                int64_t c2 = 2 * origin[a] + (2 * idx[a] + 1) * s;   /* twice the centre */
                if (!(2 * (int64_t)boxes[6 * b + a] < c2 && c2 < 2 * (int64_t)boxes[6 * b + 3 + a])) inside = 0;
            }
            core[v] = (uint8_t)inside;
        }
    }
    int64_t R = clearance / s, r2 = (int64_t)clearance * clearance;
    for (int64_t v = 0; v < G; v++) {
        int64_t idx[3] = {v % dims[0], (v / dims[0]) % dims[1], v / ((int64_t)dims[0] * dims[1])};
        uint8_t o = 0;
        for (int64_t dk = -R; dk <= R && !o; dk++)
            for (int64_t dj = -R; dj <= R && !o; dj++)
                for (int64_t di = -R; di <= R && !o; di++) {
                    if ((di * di + dj * dj + dk * dk) * s * s > r2) continue;
                    int64_t i = idx[0] + di, j = idx[1] + dj, k = idx[2] + dk;
                    if (i < 0 || j < 0 || k < 0 || i >= dims[0] || j >= dims[1] || k >= dims[2]) continue;
                    o = core[i + dims[0] * (j + (int64_t)dims[1] * k)];
                }
        occ[v] = o;
    }
    free(core);
    return OR_OK;
}

typedef struct { int64_t d; int64_t v; } heap_item;

static void heap_push(heap_item *h, int64_t *len, heap_item it)
{
    int64_t i = (*len)++;
    h[i] = it;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= h[i].d) break;
        heap_item t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static heap_item heap_pop(heap_item *h, int64_t *len)
{
    heap_item top = h[0];
    h[0] = h[--(*len)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *len && h[l].d < h[m].d) m = l;
        if (r < *len && h[r].d < h[m].d) m = r;
        if (m == i) break;
        heap_item t = h[m]; h[m] = h[i]; h[i] = t;
        i = m;
    }
    return top;
}

int32_t or_build_dist_voxel(const int32_t *vp, int32_t n, const int32_t *boxes, int32_t nb, int32_t clearance,
                            int32_t s, int32_t a1, int32_t a2, int32_t a3, int32_t *D)
{
    if (!D || a1 < 1 || a2 < 1 || a3 < 1 || a1 > (1 << 20) || a2 > (1 << 20) || a3 > (1 << 20)) return OR_EINVAL;
    int32_t dims[3];
    int64_t origin[3];
    int32_t st = or_voxel_grid(vp, n, boxes, nb, clearance, s, dims, origin, NULL);
    if (st) return st;
    const int64_t G = (int64_t)dims[0] * dims[1] * dims[2];
    uint8_t *occ = malloc((size_t)G);
    int64_t *vox = malloc(sizeof(int64_t) * (size_t)n);
    if (!occ || !vox) { free(occ); free(vox); return OR_ENOMEM; }
    or_voxel_grid(vp, n, boxes, nb, clearance, s, dims, origin, occ);
    for (int32_t i = 0; i < n; i++) {
        int64_t id[3];
        for (int a = 0; a < 3; a++) id[a] = ((int64_t)vp[3 * i + a] - origin[a]) / s;
        vox[i] = id[0] + dims[0] * (id[1] + (int64_t)dims[1] * id[2]);
    }
    const int32_t wgt[3] = {a1, a2, a3};
    int32_t status = OR_OK;
    #pragma omp parallel for schedule(dynamic)
    for (int32_t src = 0; src < n; src++) {
        int64_t *dist = malloc(sizeof(int64_t) * (size_t)G);
        heap_item *heap = malloc(sizeof(heap_item) * (size_t)(27 * G + 1));
        int64_t hl = 0;
        for (int64_t v = 0; v < G; v++) dist[v] = INT64_MAX;
        dist[vox[src]] = 0;
        heap_push(heap, &hl, (heap_item){0, vox[src]});
        while (hl > 0) {
            heap_item it = heap_pop(heap, &hl);
            int64_t u = it.v;
            if (it.d != dist[u]) continue;            /* stale entry */
            if (occ[u] && u != vox[src]) continue;    /* an occupied end voxel: not passed through */
            int64_t ui = u % dims[0], uj = (u / dims[0]) % dims[1], uk = u / ((int64_t)dims[0] * dims[1]);
            for (int dk = -1; dk <= 1; dk++)
                for (int dj = -1; dj <= 1; dj++)
                    for (int di = -1; di <= 1; di++) {
                        if (!di && !dj && !dk) continue;
                        int64_t i = ui + di, j = uj + dj, k = uk + dk;
                        if (i < 0 || j < 0 || k < 0 || i >= dims[0] || j >= dims[1] || k >= dims[2]) continue;
                        int64_t v = i + dims[0] * (j + (int64_t)dims[1] * k);
                        int64_t nd = it.d + (int64_t)wgt[0] * di * di + (int64_t)wgt[1] * dj * dj +
                                     (int64_t)wgt[2] * dk * dk;
                        if (nd < dist[v]) { dist[v] = nd; heap_push(heap, &hl, (heap_item){nd, v}); }
                    }
        }
        for (int32_t j = 0; j < n; j++) {
            int64_t d = dist[vox[j]];
            if (d == INT64_MAX) { D[(int64_t)src * n + j] = OR_D_INF; continue; }
            d *= s;
            if (d >= OR_D_INF) {
                #pragma omp critical
                status = OR_ERANGE;
                d = OR_D_INF;
            }
            D[(int64_t)src * n + j] = (int32_t)d;
        }
        free(dist); free(heap);
    }
    free(occ); free(vox);
    return status;
}

int32_t or_build_dist(const int32_t *vp, int32_t n, const int32_t *boxes, int32_t nb,
                      int32_t clearance, int32_t *D)
{
    if (n < 1 || n > 65535 || nb < 0 || clearance < 0 || !vp || !D || (nb > 0 && !boxes))
        return OR_EINVAL;
    const int64_t LIM = (int64_t)1 << 26;
    for (int64_t i = 0; i < 3 * (int64_t)n; i++)
        if (vp[i] <= -LIM || vp[i] >= LIM) return OR_ERANGE;
    for (int32_t b = 0; b < nb; b++)
        for (int a = 0; a < 3; a++) {
            if (boxes[6 * b + a] > boxes[6 * b + 3 + a]) return OR_EINVAL;
            if ((int64_t)boxes[6 * b + a] - clearance <= -LIM || (int64_t)boxes[6 * b + 3 + a] + clearance >= LIM)
                return OR_ERANGE;
        }
    int32_t V = n + 8 * nb;
    int64_t *node = malloc(sizeof(int64_t) * 3 * (size_t)V);
    int64_t *L = malloc(sizeof(int64_t) * 3 * (size_t)(nb > 0 ? nb : 1));
    int64_t *H = malloc(sizeof(int64_t) * 3 * (size_t)(nb > 0 ? nb : 1));
    int64_t *W = malloc(sizeof(int64_t) * (size_t)V * (size_t)V);
    if (!node || !L || !H || !W) { free(node); free(L); free(H); free(W); return OR_ENOMEM; }
    for (int32_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) node[3 * i + a] = vp[3 * i + a];
    for (int32_t b = 0; b < nb; b++) {
        for (int a = 0; a < 3; a++) {
            L[3 * b + a] = (int64_t)boxes[6 * b + a] - clearance;
            H[3 * b + a] = (int64_t)boxes[6 * b + 3 + a] + clearance;
        }
        for (int c = 0; c < 8; c++)
            for (int a = 0; a < 3; a++)
                node[3 * (n + 8 * b + c) + a] = (c >> a) & 1 ? H[3 * b + a] : L[3 * b + a];
    }
    const int64_t NONE = INT64_MAX;
    #pragma omp parallel for schedule(dynamic)
    for (int32_t u = 0; u < V; u++) {
        W[(int64_t)u * V + u] = 0;
        for (int32_t v = u + 1; v < V; v++) {
            int free_path = 1;
            for (int32_t b = 0; b < nb && free_path; b++)
                if (or_segment_hits_box(&node[3 * u], &node[3 * v], &L[3 * b], &H[3 * b])) free_path = 0;
            int64_t w = free_path ? or_round_len(node[3 * v] - node[3 * u], node[3 * v + 1] - node[3 * u + 1],
                                                 node[3 * v + 2] - node[3 * u + 2])
                                  : NONE;
            W[(int64_t)u * V + v] = w;
            W[(int64_t)v * V + u] = w;
        }
    }
    int32_t status = OR_OK;
    #pragma omp parallel for schedule(dynamic)
    for (int32_t src = 0; src < n; src++) {
        /* Dijkstra with an array scan: settle the closest unsettled node. */
        int64_t *dist = malloc(sizeof(int64_t) * (size_t)V);
        char *done = calloc((size_t)V, 1);
        for (int32_t v = 0; v < V; v++) dist[v] = NONE;
        dist[src] = 0;
        for (;;) {
            int32_t u = -1;
            for (int32_t v = 0; v < V; v++)
                if (!done[v] && dist[v] != NONE && (u < 0 || dist[v] < dist[u])) u = v;
            if (u < 0) break;
            done[u] = 1;
            for (int32_t v = 0; v < V; v++) {
                int64_t w = W[(int64_t)u * V + v];
                if (!done[v] && w != NONE && dist[u] + w < dist[v]) dist[v] = dist[u] + w;
            }
        }
        for (int32_t j = 0; j < n; j++) {
            int64_t d = dist[j];
            if (d == NONE) d = OR_D_INF;
            else if (d >= OR_D_INF) {
                #pragma omp atomic write
                status = OR_ERANGE;
                d = OR_D_INF;
            }
            D[(int64_t)src * n + j] = (int32_t)d;
        }
        free(dist); free(done);
    }
    free(node); free(L); free(H); free(W);
    return status;
}
