/*
 * amber_oracle.c -- reference CPU implementation of the columnar ABM step
 * (TEST INFRASTRUCTURE ONLY).
 *
 * This file is the oracle that the HIP path is checked against.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It is deliberately plain, single threaded and slow: every random word
 * is produced by a full Philox block, every step copies whole columns, and
 * nothing is fused or reordered beyond what the model definitions state.
 * It shares no code, header or table with the GPU library.
 *
 * What it computes (paper: "AMBER: A Columnar Architecture for Scalable
 * Agent-Based Modelling in Python", arXiv 2601.16292):
 *   - columnar state: one typed array per agent attribute, agents are the
 *     sequential ids 0..N-1 (Sec. 3.1.1, "Columnar State Management");
 *   - synchronous (snapshot) update semantics: every agent reads the state
 *     at the start of the step (Sec. 3.4, "State Evolution Semantics");
 *   - wealth transfer: agents with positive wealth give one unit to a random
 *     recipient; duplicate recipients accumulate, as the scatter-add view
 *     does (Sec. 3.1.1 filtered-view and scatter-add listings; Sec. 3.3;
 *     Sec. 5.1.2 "Benchmark Models");
 *   - random walk on a torus grid with the 8 Moore moves (Sec. 4.1 grid
 *     environment; Sec. 5.1.2, reformulated on the grid);
 *   - spatial SIR on the same grid: move, count infected agents in the
 *     3x3 Moore block of cells, infect with 1-(1-beta)^k, recover with
 *     gamma (Sec. 5.1.2, reformulated on the grid; torus-wrap neighbour
 *     deduplication per Sec. 6.1);
 *   - the invariant checks of Sec. 5.1.3 / Sec. 6.2.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * Random Numbers: As Easy as 1, 2, 3", SC'11), keyed (seed, stream), with
 * counter (floor(g/4), t, purpose, 0) and word g mod 4, g = a*W + j.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- Philox */

/* One Philox4x32-10 block: 10 rounds; the key is bumped between rounds,
 * the first round uses the key as given. */
void orc_philox4x32_10(const uint32_t ctr_in[4], uint32_t k0, uint32_t k1,
                       uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Purposes of the random stream and their words per agent. */
enum { P_INIT_POS = 0, P_MOVE = 1, P_EPI = 2, P_RECIPIENT = 3, P_ORDER = 4, P_STEP = 5 };

/* Word j of agent a for purpose p at step t. */
uint32_t orc_word(uint32_t seed, uint32_t stream, uint32_t purpose,
                  uint32_t words_per_agent, uint32_t t, uint32_t a, uint32_t j)
{
    uint64_t g = (uint64_t)a * words_per_agent + j;
    uint32_t ctr[4] = { (uint32_t)(g / 4), t, purpose, 0 };
    uint32_t out[4];
    orc_philox4x32_10(ctr, seed, stream, out);
    return out[g % 4];
}

/* ------------------------------------------------------ integer mappings */

/* Uniform grid coordinate in [0, L): floor(u * L / 2^32). */
static uint32_t grid_coord(uint32_t u, uint32_t L)
{
    return (uint32_t)(((uint64_t)u * L) >> 32);
}

/* Uniform recipient in [0, N): floor(U * N / 2^64), U = hi:lo. */
static uint32_t recipient_of(uint32_t hi, uint32_t lo, uint32_t n)
{
    unsigned __int128 U = ((unsigned __int128)hi << 32) | lo;
    return (uint32_t)((U * n) >> 64);
}

/* The 8 Moore moves, in this fixed order, indexed by the top 3 bits. */
static const int MOVE_DX[8] = { -1, -1, -1,  0, 0,  1, 1, 1 };
static const int MOVE_DY[8] = { -1,  0,  1, -1, 1, -1, 0, 1 };

static int32_t torus(int64_t v, uint32_t L)
{
    int64_t m = v % (int64_t)L;
    if (m < 0) m += L;
    return (int32_t)m;
}

/* ------------------------------------------------------------ init */

void orc_init_wealth(uint32_t n, int32_t w_init, int32_t *w)
{
    for (uint32_t a = 0; a < n; a++) w[a] = w_init;
}

void orc_init_positions(uint32_t n, uint32_t L, uint32_t seed, uint32_t stream,
                        int32_t *x, int32_t *y)
{
    for (uint32_t a = 0; a < n; a++) {
        x[a] = (int32_t)grid_coord(orc_word(seed, stream, P_INIT_POS, 2, 0, a, 0), L);
        y[a] = (int32_t)grid_coord(orc_word(seed, stream, P_INIT_POS, 2, 0, a, 1), L);
    }
}

void orc_init_states(uint32_t n, uint32_t i0, uint8_t *s)
{
    for (uint32_t a = 0; a < n; a++) s[a] = (a < i0) ? 1 : 0;
}

/* ------------------------------------------------------------ wealth */

/* Recipient draw of agent a at step t. */
uint32_t orc_recipient(uint32_t n, uint32_t seed, uint32_t stream, uint32_t t,
                       uint32_t a)
{
    uint32_t hi = orc_word(seed, stream, P_RECIPIENT, 2, t, a, 0);
    uint32_t lo = orc_word(seed, stream, P_RECIPIENT, 2, t, a, 1);
    return recipient_of(hi, lo, n);
}

/* Apply one synchronous transfer round given each agent's recipient:
 * donors are the agents with w > 0 in the snapshot; each donor loses one
 * unit and its recipient gains one (duplicates accumulate).  recip[a] is
 * read only for donors.  new_w is scratch of length n. */
void orc_wealth_apply(uint32_t n, int32_t *w, const uint32_t *recip,
                      int32_t *new_w)
{
    memcpy(new_w, w, (size_t)n * sizeof(int32_t));
    for (uint32_t a = 0; a < n; a++) {
        if (w[a] > 0) {
            new_w[a] -= 1;
            new_w[recip[a]] += 1;
        }
    }
    memcpy(w, new_w, (size_t)n * sizeof(int32_t));
}

/* One wealth-transfer step t.  scratch: n uint32 + n int32. */
void orc_wealth_step(uint32_t n, uint32_t seed, uint32_t stream, uint32_t t,
                     int32_t *w, uint32_t *recip_scratch, int32_t *w_scratch)
{
    for (uint32_t a = 0; a < n; a++)
        recip_scratch[a] = (w[a] > 0) ? orc_recipient(n, seed, stream, t, a) : 0;
    orc_wealth_apply(n, w, recip_scratch, w_scratch);
}

/* ------------------------------------------------------------ random walk */

/* Move agent a one Moore step at step t, wrapping on the L x L torus. */
static void move_agent(uint32_t L, uint32_t seed, uint32_t stream, uint32_t t,
                       uint32_t a, int32_t *x, int32_t *y)
{
    uint32_t d = orc_word(seed, stream, P_MOVE, 1, t, a, 0) >> 29;
    x[a] = torus((int64_t)x[a] + MOVE_DX[d], L);
    y[a] = torus((int64_t)y[a] + MOVE_DY[d], L);
}

void orc_walk_step(uint32_t n, uint32_t L, uint32_t seed, uint32_t stream,
                   uint32_t t, int32_t *x, int32_t *y)
{
    for (uint32_t a = 0; a < n; a++) move_agent(L, seed, stream, t, a, x, y);
}

/* ------------------------------------------------------------ SIR */

enum { S_SUS = 0, S_INF = 1, S_REC = 2 };

/* Number of infected agents in the distinct cells of the 3x3 torus block
 * around (cx, cy), given per-cell infected counts C (row-major, c = y*L+x).
 * When L < 3 wrapped neighbours coincide and each distinct cell counts once. */
uint64_t orc_neighbour_infected(uint32_t L, const uint32_t *C, int32_t cx, int32_t cy)
{
    uint64_t cells[9];
    int nc = 0;
    for (int dx = -1; dx <= 1; dx++) {
        for (int dy = -1; dy <= 1; dy++) {
            uint64_t c = (uint64_t)torus((int64_t)cy + dy, L) * L
                       + (uint64_t)torus((int64_t)cx + dx, L);
            int seen = 0;
            for (int i = 0; i < nc; i++) if (cells[i] == c) seen = 1;
            if (!seen) cells[nc++] = c;
        }
    }
    uint64_t k = 0;
    for (int i = 0; i < nc; i++) k += C[cells[i]];
    return k;
}

/* One SIR step t.
 *   1. every agent moves exactly as in the random walk;
 *   2. C[c] = number of agents infected at the start of the step whose
 *      post-move cell is c;
 *   3. a susceptible agent with k infected in its distinct 3x3 block becomes
 *      infected iff its EPI word u < T_inf[min(k, k_sat)] (k >= 1);
 *      an infected agent recovers iff u < T_rec; recovered stays recovered.
 * C is scratch of L*L uint32; s_new is scratch of n bytes. */
void orc_sir_step(uint32_t n, uint32_t L, uint32_t seed, uint32_t stream,
                  uint32_t t, int32_t *x, int32_t *y, uint8_t *s,
                  const uint32_t *t_inf, uint32_t k_sat, uint32_t t_rec,
                  uint32_t *C, uint8_t *s_new)
{
    for (uint32_t a = 0; a < n; a++) move_agent(L, seed, stream, t, a, x, y);

    memset(C, 0, (size_t)L * L * sizeof(uint32_t));
    for (uint32_t a = 0; a < n; a++)
        if (s[a] == S_INF) C[(uint64_t)y[a] * L + x[a]] += 1;

    for (uint32_t a = 0; a < n; a++) {
        s_new[a] = s[a];
        if (s[a] == S_SUS) {
            uint64_t k = orc_neighbour_infected(L, C, x[a], y[a]);
            if (k >= 1) {
                uint32_t u = orc_word(seed, stream, P_EPI, 1, t, a, 0);
                uint64_t kk = k < k_sat ? k : k_sat;
                if (u < t_inf[kk]) s_new[a] = S_INF;
            }
        } else if (s[a] == S_INF) {
            uint32_t u = orc_word(seed, stream, P_EPI, 1, t, a, 0);
            if (u < t_rec) s_new[a] = S_REC;
        }
    }
    memcpy(s, s_new, n);
}

/* ------------------------------------------------------------ checks */

/* SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA'14). */
static uint64_t fmix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* The finaliser alone, exported so that tests can pin it to SplitMix64's
 * published outputs (the generator's k-th output is the finaliser applied
 * to k times its increment 0x9E3779B97F4A7C15). */
uint64_t orc_fmix64(uint64_t z)
{
    return fmix64(z);
}

/* Order-free digest of a population: sum over agents (mod 2^64) of
 * h_a, where h = fmix64(a) and then, for each column value v_j of the row
 * in column order, h = fmix64(h ^ ((j+1) << 32 | v_j)). */
uint64_t orc_digest(uint32_t n, uint32_t ncols, const uint32_t *const *cols,
                    const uint32_t *widths)
{
    uint64_t acc = 0;
    for (uint32_t a = 0; a < n; a++) {
        uint64_t h = fmix64((uint64_t)a);
        for (uint32_t j = 0; j < ncols; j++) {
            uint32_t v;
            if (widths[j] == 1) v = ((const uint8_t *)cols[j])[a];
            else v = cols[j][a];
            h = fmix64(h ^ (((uint64_t)(j + 1) << 32) | v));
        }
        acc += h;
    }
    return acc;
}

/* Invariants of Sec. 5.1.3 plus bookkeeping.  Any column may be NULL.
 * out_of_bounds counts rows outside the model's domain: negative wealth,
 * coordinates outside [0, L), or a state code above 2. */
typedef struct {
    int64_t  wealth_sum;
    int32_t  wealth_min;
    uint64_t n_s, n_i, n_r;
    uint64_t out_of_bounds;
} orc_invariants_t;

void orc_invariants(uint32_t n, uint32_t L, const int32_t *w, const int32_t *x,
                    const int32_t *y, const uint8_t *s, orc_invariants_t *out)
{
    memset(out, 0, sizeof(*out));
    out->wealth_min = INT32_MAX;
    for (uint32_t a = 0; a < n; a++) {
        int bad = 0;
        if (w) {
            out->wealth_sum += w[a];
            if (w[a] < out->wealth_min) out->wealth_min = w[a];
            if (w[a] < 0) bad = 1;
        }
        if (x && (x[a] < 0 || (uint32_t)x[a] >= L)) bad = 1;
        if (y && (y[a] < 0 || (uint32_t)y[a] >= L)) bad = 1;
        if (s) {
            if (s[a] == S_SUS) out->n_s++;
            else if (s[a] == S_INF) out->n_i++;
            else if (s[a] == S_REC) out->n_r++;
            else bad = 1;
        }
        out->out_of_bounds += bad;
    }
    if (!w) out->wealth_min = 0;
}

/* ------------------------------------------------------ view primitives */

/* The three views of Sec. 3.3 on one typed column of n rows, written as the
 * plain definitions (Sec. 3.1.1 listings):
 *   full view      every row:            v <- a*v + b
 *   filtered view  rows where p CMP thr: v <- a*v + b, the predicate read on
 *                  the column values before the update (snapshot)
 *   scatter view   for j = 0..m-1 in list order: col[ids[j]] += vals[j]
 *                  (duplicates accumulate, as numpy's add.at does); ids
 *                  outside [0, n) are skipped.
 * int32 arithmetic wraps modulo 2^32; float32 updates are the fused
 * multiply-add a*v + b with one rounding to nearest, and float32 scatter
 * adds round after every addition, in list order. */

enum { ORC_LT = 0, ORC_LE = 1, ORC_EQ = 2, ORC_NE = 3, ORC_GE = 4, ORC_GT = 5 };

static int cmp_i32(int32_t v, int cmp, int32_t thr)
{
    switch (cmp) {
    case ORC_LT: return v < thr;
    case ORC_LE: return v <= thr;
    case ORC_EQ: return v == thr;
    case ORC_NE: return v != thr;
    case ORC_GE: return v >= thr;
    case ORC_GT: return v > thr;
    }
    return 0;
}

static int cmp_f32(float v, int cmp, float thr)
{
    switch (cmp) {
    case ORC_LT: return v < thr;
    case ORC_LE: return v <= thr;
    case ORC_EQ: return v == thr;
    case ORC_NE: return v != thr;
    case ORC_GE: return v >= thr;
    case ORC_GT: return v > thr;
    }
    return 0;
}

static int32_t affine_i32(int32_t v, int32_t a, int32_t b)
{
    return (int32_t)((uint32_t)a * (uint32_t)v + (uint32_t)b);
}

/* pred: NULL = full view; pred_f32 says which of pred_i / pred_f is the
 * predicate column (it may be the updated column itself). */
void orc_view_update_i32(uint64_t n, int32_t *col, int32_t a, int32_t b,
                         const int32_t *pred_i, const float *pred_f, int cmp,
                         int32_t thr_i, float thr_f)
{
    unsigned char *take = malloc(n ? n : 1);
    if (!take) return;
    for (uint64_t r = 0; r < n; r++)
        take[r] = pred_i ? cmp_i32(pred_i[r], cmp, thr_i)
                         : pred_f ? cmp_f32(pred_f[r], cmp, thr_f) : 1;
    for (uint64_t r = 0; r < n; r++)
        if (take[r]) col[r] = affine_i32(col[r], a, b);
    free(take);
}

void orc_view_update_f32(uint64_t n, float *col, float a, float b,
                         const int32_t *pred_i, const float *pred_f, int cmp,
                         int32_t thr_i, float thr_f)
{
    unsigned char *take = malloc(n ? n : 1);
    if (!take) return;
    for (uint64_t r = 0; r < n; r++)
        take[r] = pred_i ? cmp_i32(pred_i[r], cmp, thr_i)
                         : pred_f ? cmp_f32(pred_f[r], cmp, thr_f) : 1;
    for (uint64_t r = 0; r < n; r++)
        if (take[r]) col[r] = fmaf(a, col[r], b);
    free(take);
}

/* vals NULL: every entry adds *scalar. */
void orc_view_scatter_add_i32(uint64_t n, int32_t *col, uint64_t m, const uint32_t *ids,
                              const int32_t *vals, int32_t scalar)
{
    for (uint64_t j = 0; j < m; j++) {
        if (ids[j] >= n) continue;
        col[ids[j]] = (int32_t)((uint32_t)col[ids[j]] + (uint32_t)(vals ? vals[j] : scalar));
    }
}

void orc_view_scatter_add_f32(uint64_t n, float *col, uint64_t m, const uint32_t *ids,
                              const float *vals, float scalar)
{
    for (uint64_t j = 0; j < m; j++) {
        if (ids[j] >= n) continue;
        col[ids[j]] = col[ids[j]] + (vals ? vals[j] : scalar);
    }
}

/* Buffered per-agent writes (Sec. 3.2.1: record / update_data calls are kept
 * in a pending-writes dictionary keyed by agent and flushed once per step by
 * one update on id): the log entries j = 0..m-1 are applied in log order,
 * col[ids[j]] = vals[j], so the last write to an id is the one that stays;
 * ids outside [0, n) are skipped.  Values are copied bit for bit (either
 * dtype: 4-byte words). */
void orc_view_write_log(uint64_t n, uint32_t *col, uint64_t m, const uint32_t *ids,
                        const uint32_t *vals)
{
    for (uint64_t j = 0; j < m; j++)
        if (ids[j] < n) col[ids[j]] = vals[j];
}

/* ------------------------------------------------- asynchronous semantics */

/* Asynchronous (sequential) updates (Sec. 3.4): within a step the agents act
 * one after another and each sees what the agents before it did.  The order
 * of step t is a random permutation: agents sorted by (ORDER word, id),
 * where agent a's ORDER word is word(seed, stream, ORDER, 1, t, a, 0).
 * Wealth transfer under this semantics: in that order, an agent whose
 * current wealth is positive gives one unit to its recipient (the same
 * RECIPIENT draw as the synchronous model). */
typedef struct { uint32_t key, id; } orc_order_t;

static int order_cmp(const void *pa, const void *pb)
{
    const orc_order_t *a = pa, *b = pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

/* The permutation of step t: out[i] = the i-th agent to act. */
int orc_async_order(uint32_t n, uint32_t seed, uint32_t stream, uint32_t t, uint32_t *out)
{
    orc_order_t *o = malloc((size_t)(n ? n : 1) * sizeof(orc_order_t));
    if (!o) return -1;
    for (uint32_t a = 0; a < n; a++) {
        o[a].key = orc_word(seed, stream, P_ORDER, 1, t, a, 0);
        o[a].id = a;
    }
    qsort(o, n, sizeof(orc_order_t), order_cmp);
    for (uint32_t i = 0; i < n; i++) out[i] = o[i].id;
    free(o);
    return 0;
}

int orc_run_wealth_async(uint32_t n, uint32_t seed, uint32_t stream, uint32_t t0,
                         uint32_t n_steps, int32_t *w)
{
    uint32_t *order = malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    if (!order) return -1;
    for (uint32_t t = t0; t < t0 + n_steps; t++) {
        if (orc_async_order(n, seed, stream, t, order) != 0) { free(order); return -1; }
        for (uint32_t i = 0; i < n; i++) {
            const uint32_t a = order[i];
            if (w[a] > 0) {
                w[a] -= 1;
                w[orc_recipient(n, seed, stream, t, a)] += 1;
            }
        }
    }
    free(order);
    return 0;
}

/* ---------------------------------------------------- spatial environments */

/* Environments of Sec. 4.1: grid lattices of ndim <= 4 dimensions (cell of
 * coordinates c_0..c_{d-1} is sum c_i * stride_i with stride_0 = 1 and
 * stride_i = stride_{i-1} * dims_{i-1}; in 2-D that is y * L + x) with Moore
 * or von Neumann neighbourhoods, torus-wrapped or bounded, and networks
 * given as adjacency lists (CSR: the neighbours of node i are
 * col[row[i] .. row[i+1]-1]). */

static int cell_of(uint32_t ndim, const uint32_t *dims, const int32_t *const *pos, uint64_t a,
                   uint64_t *cell)
{
    uint64_t c = 0, stride = 1;
    for (uint32_t i = 0; i < ndim; i++) {
        const int32_t v = pos[i][a];
        if (v < 0 || (uint32_t)v >= dims[i]) return 0;
        c += (uint64_t)v * stride;
        stride *= dims[i];
    }
    *cell = c;
    return 1;
}

/* counts[c] = number of agents a with state[a] == match (every agent when
 * state is NULL) whose position is cell c; agents off the lattice are not
 * counted.  counts is overwritten. */
void orc_grid_count(uint32_t ndim, const uint32_t *dims, uint64_t n, const int32_t *const *pos,
                    const uint8_t *state, uint32_t match, uint32_t *counts)
{
    uint64_t cells = 1;
    for (uint32_t i = 0; i < ndim; i++) cells *= dims[i];
    memset(counts, 0, cells * sizeof(uint32_t));
    for (uint64_t a = 0; a < n; a++) {
        uint64_t c;
        if (state && state[a] != match) continue;
        if (cell_of(ndim, dims, pos, a, &c)) counts[c] += 1;
    }
}

/* out[c] = sum of counts over the distinct cells of c's neighbourhood, c
 * itself included: Moore (every offset in {-1,0,1}^d) or von Neumann (the
 * offsets with |o_0| + ... + |o_{d-1}| <= 1).  torus: coordinates wrap, and
 * a cell reached by two offsets (a side below 3) counts once; bounded:
 * offsets that leave the lattice are dropped. */
void orc_grid_neighbour_sum(uint32_t ndim, const uint32_t *dims, int von_neumann, int torus_wrap,
                            const uint32_t *counts, uint32_t *out)
{
    uint64_t cells = 1;
    for (uint32_t i = 0; i < ndim; i++) cells *= dims[i];
    uint32_t noff = 1;
    for (uint32_t i = 0; i < ndim; i++) noff *= 3;
    for (uint64_t c = 0; c < cells; c++) {
        int64_t co[4];
        uint64_t rest = c;
        for (uint32_t i = 0; i < ndim; i++) {
            co[i] = (int64_t)(rest % dims[i]);
            rest /= dims[i];
        }
        uint64_t seen[81];
        uint32_t nseen = 0;
        uint64_t sum = 0;
        for (uint32_t o = 0; o < noff; o++) {
            uint32_t code = o, manhattan = 0;
            int inside = 1;
            uint64_t nb = 0, stride = 1;
            for (uint32_t i = 0; i < ndim; i++) {
                const int64_t d = (int64_t)(code % 3) - 1;
                code /= 3;
                manhattan += d != 0;
                int64_t v = co[i] + d;
                if (torus_wrap) {
                    v = ((v % (int64_t)dims[i]) + dims[i]) % dims[i];
                } else if (v < 0 || v >= (int64_t)dims[i]) {
                    inside = 0;
                }
                nb += (uint64_t)v * stride;
                stride *= dims[i];
            }
            if (!inside || (von_neumann && manhattan > 1)) continue;
            int dup = 0;
            for (uint32_t k = 0; k < nseen; k++) if (seen[k] == nb) dup = 1;
            if (dup) continue;
            seen[nseen++] = nb;
            sum += counts[nb];
        }
        out[c] = (uint32_t)sum;
    }
}

/* out[a] = table[cell of agent a], 0 for an agent off the lattice. */
void orc_grid_gather(uint32_t ndim, const uint32_t *dims, uint64_t n, const int32_t *const *pos,
                     const uint32_t *table, uint32_t *out)
{
    for (uint64_t a = 0; a < n; a++) {
        uint64_t c;
        out[a] = cell_of(ndim, dims, pos, a, &c) ? table[c] : 0;
    }
}

/* out[i] = number of neighbours j of node i with state[j] == match, each
 * adjacency entry counted (a repeated edge counts twice); entries naming a
 * node outside [0, n) are not counted. */
void orc_graph_count(uint64_t n, const uint32_t *row, const uint32_t *col, const uint8_t *state,
                     uint32_t match, uint32_t *out)
{
    for (uint64_t i = 0; i < n; i++) {
        uint32_t k = 0;
        for (uint32_t e = row[i]; e < row[i + 1]; e++)
            if (col[e] < n && state[col[e]] == match) k++;
        out[i] = k;
    }
}

/* The SIR transition of step t on its own, given each agent's infected
 * neighbour count k: S with k >= 1 becomes I iff its EPI word is below
 * T_inf[min(k, k_sat)], I becomes R iff its EPI word is below T_rec. */
void orc_sir_transition(uint64_t n, uint8_t *s, const uint32_t *k, uint32_t seed,
                        uint32_t stream, uint32_t t, const uint32_t *t_inf, uint32_t k_sat,
                        uint32_t t_rec)
{
    for (uint64_t a = 0; a < n; a++) {
        if (s[a] == S_SUS && k[a] >= 1) {
            const uint32_t u = orc_word(seed, stream, P_EPI, 1, t, (uint32_t)a, 0);
            if (u < t_inf[k[a] < k_sat ? k[a] : k_sat]) s[a] = S_INF;
        } else if (s[a] == S_INF) {
            const uint32_t u = orc_word(seed, stream, P_EPI, 1, t, (uint32_t)a, 0);
            if (u < t_rec) s[a] = S_REC;
        }
    }
}

/* ------------------------------------------------------ continuous space */

/* The benchmark models as the paper states them (Sec. 5.1.2): agents in a
 * continuous W x W world (float32 coordinates in [0, W]).
 *   init      x = float(u >> 8) * 2^-24 * W and likewise y, from the two
 *             INIT_POS words of the agent (the product rounds once);
 *   walk      each step x <- min(max(x + dx, 0), W), y likewise, with
 *             dx = float(u >> 8) * 2^-23 - 1 (exact, uniform on [-1, 1)) from
 *             the agent's first STEP word of the step and dy from its second;
 *   SIR       move as the walk, then every susceptible agent counts the
 *             agents infected at the start of the step whose post-move
 *             position lies within distance r:
 *             (xa - xb)^2 + (ya - yb)^2 <= r^2, evaluated in float32 in that
 *             order with a rounding after every operation; with k >= 1 it
 *             becomes infected iff its EPI word is below T_inf[min(k, k_sat)]
 *             (probability 1 - (1 - p)^k); an infected agent counts one more
 *             day and recovers once it has counted `recover` days; recovered
 *             agents stay recovered.  Agents 0..I0-1 start infected, day 0.
 * The contact search is the all-pairs test the paper describes. */

static float cont_coord(uint32_t u, float W)
{
    return (float)(u >> 8) * (1.0f / 16777216.0f) * W;
}

static float cont_delta(uint32_t u)
{
    return (float)(u >> 8) * (1.0f / 8388608.0f) - 1.0f;
}

static float clampf(float v, float W)
{
    return v < 0.0f ? 0.0f : (v > W ? W : v);
}

void orc_cont_init(uint32_t n, float W, uint32_t seed, uint32_t stream, float *x, float *y)
{
    for (uint32_t a = 0; a < n; a++) {
        x[a] = cont_coord(orc_word(seed, stream, P_INIT_POS, 2, 0, a, 0), W);
        y[a] = cont_coord(orc_word(seed, stream, P_INIT_POS, 2, 0, a, 1), W);
    }
}

static void cont_move(uint32_t n, float W, uint32_t seed, uint32_t stream, uint32_t t, float *x,
                      float *y)
{
    for (uint32_t a = 0; a < n; a++) {
        x[a] = clampf(x[a] + cont_delta(orc_word(seed, stream, P_STEP, 2, t, a, 0)), W);
        y[a] = clampf(y[a] + cont_delta(orc_word(seed, stream, P_STEP, 2, t, a, 1)), W);
    }
}

void orc_cont_walk(uint32_t n, float W, uint32_t seed, uint32_t stream, uint32_t t0,
                   uint32_t n_steps, float *x, float *y)
{
    for (uint32_t t = t0; t < t0 + n_steps; t++) cont_move(n, W, seed, stream, t, x, y);
}

int orc_cont_sir(uint32_t n, float W, float r, uint32_t seed, uint32_t stream,
                 const uint32_t *t_inf, uint32_t k_sat, uint32_t recover, uint32_t t0,
                 uint32_t n_steps, float *x, float *y, uint8_t *s, uint8_t *days)
{
    uint8_t *s0 = malloc(n ? n : 1);
    if (!s0) return -1;
    const float r2 = r * r;
    for (uint32_t t = t0; t < t0 + n_steps; t++) {
        cont_move(n, W, seed, stream, t, x, y);
        memcpy(s0, s, n);
        for (uint32_t a = 0; a < n; a++) {
            if (s0[a] == S_SUS) {
                uint32_t k = 0;
                for (uint32_t b = 0; b < n; b++) {
                    if (s0[b] != S_INF) continue;
                    const float dx = x[a] - x[b], dy = y[a] - y[b];
                    const float dx2 = dx * dx, dy2 = dy * dy;
                    if (dx2 + dy2 <= r2) k++;
                }
                if (k >= 1) {
                    const uint32_t u = orc_word(seed, stream, P_EPI, 1, t, a, 0);
                    if (u < t_inf[k < k_sat ? k : k_sat]) {
                        s[a] = S_INF;
                        days[a] = 0;
                    }
                }
            } else if (s0[a] == S_INF) {
                days[a] += 1;
                if (days[a] >= recover) s[a] = S_REC;
            }
        }
    }
    free(s0);
    return 0;
}

/* ------------------------------------------------------------ whole runs */

/* Run a whole simulation from init for n_steps steps (steps 0..n_steps-1).
 * Columns are caller buffers of length n; returns 0, or -1 on a bad
 * argument or allocation failure. */
int orc_run_wealth(uint32_t n, int32_t w_init, uint32_t seed, uint32_t stream,
                   uint32_t t0, uint32_t n_steps, int32_t *w, int do_init)
{
    if (n == 0) return -1;
    uint32_t *rs = malloc((size_t)n * sizeof(uint32_t));
    int32_t *ws = malloc((size_t)n * sizeof(int32_t));
    if (!rs || !ws) { free(rs); free(ws); return -1; }
    if (do_init) orc_init_wealth(n, w_init, w);
    for (uint32_t t = t0; t < t0 + n_steps; t++)
        orc_wealth_step(n, seed, stream, t, w, rs, ws);
    free(rs); free(ws);
    return 0;
}

int orc_run_walk(uint32_t n, uint32_t L, uint32_t seed, uint32_t stream,
                 uint32_t t0, uint32_t n_steps, int32_t *x, int32_t *y, int do_init)
{
    if (n == 0 || L == 0) return -1;
    if (do_init) orc_init_positions(n, L, seed, stream, x, y);
    for (uint32_t t = t0; t < t0 + n_steps; t++)
        orc_walk_step(n, L, seed, stream, t, x, y);
    return 0;
}

/* Same as orc_run_walk but only for the agents listed in ids (agents of the
 * random walk never interact, so each trajectory can be replayed alone).
 * Outputs x[i], y[i] belong to agent ids[i]. */
int orc_walk_agents(uint32_t n_ids, const uint32_t *ids, uint32_t L,
                    uint32_t seed, uint32_t stream, uint32_t n_steps,
                    int32_t *x, int32_t *y)
{
    if (L == 0) return -1;
    for (uint32_t i = 0; i < n_ids; i++) {
        uint32_t a = ids[i];
        int32_t px = (int32_t)grid_coord(orc_word(seed, stream, P_INIT_POS, 2, 0, a, 0), L);
        int32_t py = (int32_t)grid_coord(orc_word(seed, stream, P_INIT_POS, 2, 0, a, 1), L);
        for (uint32_t t = 0; t < n_steps; t++) {
            uint32_t d = orc_word(seed, stream, P_MOVE, 1, t, a, 0) >> 29;
            px = torus((int64_t)px + MOVE_DX[d], L);
            py = torus((int64_t)py + MOVE_DY[d], L);
        }
        x[i] = px; y[i] = py;
    }
    return 0;
}

int orc_run_sir(uint32_t n, uint32_t L, uint32_t seed, uint32_t stream,
                uint32_t i0, const uint32_t *t_inf, uint32_t k_sat,
                uint32_t t_rec, uint32_t t0, uint32_t n_steps,
                int32_t *x, int32_t *y, uint8_t *s, int do_init)
{
    if (n == 0 || L == 0 || i0 > n) return -1;
    uint32_t *C = malloc((size_t)L * L * sizeof(uint32_t));
    uint8_t *sn = malloc(n);
    if (!C || !sn) { free(C); free(sn); return -1; }
    if (do_init) {
        orc_init_positions(n, L, seed, stream, x, y);
        orc_init_states(n, i0, s);
    }
    for (uint32_t t = t0; t < t0 + n_steps; t++)
        orc_sir_step(n, L, seed, stream, t, x, y, s, t_inf, k_sat, t_rec, C, sn);
    free(C); free(sn);
    return 0;
}
