/*
 * amber.h -- C ABI of libamber, the MI355X (gfx950) hot path of a columnar
 * agent-based-modelling engine.
 *
 * Method: "AMBER: A Columnar Architecture for Scalable Agent-Based Modelling
 * in Python" (arXiv 2601.16292).  Agent state is a set of typed columns over
 * sequential agent ids (Sec. 3.1.1); a model step is a composition of
 * full-population, filtered and id-indexed scatter updates (Sec. 3.1.1
 * listings, Sec. 3.3) applied with synchronous snapshot semantics (Sec. 3.4).
 * The three models are the benchmark models of Sec. 5.1.2, stated here on a
 * torus grid with counter-based randomness:
 *
 *   WEALTH       every agent with wealth > 0 (filtered view) gives one unit to
 *                a recipient drawn uniformly from all N agents (self allowed);
 *                duplicate recipients accumulate (scatter-add view).
 *   RANDOM_WALK  every agent (full view) moves to one of its 8 Moore
 *                neighbours on an L x L torus (grid environment, Sec. 4.1).
 *   SIR          every agent moves as in RANDOM_WALK; then each susceptible
 *                agent with k infected agents in the distinct cells of its
 *                3x3 torus block becomes infected with probability
 *                1-(1-beta)^k, and each infected agent recovers with
 *                probability gamma (Sec. 5.1.2; torus-wrap neighbour
 *                deduplication, Sec. 6.1).
 *
 * Random numbers: Philox4x32-10 keyed (seed, stream).  Word j of agent a for
 * purpose p at step t is word (g mod 4) of the block at counter
 * (floor(g/4), t, p, 0) with g = a*W_p + j; purposes INIT_POS (p=0, W=2),
 * MOVE (1, 1), EPI (2, 1), RECIPIENT (3, 2).  Mappings: grid coordinate
 * floor(u*L/2^32); recipient floor((hi:lo)*N/2^64); direction u>>29 into the
 * moves (dx,dy) in lexicographic order without (0,0); Bernoulli(p) is
 * u < floor(p*2^32) computed exactly from the rational p.  All device
 * arithmetic is integer, so every result is bit-exact and independent of
 * launch shape, chunking and batching.
 *
 * Ownership: the caller owns every device buffer (columns and workspace) and
 * the HIP stream; they must outlive the handle.  The library allocates no
 * device memory; a handle owns host memory only.  Device pointers are plain
 * HIP device addresses on the current device.
 *
 * Errors: every call returns an amber_status_t; nothing aborts or throws
 * across the ABI.  On a validation failure nothing is written to any buffer.
 * amber_last_error() returns a thread-local message for the last failure.
 *
 * Concurrency: calls on one handle are ordered on its stream; a handle must
 * not be used from two threads at once.  Only amber_read_columns,
 * amber_invariants, amber_profile_* and amber_release synchronise with the
 * host; amber_step and amber_step_batch wait for the device only when the
 * caller opts in (sir_poll 2 in amber_tuning_t).
 */
#ifndef AMBER_H
#define AMBER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AMBER_ABI_VERSION 1u

#if defined(__GNUC__)
#define AMBER_API __attribute__((visibility("default")))
#else
#define AMBER_API
#endif

/* Largest infection-threshold table (entries) a SIR run may need. */
#define AMBER_MAX_TABLE 8192u

typedef enum {
    AMBER_WEALTH = 0,
    AMBER_RANDOM_WALK = 1,
    AMBER_SIR = 2
} amber_model_t;

typedef enum {
    AMBER_OK = 0,
    AMBER_E_INVALID = -1,      /* bad argument or descriptor                 */
    AMBER_E_NOMEM = -2,        /* host allocation failed / workspace too small */
    AMBER_E_DEVICE = -3,       /* a HIP call failed                          */
    AMBER_E_STATE = -4,        /* handle misuse (released, mixed devices)    */
    AMBER_E_UNSUPPORTED = -5   /* valid but outside what the library supports */
} amber_status_t;

typedef enum {
    AMBER_COL_WEALTH = 0,      /* int32, WEALTH                 */
    AMBER_COL_X = 1,           /* int32 in [0, L), RANDOM_WALK and SIR */
    AMBER_COL_Y = 2,           /* int32 in [0, L), RANDOM_WALK and SIR */
    AMBER_COL_STATE = 3        /* uint8 0=S 1=I 2=R, SIR         */
} amber_col_t;
#define AMBER_NUM_COLS 4

/* One simulation run.  Fields a model does not use are ignored. */
typedef struct {
    uint32_t abi_version;      /* must equal AMBER_ABI_VERSION                       */
    uint32_t model;            /* amber_model_t                                      */
    uint32_t n_agents;         /* N, 1 .. 2^31-1                                     */
    uint32_t grid_side;        /* L for RANDOM_WALK/SIR; 0 = round(sqrt(N)) (halves
                                  up); needs 1 <= L and L*L <= 2^31-1                */
    uint32_t seed;             /* Philox key word 0                                  */
    uint32_t stream;           /* Philox key word 1: replicate / request id          */
    int32_t  wealth_init;      /* WEALTH: initial wealth >= 0, N*wealth_init < 2^31  */
    uint32_t beta_num, beta_den;   /* SIR: beta = num/den, 0 <= num < den            */
    uint32_t gamma_num, gamma_den; /* SIR: gamma = num/den, 0 <= num < den           */
    uint32_t initial_infected; /* SIR: agents 0..I0-1 start infected; 0 = default
                                  max(1, floor((N+500)/1000)); must be <= N          */
} amber_run_desc_t;

/* Device buffers of one run, all caller-owned.  col[c] must be non-NULL and
 * 16-byte aligned, with at least amber_column_bytes(desc, c) bytes, for every
 * column the model uses (NULL otherwise).  Bytes past N in a column are
 * padding the library may overwrite.  workspace must be 256-byte aligned with
 * at least amber_workspace_bytes(desc) bytes; the library owns its contents
 * for the handle's life. */
typedef struct {
    void  *col[AMBER_NUM_COLS];
    void  *workspace;
    size_t workspace_bytes;
} amber_buffers_t;

/* Population invariants (Sec. 5.1.3): wealth is conserved, coordinates stay
 * on the grid, S+I+R = N.  Fields not used by the model are 0. */
typedef struct {
    uint64_t step;             /* number of steps taken since init               */
    int64_t  wealth_sum;
    int32_t  wealth_min;
    uint32_t reserved0;
    uint64_t n_s, n_i, n_r;
    uint64_t out_of_bounds;    /* rows outside the model's domain (w<0, x or y
                                  outside [0,L), state code > 2)                */
    uint64_t digest;           /* sum over agents a (mod 2^64) of h_a: h =
                                  fmix64(a), then per column value v_j in
                                  column order h = fmix64(h ^ ((j+1)<<32 | v_j));
                                  fmix64 is SplitMix64's finaliser            */
} amber_invariants_t;

/* Resolved parameters of a handle. */
typedef struct {
    uint32_t model, n_agents, grid_side, initial_infected;
    uint32_t seed, stream;
    uint32_t table_len;        /* SIR: entries in the infection table (k_sat+1) */
    uint32_t t_rec;            /* SIR: recovery threshold                        */
    uint64_t step;
} amber_pop_info_t;

typedef struct amber_pop amber_pop_t;   /* opaque host-side handle */

/* ABI version of the loaded library (AMBER_ABI_VERSION). */
AMBER_API uint32_t amber_abi_version(void);

/* Bytes the caller must allocate for column c (0 if the model does not use
 * it, or if the descriptor is invalid).  Rounded up to whole 64-agent groups. */
AMBER_API size_t amber_column_bytes(const amber_run_desc_t *desc, amber_col_t c);

/* Bytes of device workspace the run needs (0 if the descriptor is invalid;
 * every valid run needs some).  This is also the run's footprint beyond its
 * columns for admission by HBM budget. */
AMBER_API size_t amber_workspace_bytes(const amber_run_desc_t *desc);

/* Exact infection thresholds T[k] = floor(2^32 (1-(1-beta)^k)), k = 0..k_sat,
 * where k_sat is the first k with T = 2^32-1 (0 when beta = 0), computed on the
 * host with big-integer arithmetic.  Writes min(k_sat+1, cap) entries to out
 * and k_sat to *k_sat.  AMBER_E_INVALID for a bad beta, AMBER_E_UNSUPPORTED
 * when k_sat+1 > AMBER_MAX_TABLE. */
AMBER_API amber_status_t amber_infection_table(uint32_t beta_num, uint32_t beta_den,
                                     uint32_t *out, uint32_t cap, uint32_t *k_sat);

/* Bulk-create N agents (the bulk add_agents of Sec. 3.3): WEALTH sets every
 * wealth to wealth_init; RANDOM_WALK and SIR draw x and y uniformly on the
 * grid (INIT_POS words); SIR marks agents 0..I0-1 infected, the rest
 * susceptible.  Enqueues on hip_stream (a hipStream_t; NULL = default
 * stream) and returns a handle at step 0.  Does not synchronise.
 * AMBER_E_INVALID for a bad descriptor, or for a buffer that is NULL,
 * misaligned, not device memory of the current device, or (where the runtime
 * reports the extent of its allocation) shorter than the run needs;
 * AMBER_E_NOMEM when workspace_bytes is below amber_workspace_bytes(desc).
 * Nothing is enqueued when it fails. */
AMBER_API amber_status_t amber_init_population(const amber_run_desc_t *desc,
                                     const amber_buffers_t *bufs,
                                     void *hip_stream, amber_pop_t **out);

/* A run continued from a state held in host memory (the columnar bulk
 * create of Sec. 3.3, add_agents from arrays, here the state after `step`
 * steps of this descriptor's run): as amber_init_population, then the first
 * N rows of each column the model uses are copied from host_cols[c] (N
 * int32 values, uint8 for the state column; host memory read before the
 * call returns) and the handle's step count is `step`.  Stepping it on
 * gives the same columns as the uninterrupted run, since every random word
 * is addressed by (agent, step).  Synchronises the stream.  AMBER_E_INVALID,
 * with nothing enqueued, for a state outside the model's domain (negative
 * wealth or a wealth sum above 2^31-1, a coordinate off the grid, a state
 * code above 2) or step > 2^32-1; other errors as amber_init_population. */
AMBER_API amber_status_t amber_resume_population(const amber_run_desc_t *desc,
                                                 const amber_buffers_t *bufs,
                                                 const void *const *host_cols, uint64_t step,
                                                 void *hip_stream, amber_pop_t **out);

/* Bytes of device scratch behind amber_init_population_noalloc, per GPU. */
#define AMBER_NOALLOC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * bulk create as amber_init_population, but the run's workspace is a device
 * array inside the library (AMBER_NOALLOC_SCRATCH_BYTES per GPU, held until
 * the process ends) instead of a caller buffer.  The caller still owns the
 * columns and the stream; bufs->workspace must be NULL and
 * bufs->workspace_bytes 0.  Neither this call nor any later call on the
 * handle allocates device or pinned host memory: the handle takes no pinned
 * early-stop word, so its SIR calls never stop early or switch from the
 * tiled to the gather mode (results unchanged).  The scratch is shared by
 * every such handle on the GPU and keeps the last handle's contents; init
 * rewrites what must start at zero.  At most one handle from this call may
 * be live per GPU: a second returns AMBER_E_STATE until the first is
 * released (calls that overlapped on one scratch would race).
 * AMBER_E_UNSUPPORTED when amber_workspace_bytes(desc) exceeds the scratch
 * (for instance SIR runs beyond a few hundred thousand agents); other errors
 * as amber_init_population.  The handle is used and released as any other. */
AMBER_API amber_status_t amber_init_population_noalloc(const amber_run_desc_t *desc,
                                                       const amber_buffers_t *bufs,
                                                       void *hip_stream, amber_pop_t **out);

/* One model step composed of full-population, filtered and id-indexed
 * scatter updates over the columns (Sec. 3.1.1 listings and Sec. 3.3 view
 * API), applied with synchronous snapshot semantics (Sec. 3.4): every rule
 * of step t reads the state at the start of step t.  The per-model rules are
 * those of the benchmark models (Sec. 5.1.2) in the torus-grid restatement
 * at the top of this header.
 * Enqueues steps t .. t+n_steps-1 on the handle's stream, where t is the
 * handle's step count; on return the step count is t+n_steps.  When the
 * enqueued work completes, the caller's columns hold the state after those
 * steps.  Any split of a run into calls gives bit-identical results.  With
 * the default tuning (sir_poll 0) it never waits for the device: it returns
 * once everything is enqueued.  AMBER_E_STATE for a released handle,
 * AMBER_E_INVALID when t+n_steps would exceed 2^32-1, AMBER_E_UNSUPPORTED
 * for a tuning the run does not fit, AMBER_E_DEVICE when a launch fails. */
AMBER_API amber_status_t amber_step(amber_pop_t *pop, uint32_t n_steps);

/* Many runs stepped together: the replicates and parameter sweeps of an
 * experiment (Sec. 4.2), each run still the plain run of its own descriptor
 * and key.  Enqueues the same n_steps on each of n handles as fused batched
 * launches (one kernel per phase for many runs), ordered on the first
 * handle's stream (the other handles' streams are joined before and after).
 * Results are bit-identical to calling amber_step on each handle alone.
 * Handles must be distinct and on one device; models may be mixed.  Like
 * amber_step it only enqueues unless every SIR run of the batch has
 * sir_poll 2.  Errors as amber_step, and AMBER_E_INVALID for a repeated
 * handle, AMBER_E_STATE for handles on different devices. */
AMBER_API amber_status_t amber_step_batch(amber_pop_t *const *pops, uint32_t n, uint32_t n_steps);

/* Read access to the agent-state columns (the column reads of the view API,
 * Sec. 3.3).  Copies the columns selected by col_mask (bit c =
 * column c) to host memory: host_dst[c] receives N elements of column c
 * (int32, or uint8 for the state column), host memory owned by the caller.
 * Synchronises the stream.  AMBER_E_INVALID for a column the model does not
 * use, a NULL destination or unknown mask bits (nothing is copied);
 * AMBER_E_DEVICE when a copy fails or a kernel raised the sticky device
 * error word since the handle was created. */
AMBER_API amber_status_t amber_read_columns(amber_pop_t *pop, uint32_t col_mask,
                                  void *const *host_dst);

/* Reduce the invariants and the digest on the device and copy them to *out.
 * Synchronises the stream. */
AMBER_API amber_status_t amber_invariants(amber_pop_t *pop, amber_invariants_t *out);

/* Resolved parameters and step count of a handle (host only, no sync). */
AMBER_API amber_status_t amber_pop_info(const amber_pop_t *pop, amber_pop_info_t *out);

/* ------------------------------------------------------------------ views
 * The view primitives of the method (Sec. 3.3 view API; Sec. 3.1.1
 * listings) on any int32 or float32 column in device memory, outside any
 * run: a full-population update, a filtered (predicate) update and an
 * id-indexed scatter-add with duplicate ids accumulating.  Columns, ids,
 * values and workspace are caller-owned device buffers on the current
 * device (4-byte aligned; 16-byte alignment gives vector accesses); calls
 * are enqueued on hip_stream (NULL = default stream) and do not synchronise.
 * int32 arithmetic wraps modulo 2^32.  float32 updates are one fused
 * multiply-add (a*v + b rounded once to nearest); a float32 scatter-add
 * rounds after every addition, in the order of the list, so its result is
 * that of numpy's add.at.  Every result is independent of launch shape. */
typedef enum { AMBER_DT_I32 = 0, AMBER_DT_F32 = 1 } amber_dtype_t;
typedef enum {
    AMBER_CMP_LT = 0, AMBER_CMP_LE = 1, AMBER_CMP_EQ = 2,
    AMBER_CMP_NE = 3, AMBER_CMP_GE = 4, AMBER_CMP_GT = 5
} amber_cmp_t;
typedef union { int32_t i; float f; } amber_value_t;   /* member by dtype */

/* Full view (pred NULL): col[r] = a*col[r] + b for r < n.  Filtered view:
 * the same for the rows where pred[r] CMP thr, pred being an int32 or
 * float32 column of n rows (it may be col itself: it is read before the
 * update), thr of pred's dtype; NaN compares false except under NE.
 * AMBER_E_INVALID for a bad dtype or comparison, or a buffer that is NULL,
 * misaligned, not device memory of the current device or shorter than n
 * rows (nothing is enqueued); AMBER_E_UNSUPPORTED for n >= 2^40. */
AMBER_API amber_status_t amber_view_update(void *col, uint32_t dtype, uint64_t n,
                                           amber_value_t a, amber_value_t b, const void *pred,
                                           uint32_t pred_dtype, uint32_t cmp, amber_value_t thr,
                                           void *hip_stream);

/* Device workspace bytes of amber_view_scatter_add for m entries (0 for
 * int32, which needs none; 0 as well for a bad dtype or m > 2^31). */
AMBER_API size_t amber_view_scatter_workspace_bytes(uint32_t dtype, uint64_t n, uint64_t m);

/* Scatter view: for j = 0 .. m-1, col[ids[j]] += vals[j] (vals NULL: the
 * scalar), duplicates accumulating; entries with ids[j] >= n are skipped.
 * int32: one atomic add per entry (any order gives the same column).
 * float32: the entries are ordered by (id, j) with a stable radix sort in
 * the workspace, then each id's entries are added one after the other in
 * list order (an id with k entries costs k dependent adds on one thread).
 * AMBER_E_INVALID / AMBER_E_NOMEM for bad or short buffers (nothing is
 * enqueued), AMBER_E_UNSUPPORTED for n >= 2^32 or m > 2^31. */
AMBER_API amber_status_t amber_view_scatter_add(void *col, uint32_t dtype, uint64_t n,
                                                const uint32_t *ids, uint64_t m,
                                                const void *vals, amber_value_t scalar,
                                                void *workspace, size_t workspace_bytes,
                                                void *hip_stream);

/* The buffered per-agent write path (Sec. 3.2.1: record / update_data calls
 * kept in a pending-writes dictionary and flushed once per step by one
 * update on id), as a device write log: entries j = 0 .. m-1 are applied in
 * log order, col[ids[j]] = vals[j], so the last write to an id stays; ids
 * >= n are skipped; values are copied bit for bit (int32 or float32 columns
 * alike).  The entries are ordered by (id, j) with a stable radix sort in the
 * workspace (amber_view_write_log_workspace_bytes(m) bytes, 16-byte
 * aligned), then the last entry of each id writes.  Errors as
 * amber_view_scatter_add. */
AMBER_API size_t amber_view_write_log_workspace_bytes(uint64_t m);
AMBER_API amber_status_t amber_view_write_log(void *col, uint32_t dtype, uint64_t n,
                                              const uint32_t *ids, uint64_t m, const void *vals,
                                              void *workspace, size_t workspace_bytes,
                                              void *hip_stream);

/* Asynchronous (sequential) update semantics (Sec. 3.4): within step t the
 * agents act one at a time and each sees what the agents before it did.  The
 * order of step t is the agents sorted by (ORDER word, id), the ORDER word of
 * agent a being word (a mod 4) of the Philox block at counter (floor(a/4),
 * t, 4, 0).  WEALTH: in that order an agent with positive wealth gives one
 * unit to its recipient (the RECIPIENT draw of the synchronous model).
 * RANDOM_WALK: no agent reads another's state, so the step is the
 * synchronous one.  SIR: AMBER_E_UNSUPPORTED.
 * The GPU builds the donor set as a fixed point (an agent gives iff it starts
 * with wealth or a donor acting before it draws it), in at most 64
 * generations per step, then applies every transfer; a step whose donor set
 * is not closed by then raises the sticky device error (reported as
 * AMBER_E_DEVICE by the next synchronising call).  Enqueued on the handle's
 * stream, no synchronisation; steps t .. t+n_steps-1 as amber_step, and the
 * two may alternate on one handle.  workspace: caller-owned device memory
 * of amber_async_workspace_bytes(desc) bytes, 16-byte aligned, free for
 * other use between calls. */
AMBER_API size_t amber_async_workspace_bytes(const amber_run_desc_t *desc);
AMBER_API amber_status_t amber_step_async(amber_pop_t *pop, uint32_t n_steps, void *workspace,
                                          size_t workspace_bytes);

/* ----------------------------------------------------------- environments
 * The spatial environments of the method (Sec. 4.1) as device primitives:
 * grid lattices of 1 to AMBER_MAX_DIMS axes with Moore or von Neumann
 * neighbourhoods, torus-wrapped or bounded, and networks given as CSR
 * adjacency lists (the neighbours of node i are col[row[i] .. row[i+1]-1]).
 * A grid cell's index is sum_i pos_i * stride_i with stride_0 = 1 and
 * stride_i = stride_{i-1} * dims_{i-1} (first axis fastest; in 2-D y*L + x,
 * the SIR model's count grid).  pos is a host array of ndim device columns
 * (int32, n rows each); dims a host array.  Device buffers are caller-owned
 * and on the current device; calls are enqueued on hip_stream and do not
 * synchronise.  Agents off the lattice (a coordinate outside [0, dims_i))
 * are neither counted nor looked up.  AMBER_E_INVALID for a bad argument or
 * a buffer that is NULL, misaligned, not device memory of the current device
 * or shorter than the call needs (nothing is enqueued); AMBER_E_UNSUPPORTED
 * for lattices of 2^32 cells or more, 2^32 agents or more. */
#define AMBER_MAX_DIMS 4u
typedef enum { AMBER_MOORE = 0, AMBER_VON_NEUMANN = 1 } amber_neighbourhood_t;

/* counts[c] (overwritten) = number of agents a whose cell is c and, when
 * state is not NULL, whose state[a] == match. */
AMBER_API amber_status_t amber_grid_count(const int32_t *const *pos, uint32_t ndim,
                                          const uint32_t *dims, uint64_t n, const uint8_t *state,
                                          uint32_t match, uint32_t *counts, void *hip_stream);

/* out[c] = sum of counts over the distinct cells of c's neighbourhood, c
 * included: Moore, every offset in {-1,0,1}^ndim; von Neumann, the offsets
 * with at most one non-zero component.  torus != 0: coordinates wrap (a side
 * below 3 reaches a cell twice, which counts once); torus == 0: cells off
 * the lattice are left out.  out must not alias counts. */
AMBER_API amber_status_t amber_grid_neighbour_sum(const uint32_t *counts, uint32_t ndim,
                                                  const uint32_t *dims, uint32_t neighbourhood,
                                                  uint32_t torus, uint32_t *out,
                                                  void *hip_stream);

/* out[a] = table[cell of agent a] (0 for an agent off the lattice). */
AMBER_API amber_status_t amber_grid_gather(const uint32_t *table, const int32_t *const *pos,
                                           uint32_t ndim, const uint32_t *dims, uint64_t n,
                                           uint32_t *out, void *hip_stream);

/* Network neighbour query: out[i] = number of adjacency entries j of node i
 * (i < n) with state[j] == match; a repeated entry counts each time, and
 * entries past nnz or naming no node (j >= n) are not counted.  row holds
 * n+1 offsets, col nnz ids. */
AMBER_API amber_status_t amber_graph_neighbour_count(const uint32_t *row, const uint32_t *col,
                                                     uint64_t n, uint64_t nnz,
                                                     const uint8_t *state, uint32_t match,
                                                     uint32_t *out, void *hip_stream);

/* T_rec = floor(2^32 * gamma) for gamma = gamma_num / gamma_den, computed
 * exactly (the recovery threshold of the SIR model). */
AMBER_API amber_status_t amber_recovery_threshold(uint32_t gamma_num, uint32_t gamma_den,
                                                  uint32_t *out);

/* The SIR transition of step t on its own (Sec. 5.1.2 with exact
 * thresholds), for SIR variants built from the environment primitives:
 * given k[a], the infected count agent a sees, an S agent with k >= 1
 * becomes I iff its EPI word is below t_inf[min(k, table_len-1)], and an I
 * agent becomes R iff its EPI word is below t_rec; EPI words as in the SIR
 * model (key (seed, stream_id)).  t_inf: a device copy of the table of
 * amber_infection_table (table_len = k_sat + 1 entries). */
AMBER_API amber_status_t amber_sir_transition(uint8_t *state, const uint32_t *k, uint64_t n,
                                              uint32_t seed, uint32_t stream_id, uint32_t t,
                                              const uint32_t *t_inf, uint32_t table_len,
                                              uint32_t t_rec, void *hip_stream);

/* ------------------------------------------------------- continuous space
 * The paper's own benchmark models (Sec. 5.1.2) in continuous space, on
 * caller-owned float32 columns x, y (and uint8 state and days for the SIR),
 * n agents in a W x W world; keys (seed, stream_id) and step indices as for
 * the grid models.  Every float operation is one IEEE float32 operation
 * rounded to nearest, in the order written, so results are bit-exact.
 *   init   x = float(u >> 8) * 2^-24 * W, y likewise (INIT_POS words); SIR:
 *          agents 0 .. initial_infected-1 infected, the rest susceptible,
 *          days 0.  state and days both NULL: the walk.
 *   walk   per step x <- min(max(x + dx, 0), W), y likewise, with
 *          dx = float(u >> 8) * 2^-23 - 1 from the agent's first STEP word
 *          of the step (purpose 5, two words per agent) and dy from its
 *          second.
 *   SIR    the walk's move; then a susceptible agent counts the agents
 *          infected at the start of the step within distance r of it,
 *          (xa - xb)^2 + (ya - yb)^2 <= r^2, and with k >= 1 becomes infected
 *          iff its EPI word is below floor(2^32 (1 - (1 - p)^k)), p =
 *          p_num / p_den exactly (the paper: p = 0.1 per contact); an infected
 *          agent adds a day and recovers at `recover` days (the paper: 14).
 * The contact search uses a cell list of side r (the infected agents of the
 * step counting-sorted by cell in the workspace); W / r must stay below
 * 4096 (AMBER_E_UNSUPPORTED).  Calls are enqueued and do not synchronise,
 * except that amber_cont_sir builds its threshold table on the host.
 * AMBER_E_INVALID for bad arguments or short buffers (nothing enqueued). */
AMBER_API amber_status_t amber_cont_init(float *x, float *y, uint8_t *state, uint8_t *days,
                                         uint64_t n, float W, uint32_t seed, uint32_t stream_id,
                                         uint32_t initial_infected, void *hip_stream);
AMBER_API amber_status_t amber_cont_walk(float *x, float *y, uint64_t n, float W, uint32_t seed,
                                         uint32_t stream_id, uint32_t t0, uint32_t n_steps,
                                         void *hip_stream);
/* Workspace bytes of amber_cont_sir (0 for arguments it would refuse). */
AMBER_API size_t amber_cont_sir_workspace_bytes(uint64_t n, float W, float r, uint32_t p_num,
                                                uint32_t p_den);
AMBER_API amber_status_t amber_cont_sir(float *x, float *y, uint8_t *state, uint8_t *days,
                                        uint64_t n, float W, float r, uint32_t seed,
                                        uint32_t stream_id, uint32_t p_num, uint32_t p_den,
                                        uint32_t recover, uint32_t t0, uint32_t n_steps,
                                        void *workspace, size_t workspace_bytes,
                                        void *hip_stream);

/* Launch-shape knobs.  They never change results (all arithmetic is integer
 * and every random word is addressed by agent and step), only speed. */
typedef struct {
    uint32_t block;            /* threads per workgroup of the per-step kernels:
                                  multiple of 64 in [64, 1024]; default 256       */
    uint32_t sir_form;         /* 0 = automatic, 1 = pipelined (one kernel per
                                  step), 2 = persistent (one cooperative kernel
                                  per call, state in registers; fails with
                                  AMBER_E_UNSUPPORTED when N does not fit)        */
    uint32_t max_groups_per_thread; /* persistent form: largest number of 4-agent
                                  groups a thread may hold (1, 2, 4, 8; 0 = 8)    */
    uint32_t sir_count;        /* SIR neighbour counts in the pipelined form:
                                  0 = automatic: for calls of 128 steps or
                                  more, 5 on grids of more than 2M cells when
                                  sir_poll is 2, else 1; for shorter calls, 1 on grids of at most
                                  16M cells, else 4 for 16 to 127 steps and 2
                                  below (in batches: 1 for long calls, else 1
                                  or 2 by the same grid rule),
                                  1 = sum the 3x3 block of the
                                  count grid per agent, 2 = box-sum the grid once
                                  per step (one stencil kernel) and read one
                                  cell per agent, 3 = exchange: infected cells are
                                  counting-sorted by row band in LDS and counted
                                  per band into the box-summed grid, with no
                                  global atomics (AMBER_E_UNSUPPORTED when the
                                  grid is too small or too wide for it; inside
                                  amber_step_batch such runs use mode 1),
                                  4 = tiled: during a call the agents live as
                                  records sorted by grid tile, one workgroup per
                                  tile bins and sums the counts in LDS (needs a
                                  grid side of at least 2 x tile + 2, else
                                  AMBER_E_UNSUPPORTED; inside amber_step_batch
                                  such runs use the automatic mode),
                                  5 = tiled, then gather: as 4, and every 16
                                  steps of calls over 32 steps the host reads a
                                  device count of susceptible agents from the
                                  previous poll; once 4 S <= N it ends the
                                  tiled part (records back to the columns) and
                                  runs the rest of the call as mode 1 (same
                                  condition and fallback as 4; with sir_poll 1
                                  or under graph capture it stays tiled, and
                                  with sir_poll 0 it switches only if the count
                                  is already there when the host looks)         */
    uint32_t wealth_form;      /* WEALTH above 8192 agents: 0 = automatic,
                                  1 = global atomic scatter-add, 2 = partition
                                  exchange (recipient ids counting-sorted by
                                  destination in LDS, counted by the owner;
                                  AMBER_E_UNSUPPORTED above 2^27 agents),
                                  3 = as 2, with the owners of partitions of
                                  2^15 and 2^16 agents (above 2^24 agents)
                                  counting in 32-bit words in two passes, the
                                  form they take by themselves only when one
                                  agent receives 65536 units in a step (slower;
                                  below 2^24 agents the same as 2)               */
    uint32_t sir_tile;         /* tiled count mode: tile side 32 or 64 cells
                                  (0 = automatic)                                 */
    uint32_t sir_poll;         /* SIR calls of more than 32 steps in the gather
                                  mode (sir_count 1) and the tiled-then-gather
                                  mode (5).  In the gather mode, once no
                                  susceptible agent is left, one launch runs
                                  the call's remaining steps and stores the
                                  call's number in a pinned host word; the
                                  later launches do nothing.
                                  0 = read without waiting (default): every 16
                                  launches the host reads that word and stops
                                  enqueueing once it is set; mode 5 reads the
                                  susceptible count of the previous poll only
                                  if the device has already written it.
                                  amber_step never waits for the device.
                                  1 = off: one launch per step, no reads.
                                  2 = paced (opt-in; blocks): as 0, but every
                                  16 launches the host first waits until at
                                  most 32 of the call's launches are queued,
                                  so the early stop and the switch of mode 5
                                  take effect at once.  Only with 2 does the
                                  automatic count mode choose 5.
                                  In amber_step_batch the same per run (paced
                                  only when every gather-mode run of the batch
                                  has 2).  Nothing is read while the stream is
                                  being captured into a graph.                   */
    uint32_t reserved;
} amber_tuning_t;

/* Set / get a handle's launch-shape knobs (host only). */
AMBER_API amber_status_t amber_set_tuning(amber_pop_t *pop, const amber_tuning_t *t);
AMBER_API amber_status_t amber_get_tuning(const amber_pop_t *pop, amber_tuning_t *t);

/* Accumulated device time of one kernel of the path. */
typedef struct {
    char     name[40];
    uint64_t launches;
    double   total_ms;
} amber_kernel_time_t;

/* Measurement aid: while enabled, the kernels the handle enqueues are timed
 * with HIP events on the handle's stream.  Consecutive launches of one kernel
 * within one call share a single pair of events (one before the first, one
 * after the last), so total_ms / launches is the back-to-back time per launch
 * and no event sits between them; a kernel launched alone gets its own pair.
 * Enabling waits for the stream and clears the totals.  Off by default;
 * results are unaffected. */
AMBER_API amber_status_t amber_profile_enable(amber_pop_t *pop, int enable);

/* Waits for the stream, folds the recorded events into per-kernel totals and
 * copies min(cap, *count) entries to out; *count receives the number of
 * distinct kernels seen. */
AMBER_API amber_status_t amber_profile_read(amber_pop_t *pop, amber_kernel_time_t *out,
                                            uint32_t cap, uint32_t *count);

/* Free the handle (host memory only; device buffers stay the caller's).
 * Waits for the handle's enqueued work first. */
AMBER_API amber_status_t amber_release(amber_pop_t *pop);

/* Message for the last failed call on this thread ("" if none). */
AMBER_API const char *amber_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AMBER_H */
