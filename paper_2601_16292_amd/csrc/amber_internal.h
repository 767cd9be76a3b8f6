// amber_internal.h -- launchers shared by the host runtime (amber_host.cpp)
// and the gfx950 kernels (amber_device.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace amber {

// Purposes of the counter-based random stream (counter word 2).
enum : uint32_t { P_INIT_POS = 0, P_MOVE = 1, P_EPI = 2, P_RECIPIENT = 3, P_ORDER = 4,
                  P_STEP = 5 };

// State codes of the SIR column.
enum : uint8_t { ST_S = 0, ST_I = 1, ST_R = 2 };

// Every column is padded to whole groups of this many agents.
constexpr uint32_t AGENT_PAD = 64;

// Device-side accumulators of amber_invariants (lives at workspace offset 0).
struct DevInvariants {
    unsigned long long wealth_sum;   // two's-complement int64 sum
    unsigned long long n_s, n_i, n_r;
    unsigned long long out_of_bounds;
    unsigned long long digest;
    int wealth_min;
    int pad[3];
};
static_assert(sizeof(DevInvariants) <= 64, "invariants block must fit 64 B");

// Workspace head: the reduced invariants at offset 0, then up to
// INV_MAX_BLOCKS per-workgroup partials.
constexpr uint32_t INV_MAX_BLOCKS = 1024;
constexpr uint64_t ERR_FLAG_OFFSET = 128;      // sticky device error word (uint32)
constexpr uint64_t INV_PARTIALS_OFFSET = 256;
constexpr uint64_t INV_REGION = INV_PARTIALS_OFFSET + 64ull * INV_MAX_BLOCKS;

// Per-run parameters of a SIR step, passed by value as a kernel argument.
struct SirParams {
    int32_t *x;
    int32_t *y;
    uint8_t *s;
    uint32_t *count[3];        // per-cell infected counts, rotating with step mod 3
    const uint32_t *t_inf;     // infection thresholds, table_len entries
    uint32_t table_len;        // k_sat + 1
    uint32_t t_rec;
    uint32_t n;
    int32_t L;
    uint32_t k0, k1;           // Philox key (seed, stream)
    uint32_t groups;           // ceil(n / 4), filled by the launcher
    uint32_t quads;            // ceil(L*L / 4), filled by the launcher
    uint32_t dquads;           // ceil(L*L / 16): 16-byte words of a demand map
    uint32_t t_base;           // first step of the current call (grid rotation origin)
    uint32_t t_last;           // last step of the current call (gather mode), set per call
    // gather mode: when non-null, the launch that runs the call's remaining
    // steps stores stop_seq here (pinned host memory, system scope)
    uint32_t *stop_word;
    uint32_t stop_seq;
    // demand-driven binning (gather mode, see sir_body_demand): dmap[g] marks
    // the cells some susceptible agent may read; nsi holds per-step S and I
    // counts and the targeted-binning flags
    uint8_t *dmap[3];
    uint32_t *nsi;
    // exchange count mode (see sir_exchange_produce): null xrec = unavailable
    uint32_t *xrec;            // xW segments of 3*1024 cell records
    uint32_t *xtab;            // xtab[w*xP + band] = offset << 16 | count
    uint32_t xh, xP, xW;       // rows per band, bands (>= 3), producer workgroups
    // side of the coarse demand maps (one byte per 8 x 8 cells, stored after
    // each fine map at its 256-byte-rounded end), 0 = none
    uint32_t cside;
};

// Counts area of the demand-driven binning: for each call-relative step
// parity (4), the S and I counts of that step spread over NSI_SLOTS words
// each, one word per 128-byte line (atomics on one line serialise like
// atomics on one word), then one targeted-binning flag per parity.
constexpr uint32_t NSI_SLOTS = 64;
constexpr uint32_t NSI_STRIDE = 32;
constexpr uint32_t NSI_FLAGS = 4 * 2 * NSI_SLOTS * NSI_STRIDE;
constexpr uint32_t NSI_WORDS = NSI_FLAGS + 4;

// Record slots per producer workgroup of the SIR exchange mode (3 per agent).
constexpr uint32_t XSEG_WORDS = 3 * 1024;

// Device-wide barrier state of the persistent SIR form (inside the workspace).
constexpr uint32_t SYNC_WORDS = 64 * 32;      // up to 63 counter groups + the top counter
struct SyncParams {
    uint32_t *words;           // group counters every 32 words, then the top counter
    uint32_t *err;             // sticky: set when a barrier wait gave up
    uint32_t group_size;       // workgroups per group counter
    uint32_t ngroups;
};

// Launch configuration knobs (results never depend on them).
struct Tuning {
    uint32_t block = 256;      // threads per workgroup (multiple of 64, <= 1024)
    uint32_t sir_form = 0;     // 0 = automatic, 1 = pipelined, 2 = persistent
    uint32_t max_g = 8;        // persistent form: largest groups-per-thread to try
    uint32_t sir_count = 0;    // 0 = automatic, 1 = gather 3x3 cells, 2 = box-summed grid,
                               // 3 = exchange (sorted records, per-band counts),
                               // 4 = tiled (tile-sorted working copy, counts in LDS)
    uint32_t wealth_form = 0;  // 0 = automatic, 1 = atomic scatter, 2 = partition exchange,
                               // 3 = partition exchange with the 32-bit fold
    uint32_t sir_tile = 0;     // tiled mode: tile side 32 or 64 (0 = automatic)
    uint32_t sir_poll = 0;     // gather mode: 0 = poll for the early stop, 1 = never
};

hipError_t launch_init_wealth(int32_t *w, int32_t *inc0, int32_t *inc1, uint32_t n,
                              int32_t w_init, hipStream_t st);
hipError_t launch_init_positions(int32_t *x, int32_t *y, uint32_t n, int32_t L,
                                 uint32_t k0, uint32_t k1, hipStream_t st);
hipError_t launch_init_states(uint8_t *s, uint32_t n, uint32_t i0, hipStream_t st);
hipError_t launch_zero_words(uint32_t *p, uint64_t words, hipStream_t st);
// Copies count host words to dst through kernel arguments (no host wait).
hipError_t launch_write_words(uint32_t *dst, const uint32_t *src, uint64_t count, hipStream_t st);

// View primitives on arbitrary columns (amber_views.hip).
union ViewValue {
    int32_t i;
    float f;
};
constexpr uint32_t VIEW_I32 = 0, VIEW_F32 = 1;
// Workspace bytes of a float32 scatter-add of m entries.
uint64_t view_scatter_f32_workspace(uint64_t m);
hipError_t launch_view_update(void *col, uint32_t dtype, uint64_t n, ViewValue a, ViewValue b,
                              const void *pred, uint32_t pred_dtype, uint32_t cmp, ViewValue thr,
                              hipStream_t st);
// ws: view_scatter_f32_workspace(m) bytes, 16-byte aligned (float32 only).
hipError_t launch_view_scatter_add(void *col, uint32_t dtype, uint64_t n, const uint32_t *ids,
                                   uint64_t m, const void *vals, ViewValue scalar, void *ws,
                                   hipStream_t st);
// The write log: in log order col[ids[j]] = vals[j] (last write stays); ws as
// for the float32 scatter-add.
hipError_t launch_view_write_log(uint32_t *col, uint64_t n, const uint32_t *ids, uint64_t m,
                                 const uint32_t *vals, void *ws, hipStream_t st);
// Stable LSD radix sort of entries j < m by key min(ids[j], n) (n below 2^32;
// n = 2^32 - 1 sorts the full 32-bit values), carrying j.  ws holds
// view_scatter_f32_workspace(m) bytes; *keys / *pos receive the sorted
// arrays inside it.
hipError_t radix_sort_ids(const uint32_t *ids, uint64_t n, uint64_t m, void *ws, hipStream_t st,
                          const uint32_t **keys, const uint32_t **pos);

// Environments (amber_env.hip): a lattice of ndim <= MAX_DIMS axes, cell
// index sum pos_i * stride_i with stride_0 = 1 (first axis fastest).
constexpr uint32_t MAX_DIMS = 4;
struct GridDesc {
    const int32_t *pos[MAX_DIMS];
    uint32_t dims[MAX_DIMS];
    uint32_t stride[MAX_DIMS];
    uint32_t ndim;
};
// counts (cells words) is overwritten with the agents per cell.
hipError_t launch_grid_count(const GridDesc &g, uint64_t n, const uint8_t *state, uint32_t match,
                             uint32_t *counts, uint64_t cells, hipStream_t st);
hipError_t launch_grid_neighbour_sum(const GridDesc &g, uint64_t cells, uint32_t von_neumann,
                                     uint32_t torus, uint32_t dedup, const uint32_t *counts,
                                     uint32_t *out, hipStream_t st);
hipError_t launch_grid_gather(const GridDesc &g, uint64_t n, const uint32_t *table, uint32_t *out,
                              hipStream_t st);
hipError_t launch_graph_count(const uint32_t *row, const uint32_t *col, uint64_t n, uint64_t nnz,
                              const uint8_t *state, uint32_t match, uint32_t *out, hipStream_t st);
hipError_t launch_sir_transition_only(uint8_t *s, const uint32_t *k, uint64_t n, uint32_t k0,
                                      uint32_t k1, uint32_t t, const uint32_t *t_inf,
                                      uint32_t table_len, uint32_t t_rec, hipStream_t st);

// Continuous-space walk and SIR (amber_cont.hip); nc = cells per axis of the
// SIR's cell list (floor(W / r) + 1).
uint64_t cont_sir_workspace(uint32_t n, uint32_t nc, uint32_t table_len);
hipError_t launch_cont_init(float *x, float *y, uint32_t n, float W, uint32_t k0, uint32_t k1,
                            hipStream_t st);
// SIR states: agents below i0 infected, the rest susceptible, days 0.
hipError_t launch_cont_states(uint8_t *s, uint8_t *days, uint32_t n, uint32_t i0, hipStream_t st);
hipError_t launch_cont_walk(float *x, float *y, uint32_t n, float W, uint32_t k0, uint32_t k1,
                            uint32_t t0, uint32_t n_steps, hipStream_t st);
hipError_t launch_cont_sir(float *x, float *y, uint8_t *s, uint8_t *days, uint32_t n, float W,
                           float r, uint32_t nc, uint32_t k0, uint32_t k1, const uint32_t *table,
                           uint32_t table_len, uint32_t recover, uint32_t t0, uint32_t n_steps,
                           void *ws, hipStream_t st);

// Asynchronous (sequential) wealth steps t0 .. t0 + n_steps - 1 on the column
// w; ws holds async_wealth_workspace(n) bytes (16-byte aligned); err is the
// handle's sticky device error word.
uint64_t async_wealth_workspace(uint32_t n);
hipError_t launch_wealth_async(int32_t *w, uint32_t n, uint32_t k0, uint32_t k1, uint32_t t0,
                               uint32_t n_steps, void *ws, uint32_t *err, hipStream_t st);

// Device workspace of the no-allocation handles: a file-scope device array
// of NOALLOC_SCRATCH_BYTES per GPU.  noalloc_scratch returns its address on
// `device`, which must be the current device (looked up once per device).
constexpr uint64_t NOALLOC_SCRATCH_BYTES = 32ull << 20;
constexpr uint32_t NOALLOC_MAX_DEVICES = 64;
hipError_t noalloc_scratch(int device, void **ptr);

// Random walk: steps t0 .. t0+n_steps-1 with positions held in registers.
hipError_t launch_walk(int32_t *x, int32_t *y, uint32_t n, int32_t L, uint32_t k0,
                       uint32_t k1, uint32_t t0, uint32_t n_steps, const Tuning &tu,
                       hipStream_t st);

// Wealth: one step t.  The state is base + inc_cur; the step leaves base' in
// base, zeroes inc_cur and scatters the recipients' units into inc_nxt
// (which must be zero on entry).
hipError_t launch_wealth_step(int32_t *base, int32_t *inc_cur, int32_t *inc_nxt, uint32_t n,
                              uint32_t k0, uint32_t k1, uint32_t t, const Tuning &tu,
                              hipStream_t st);
// base += inc; inc = 0.
hipError_t launch_wealth_fold(int32_t *base, int32_t *inc, uint32_t n, hipStream_t st);
// Whole run segment for small N in one workgroup (state in LDS).
hipError_t launch_wealth_small(int32_t *w, uint32_t n, uint32_t k0, uint32_t k1,
                               uint32_t t0, uint32_t n_steps, hipStream_t st);
uint32_t wealth_small_max_agents();
// Partition-exchange wealth path: log2 of the partition size for n agents
// (0 when n is too large for it).  A call of n steps launches mode 2 (take
// donors) once, mode 3 (fold + take) n-1 times and mode 1 (fold) once, with
// parity_in = step offset & 1; mode bit 2 makes the 16-bit kernels (2^15 and
// 2^16 agents per partition) fold with 32-bit counters.
struct WealthXParams {
    int32_t *w;
    uint32_t *rec[2];          // P segments of 2^bits records, per parity: recipient ids
                               // (32-bit), or, for 2^15 and 2^16 agents per partition,
                               // 16-bit indices within the destination partition
    uint32_t *tab[2];          // tab[s*P + d] = offset << 16 | count (16-bit kernels:
                               // offset << 16 | (count - 1), all ones if empty), per parity
    uint32_t n, P, k0, k1;
};
uint32_t wealth_exchange_bits(uint32_t n);
hipError_t launch_wealth_exchange(const WealthXParams &x, uint32_t t, uint32_t parity_in,
                                  uint32_t mode, uint32_t bits, hipStream_t st);

// SIR, pipelined form.  Gather mode: head(t0), body(t0+1 .. t_last),
// tail(t_last), clear(1 << ((n-1) % 3)).  Box mode: head(t0), box(t0),
// then body(t), box(t) for t0 < t <= t_last, tail(t_last),
// clear(1 << ((n-1) & 1) | 4).  sir_fill() runs inside every launcher.
hipError_t launch_sir_head(SirParams p, uint32_t t, bool box, const Tuning &tu, hipStream_t st);
hipError_t launch_sir_body(SirParams p, uint32_t t, bool box, const Tuning &tu, hipStream_t st);
// i_last: call-relative index of the last body launch enqueued (gather mode)
hipError_t launch_sir_tail(SirParams p, uint32_t t, uint32_t i_last, bool box, const Tuning &tu,
                           hipStream_t st);
hipError_t launch_sir_box(SirParams p, uint32_t t, hipStream_t st);
hipError_t launch_sir_clear(SirParams p, uint32_t mask, hipStream_t st);
// Exchange count mode: xbody(t0, no transition), then xcount, and for each
// later step xbody(t, transition) + xcount; finally tail(t_last, box) and
// clear(4).  sir_exchange_shape picks the band height h, band count P and
// producer workgroup count W (false when the run does not fit the mode).
bool sir_exchange_shape(uint32_t n, uint32_t L, uint32_t *h, uint32_t *P, uint32_t *W);
hipError_t launch_sir_xbody(SirParams p, uint32_t t, bool transition, hipStream_t st);
hipError_t launch_sir_xcount(SirParams p, hipStream_t st);
// SIR, persistent form: all n steps in one cooperative launch.  Returns the
// groups-per-thread G (1, 2, 4 or 8, at most max_g) and the workgroup count
// for n agents, or 0 when the population does not fit co-resident.
uint32_t sir_persistent_groups_per_thread(uint32_t n, uint32_t max_g, uint32_t *blocks);
hipError_t launch_sir_persistent(SirParams p, uint32_t *sync_words, uint32_t *err, uint32_t t0,
                                 uint32_t n_steps, uint32_t g, uint32_t blocks, hipStream_t st);

// SIR, tiled count mode.  The grid is cut into nT x nT tiles of T x T cells
// (T = 32 or 64); the last tile of each axis is L - (nT-1)*T cells wide,
// which nT = (L-2)/T + 1 keeps within [2, T+1].  The mode needs nT >= 3.
// During a call each agent is one record {id, lx | ly << 10 | state << 20}
// (lx, ly relative to the tile holding the agent) in its tile's record list;
// one workgroup per tile runs each step.  Two generations g = 0, 1 of every
// buffer alternate with the step of the call.  A tile's list of v records
// is virtual: index u < cap sits at tile * cap + u, the rest in an overflow
// range at ovf + (u - cap) allocated from the generation's overflow area
// (which starts at nT^2 * cap and holds up to n records).
constexpr uint32_t TILE_HDR = 10;         // per tile: overflow base, 9 group counts
constexpr uint32_t TILE_MAX_AGENTS = 1u << 30;
constexpr uint32_t TILE_MIN = 32;         // smallest tile side (sizes the buffers)
struct TileParams {
    int32_t *x;
    int32_t *y;
    uint8_t *s;
    const uint32_t *t_inf;
    uint32_t table_len, t_rec, n, k0, k1;
    int32_t L;
    uint32_t T, tshift, nT;
    uint32_t rs;               // ring words per tile: 4T + 8
    uint32_t cap;              // record slots per tile
    uint32_t ovf0;             // first overflow slot: nT^2 * cap
    uint2 *rec[2];             // records, nT^2 * cap + n per generation
    uint32_t *hdr[2];          // TILE_HDR words per tile
    uint32_t *C[2];            // L*L interior infected counts
    uint32_t *ring[2];         // rs words per tile: infected counts on the ring around it
    uint32_t *cursor;          // one word per tile (initial sort)
    uint32_t *ctr;             // overflow allocators: ctr[0] and ctr[64]
    uint32_t *err;             // sticky device error word: bit ERR_TILE_LISTS
    uint32_t *scnt;            // body launches: susceptible agents per tile after the
                               // transition (NULL: not counted)
    // Hand-off to a gather segment (tiled, then gather): when mark is set,
    // the launch that writes the columns back also marks, for every
    // susceptible agent, the 3 x 3 block around its position after the move
    // of step mark_t in demand map mark (and in its coarse map when
    // mark_cside != 0), and sets the gather segment's first two
    // targeted-binning flags (mark_flags[0] and [1]) to 1.
    uint8_t *mark;
    uint8_t *mark_coarse;
    uint32_t mark_cside;
    uint32_t mark_t;
    uint32_t *mark_flags;
};
// Bits of the sticky device error word at ERR_FLAG_OFFSET.
constexpr uint32_t ERR_BARRIER = 1u;      // a persistent-form barrier wait gave up
constexpr uint32_t ERR_TILE_LISTS = 2u;   // tiled mode: record lists out of range
constexpr uint32_t ERR_ASYNC_GENERATIONS = 4u;   // asynchronous step: donor set not closed
// Tile count per axis for side T (0 when the grid is too small for it).
uint32_t sir_tile_count(uint32_t L, uint32_t T);
// Words of the tiled buffers for grid side L with the smallest tile side.
uint64_t sir_tile_ring_words(uint32_t L);
// Record slots per tile for n agents on nt tiles: twice the mean plus 64.
uint32_t sir_tile_cap(uint32_t n, uint32_t nt);
// A call of n steps: sort (columns -> records, generation 0), then step(i)
// for i = 0 .. n with i = 0 the head (move + bin only) and i = n the tail
// (transition, then records -> columns).
hipError_t launch_sir_tile_sort(const TileParams &p, hipStream_t st);
hipError_t launch_sir_tile_step(const TileParams &p, uint32_t t0, uint32_t i, uint32_t n,
                                uint32_t block, hipStream_t st);
// dst[0] = a[0] + ... + a[n-1] (one workgroup; dst may be mapped host memory).
hipError_t launch_sum_words(const uint32_t *a, uint32_t n, uint32_t *dst, hipStream_t st);

// ------------------------------------------------------------------ batches
// Run tables of the batched launches, passed by value as kernel arguments.
// run r owns workgroups [block_end[r-1], block_end[r]).
constexpr uint32_t BATCH_RUNS = 16;          // runs per launch (per-step kernels)
constexpr uint32_t BATCH_SMALL_RUNS = 48;    // runs per launch (one workgroup per run)

struct WalkBatch {
    int32_t *x[BATCH_RUNS];
    int32_t *y[BATCH_RUNS];
    uint32_t n[BATCH_RUNS], k0[BATCH_RUNS], k1[BATCH_RUNS], t0[BATCH_RUNS];
    int32_t L[BATCH_RUNS];
    uint32_t block_end[BATCH_RUNS];
    uint32_t nruns;
};

struct WealthSmallBatch {
    int32_t *w[BATCH_SMALL_RUNS];
    uint32_t n[BATCH_SMALL_RUNS], k0[BATCH_SMALL_RUNS], k1[BATCH_SMALL_RUNS], t0[BATCH_SMALL_RUNS];
    uint32_t nruns;
};

struct WealthBatch {
    int32_t *base[BATCH_RUNS];
    int32_t *inc[2][BATCH_RUNS];
    uint32_t n[BATCH_RUNS], k0[BATCH_RUNS], k1[BATCH_RUNS], t0[BATCH_RUNS];
    uint32_t block_end[BATCH_RUNS];
    uint32_t nruns;
};

struct WealthXBatch {
    WealthXParams run[BATCH_RUNS];
    uint32_t t0[BATCH_RUNS];
    uint32_t block_end[BATCH_RUNS];       // over partitions (one workgroup each)
    uint32_t nruns;
};
// Partition-exchange wealth, batched: every run of the chunk uses the same
// partition size 2^bits; launches as in the single-run path, one per step.
hipError_t launch_wealth_exchange_batch(const WealthXBatch &b, uint32_t n_steps, uint32_t bits,
                                        hipStream_t st);

struct SirBatch {
    SirParams run[BATCH_RUNS];   // groups, quads and t_base filled in
    uint32_t t0[BATCH_RUNS];
    uint32_t block_end[BATCH_RUNS];       // over agent groups (block threads each)
    uint32_t cell_block_end[BATCH_RUNS];  // over grid quads (256 threads each)
    uint32_t xblock_end[BATCH_RUNS];      // exchange mode: producer workgroups (xW each)
    uint32_t band_end[BATCH_RUNS];        // exchange mode: count workgroups (xP each)
    uint32_t i_last[BATCH_RUNS];          // gather mode: last body launch that held the run
    uint32_t nruns;
};

// Random walk: every step of the call, one launch for the chunk.
hipError_t launch_walk_batch(const WalkBatch &b, uint32_t n_steps, uint32_t block, hipStream_t st);
// Wealth, runs of at most wealth_small_max_agents(): one launch for the chunk.
hipError_t launch_wealth_small_batch(const WealthSmallBatch &b, uint32_t n_steps, hipStream_t st);
// Wealth, larger runs: one launch per step for the chunk, then one fold.
hipError_t launch_wealth_batch(const WealthBatch &b, uint32_t n_steps, uint32_t block,
                               hipStream_t st);
// SIR, pipelined, box (mode 2) or exchange (mode 3) count mode: head,
// n_steps-1 bodies and a tail, each one launch for the chunk.
hipError_t launch_sir_batch(const SirBatch &b, uint32_t n_steps, uint32_t mode, uint32_t block,
                            hipStream_t st);
// SIR, pipelined, gather mode: one phase for the runs of b (the host
// enqueues the steps of all runs step by step, so that runs that have run
// their remaining steps can leave the later launches).  phase 0 = head,
// 1 = body of call-relative step i, 2 = tail (dirty check on b.i_last),
// 3 = clear of count grid (n_steps - 1) % 3 given as i.
hipError_t launch_sir_gather_batch(const SirBatch &b, uint32_t phase, uint32_t i, uint32_t n_steps,
                                   uint32_t block, hipStream_t st);
void sir_fill(SirParams &p);

// Two-stage reduction: per-workgroup partials, then one workgroup folds them
// into *acc.  No atomics, so the result does not depend on timing.
hipError_t launch_invariants(uint32_t model, uint32_t n, int32_t L, const int32_t *w,
                             const int32_t *x, const int32_t *y, const uint8_t *s,
                             DevInvariants *acc, DevInvariants *partials, hipStream_t st);

}  // namespace amber
