// amber_device.hip -- gfx950 kernels of the columnar ABM hot path (one run
// per launch).  The batched forms live in amber_batch.hip.
//
// Columns are structure-of-arrays (Sec. 3.1.1): int32 wealth, int32 x, int32 y,
// uint8 state, each padded to whole 64-agent groups.  A thread owns 4
// consecutive agents, so every column access is a 16-byte (int32) or 4-byte
// (state) vector load or store, coalesced across the wavefront.  4 agents is
// also exactly one Philox block of MOVE/EPI words (1 word per agent) and two
// blocks of INIT_POS/RECIPIENT words (2 words per agent), so each thread
// computes whole blocks and never shares words with another thread.
//
// Everything is integer arithmetic; there is no dense contraction on this path
// (no MFMA).  The kernels are bound by HBM (or cache) bandwidth, by integer
// VALU throughput for Philox, and by atomic throughput for the scatter-adds.
#include "amber_device_common.h"

namespace amber {

// ------------------------------------------------------------------ init

__global__ void k_init_wealth(int4 *__restrict__ w, int4 *__restrict__ inc0,
                              int4 *__restrict__ inc1, uint32_t groups, uint32_t n,
                              int32_t w0)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= groups) return;
    const uint32_t a = 4 * q;
    w[q] = make_int4(a + 0 < n ? w0 : 0, a + 1 < n ? w0 : 0, a + 2 < n ? w0 : 0,
                     a + 3 < n ? w0 : 0);
    inc0[q] = make_int4(0, 0, 0, 0);
    inc1[q] = make_int4(0, 0, 0, 0);
}

// INIT_POS has 2 words per agent: block 2q covers agents 4q, 4q+1 as
// (x, y, x, y), block 2q+1 covers agents 4q+2, 4q+3.  Padding agents get
// valid coordinates too, so every padded lane stays on the grid.
__global__ void k_init_positions(int4 *__restrict__ x, int4 *__restrict__ y, uint32_t groups,
                                 int32_t L, uint32_t k0, uint32_t k1)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= groups) return;
    const uint4 b0 = philox(2 * q, 0, P_INIT_POS, k0, k1);
    const uint4 b1 = philox(2 * q + 1, 0, P_INIT_POS, k0, k1);
    x[q] = make_int4(grid_coord(b0.x, L), grid_coord(b0.z, L), grid_coord(b1.x, L),
                     grid_coord(b1.z, L));
    y[q] = make_int4(grid_coord(b0.y, L), grid_coord(b0.w, L), grid_coord(b1.y, L),
                     grid_coord(b1.w, L));
}

__global__ void k_init_states(uint32_t *__restrict__ s4, uint32_t groups, uint32_t i0)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= groups) return;
    const uint32_t a = 4 * q;
    uint32_t v = 0;
    for (uint32_t j = 0; j < 4; ++j) v |= (a + j < i0 ? (uint32_t)ST_I : 0u) << (8 * j);
    s4[q] = v;
}

__global__ void k_zero_words(uint4 *__restrict__ p, uint64_t quads)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < quads; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
}

// ------------------------------------------------------------------ random walk
// Agents of the random walk never interact, so a thread carries its 4 agents
// through all requested steps in registers: the columns are read and written
// once per call and only Philox (1 block per 4 agent-steps) remains per step.
__global__ void k_walk(int4 *__restrict__ x, int4 *__restrict__ y, uint32_t groups, int32_t L,
                       uint32_t k0, uint32_t k1, uint32_t t0, uint32_t n_steps)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < groups) walk_group(x, y, q, L, k0, k1, t0, n_steps);
}

// ------------------------------------------------------------------ wealth

__global__ void k_wealth_step(int4 *__restrict__ base, int4 *__restrict__ inc_cur,
                              int32_t *__restrict__ inc_nxt, uint32_t groups, uint32_t n,
                              uint32_t k0, uint32_t k1, uint32_t t)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < groups) wealth_step_group(base, inc_cur, inc_nxt, q, n, k0, k1, t);
}

__global__ void k_wealth_fold(int4 *__restrict__ base, int4 *__restrict__ inc, uint32_t groups)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < groups) wealth_fold_group(base, inc, q);
}

__global__ __launch_bounds__(WEALTH_SMALL_THREADS) void k_wealth_small(
    int32_t *__restrict__ w, uint32_t n, uint32_t k0, uint32_t k1, uint32_t t0, uint32_t n_steps)
{
    __shared__ int32_t sw[WEALTH_SMALL_MAX];
    __shared__ int32_t sinc[WEALTH_SMALL_MAX];
    wealth_small_run(w, sw, sinc, n, k0, k1, t0, n_steps);
}

// Partition-exchange wealth step (see wealth_exchange_partition).  mode bit 0:
// fold the records of the previous step; bit 1: take this step's donors.
// 2^14-agent partitions (72 KB of LDS) keep within 64 registers so that two
// workgroups share a CU.
template <int XB, int PMAX, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(XB == 14 ? 8 : 1)))
void k_wealth_x(WealthXParams x, uint32_t t, uint32_t parity_in, uint32_t mode)
{
    __shared__ __align__(16) int32_t hist[1u << XB];
    __shared__ uint32_t pcount[PMAX];
    __shared__ uint32_t poff[PMAX];
    wealth_exchange_partition<XB, PMAX, NT>(x, xcd_partition(blockIdx.x, gridDim.x), t,
                                            parity_in, (mode & 1u) != 0, (mode & 2u) != 0,
                                            hist, pcount, poff);
}

// The 16-bit form of the exchange (see wealth_exchange_partition16), for
// partitions of 2^15 and 2^16 agents; mode bit 2 asks for the 32-bit fold.
// With 2^15-agent partitions (69 KB of LDS) two workgroups share a CU if
// each wavefront keeps within 64 registers (8 per SIMD): one's fold then
// runs beside the other's Philox draws.
template <int XB, int PMAX, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(XB == 15 ? 8 : 1)))
void k_wealth_x16(WealthXParams x, uint32_t t, uint32_t parity_in, uint32_t mode)
{
    __shared__ __align__(16) uint32_t h2[1u << (XB - 1)];
    __shared__ uint32_t c32[PMAX + 2];
    __shared__ uint32_t flag;
    wealth_exchange_partition16<XB, PMAX, NT>(x, xcd_partition(blockIdx.x, gridDim.x), t,
                                              parity_in, (mode & 1u) != 0, (mode & 2u) != 0,
                                              (mode & 4u) != 0, h2, c32, &flag);
}

// head: move + bin(t).  The gather-mode head also clears demand map 2 and
// counts the states of the call's first step (demand-driven binning); its
// last workgroup holds no agents and does the bookkeeping.
template <bool BOX>
__global__ void k_sir_head(SirParams p, uint32_t t)
{
    if (BOX) {
        const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
        if (q < p.groups) sir_head_group<BOX>(p, q, t);
        return;
    }
    const uint32_t nb = gridDim.x - 1;
    if (blockIdx.x == nb) {
        sir_demand_book(p, 0);
        return;
    }
    __shared__ uint32_t s_wc[2 * 16];              // per-wavefront S and I counts
    sir_head_demand(p, blockIdx.x * blockDim.x + threadIdx.x, nb * blockDim.x, t, blockIdx.x,
                    s_wc);
}

// body (gather mode): transition(t-1), then move + bin(t), binning only on
// the demand map's cells when F_i is set and marking the next map when
// F_{i+1} is; clears the count grid of t+1 and the demand map of t+2.  The
// last workgroup holds no agents and does the bookkeeping.
__global__ void k_sir_body(SirParams p, uint32_t t)
{
    const uint32_t i = t - p.t_base;
    const uint32_t nb = gridDim.x - 1;
    if (blockIdx.x == nb) {
        sir_demand_book(p, i);
        return;
    }
    __shared__ uint32_t s_wc[2 * 16];              // per-wavefront S and I counts
    sir_body_demand(p, blockIdx.x * blockDim.x + threadIdx.x, nb * blockDim.x, t, i, blockIdx.x,
                    s_wc);
}

// body (box mode): transition(t-1) from K, then move + bin(t).
__global__ void k_sir_body_box(SirParams p, uint32_t t)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < p.groups) sir_body_group<true>(p, q, t);
}

// tail (gather mode): transition(t); clears the grid of t+2.  When the call
// ran out of susceptible agents a body launch has already run transition(t),
// and the tail clears all three grids.  i_last is the call-relative index of
// the last body launch enqueued.
__global__ void k_sir_tail(SirParams p, uint32_t t, uint32_t i_last)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    zero_quads(grid_of(p, t + 2), p.quads, q, stride);
    if (sir_demand_dirty(p, i_last)) {
        zero_quads(grid_of(p, t), p.quads, q, stride);
        zero_quads(grid_of(p, t + 1), p.quads, q, stride);
        return;
    }
    if (q < p.groups) sir_tail_group<false>(p, q, t);
}

// tail (box mode): transition(t) from K.
__global__ void k_sir_tail_box(SirParams p, uint32_t t)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < p.groups) sir_tail_group<true>(p, q, t);
}

// box (box mode): K = box sum of C_t; clears C_{t+1}.  One thread per 4 cells.
__global__ void k_sir_box(SirParams p, uint32_t t)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    zero_quads(cgrid_box(p, t + 1), p.quads, i, gridDim.x * blockDim.x);
    if (i < p.quads) sir_box_quad(p, cgrid_box(p, t), kgrid_box(p), i);
}

// Exchange count mode: producer (transition(t-1) if TRANSITION, move(t),
// sorted records of bin(t)) and the per-band count kernel writing K.
constexpr uint32_t XPMAX = 2048;             // bands the producer can sort into
constexpr uint32_t XHIST = 16384;            // LDS counters of a band plus halo rows

template <bool TRANSITION>
__global__ __launch_bounds__(256) void k_sir_xbody(SirParams p, uint32_t t)
{
    __shared__ uint32_t pcount[XPMAX];
    __shared__ uint32_t poff[XPMAX];
    sir_exchange_produce<TRANSITION>(p, blockIdx.x, t, pcount, poff);
}

__global__ __launch_bounds__(256) void k_sir_xcount(SirParams p)
{
    __shared__ uint32_t hist[XHIST];
    __shared__ uint32_t scnt[XCHUNK];
    __shared__ uint32_t soff[XCHUNK];
    __shared__ uint32_t sraw[XCHUNK];
    sir_exchange_count(p, blockIdx.x, hist, scnt, soff, sraw);
}

// Clear the count grids in mask (bit b = count[b]) at the end of a call.
__global__ void k_sir_clear(SirParams p, uint32_t mask)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (int b = 0; b < 3; ++b)
        if (mask & (1u << b)) zero_quads(p.count[b], p.quads, i, stride);
    // the demand-binning step counts and flags start the next call at zero
    sir_demand_reset(p, i, stride);
}

// ------------------------------------------------------------------ SIR, persistent form
// One cooperative launch runs every step of the call.  Each thread keeps G
// groups of 4 agents (positions and states) in registers; the only data
// shared between workgroups are the count grids, and every access to them
// uses agent-scope atomics (adds, stores, loads), which are coherent across
// the XCDs' separate L2 caches without whole-cache write-backs.  One
// device-wide barrier per step separates bin(t) from transition(t).
//
// The barrier is two-level: workgroups arrive on one of several group
// counters (each on its own 128-byte line), the last arrival of a group bumps
// the top counter, and every workgroup waits for the top counter.  Waits are
// bounded: a wait that exceeds SYNC_SPIN_LIMIT sets a sticky error flag
// (reported by the host at the next synchronising call) and every later wait
// returns at once, so the kernel always runs to completion.

constexpr uint32_t SYNC_STRIDE = 32;          // words between counters (128 B)
constexpr uint32_t SYNC_SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void grid_sync(const SyncParams &s, uint32_t epoch)
{
    __builtin_amdgcn_s_waitcnt(0);   // this wave's adds and stores have been performed
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t g = blockIdx.x / s.group_size;
        const uint32_t first = g * s.group_size;
        const uint32_t members = min(s.group_size, gridDim.x - first);
        const uint32_t old = __hip_atomic_fetch_add(&s.words[g * SYNC_STRIDE], 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        uint32_t *top = &s.words[s.ngroups * SYNC_STRIDE];
        if (old + 1 == epoch * members)
            __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (ld_agent(top) < epoch * s.ngroups) {
            if ((++spins & 255u) == 0 && (spins > SYNC_SPIN_LIMIT || ld_agent(s.err))) {
                __hip_atomic_fetch_or(s.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
}

// Infected agents in the distinct cells of the 3x3 block, read coherently.
__device__ __forceinline__ uint32_t block_count_agent(const uint32_t *__restrict__ count, int32_t L,
                                                      int32_t cx, int32_t cy)
{
    if (!on_grid(cx, cy, L)) return 0;
    if (L >= 3) {
        const int32_t xm = cx == 0 ? L - 1 : cx - 1;
        const int32_t xp = cx == L - 1 ? 0 : cx + 1;
        const int32_t ym = cy == 0 ? L - 1 : cy - 1;
        const int32_t yp = cy == L - 1 ? 0 : cy + 1;
        const uint32_t *rm = count + (uint32_t)ym * L;
        const uint32_t *r0 = count + (uint32_t)cy * L;
        const uint32_t *rp = count + (uint32_t)yp * L;
        return ld_agent(rm + xm) + ld_agent(rm + cx) + ld_agent(rm + xp) + ld_agent(r0 + xm) +
               ld_agent(r0 + cx) + ld_agent(r0 + xp) + ld_agent(rp + xm) + ld_agent(rp + cx) +
               ld_agent(rp + xp);
    }
    uint32_t k = 0;
    for (int32_t c = 0; c < L * L; ++c) k += ld_agent(count + c);
    return k;
}

// transition(t) with coherent count reads (same rule as sir_transition4).
__device__ __forceinline__ uint32_t sir_transition4_agent(const SirParams &p,
                                                          const uint32_t *__restrict__ count,
                                                          uint32_t q, uint32_t t, uint32_t S,
                                                          const int4 &X, const int4 &Y)
{
    const uint32_t a = 4 * q;
    uint32_t st[4], k[4] = {0, 0, 0, 0};
    bool any_sus = false, need = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        st[j] = (a + j < p.n) ? (S >> (8 * j)) & 0xffu : (uint32_t)ST_R;
        any_sus |= st[j] == ST_S;
    }
    if (any_sus) {
        if (st[0] == ST_S) k[0] = block_count_agent(count, p.L, X.x, Y.x);
        if (st[1] == ST_S) k[1] = block_count_agent(count, p.L, X.y, Y.y);
        if (st[2] == ST_S) k[2] = block_count_agent(count, p.L, X.z, Y.z);
        if (st[3] == ST_S) k[3] = block_count_agent(count, p.L, X.w, Y.w);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) need |= (st[j] == ST_S && k[j] > 0) || st[j] == ST_I;
    if (!need) return S;
    const uint4 r = philox(q, t, P_EPI, p.k0, p.k1);
    const uint32_t u[4] = {r.x, r.y, r.z, r.w};
    const uint32_t k_last = p.table_len - 1;
    uint32_t out = S;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t ns = st[j];
        if (st[j] == ST_S && k[j] > 0) {
            if (u[j] < p.t_inf[k[j] < k_last ? k[j] : k_last]) ns = ST_I;
        } else if (st[j] == ST_I) {
            if (u[j] < p.t_rec) ns = ST_R;
        }
        out = (out & ~(0xffu << (8 * j))) | (ns << (8 * j));
    }
    return out;
}

template <int G>
__global__ __launch_bounds__(256) void k_sir_persistent(SirParams p, SyncParams sync, uint32_t t0,
                                                        uint32_t n_steps)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nthr = gridDim.x * blockDim.x;
    int4 X[G], Y[G];
    uint32_t S[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t q = tid + g * nthr;
        if (q < p.groups) {
            X[g] = ((const int4 *)p.x)[q];
            Y[g] = ((const int4 *)p.y)[q];
            S[g] = ((const uint32_t *)p.s)[q];
        } else {
            X[g] = Y[g] = make_int4(0, 0, 0, 0);
            S[g] = 0x02020202u;
        }
    }
    const uint32_t words = p.quads * 4;
    for (uint32_t i = 0; i < n_steps; ++i) {
        const uint32_t t = t0 + i;
        uint32_t *cur = grid_of(p, t);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t q = tid + g * nthr;
            if (q < p.groups) {
                sir_move4(p, q, t, X[g], Y[g]);
                sir_bin4(p, cur, q, S[g], X[g], Y[g]);   // agent-scope atomic adds
            }
        }
        grid_sync(sync, i + 1);
        uint32_t *clr = grid_of(p, t + 2);
        for (uint32_t w = tid; w < words; w += nthr) st_agent(clr + w, 0u);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t q = tid + g * nthr;
            if (q < p.groups) S[g] = sir_transition4_agent(p, cur, q, t, S[g], X[g], Y[g]);
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t q = tid + g * nthr;
        if (q < p.groups) {
            ((int4 *)p.x)[q] = X[g];
            ((int4 *)p.y)[q] = Y[g];
            ((uint32_t *)p.s)[q] = S[g];
        }
    }
}

__global__ void k_sync_reset(uint32_t *words, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) words[i] = 0;
}

// ------------------------------------------------------------------ invariants

__device__ __forceinline__ uint64_t fmix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t mix_col(uint64_t h, uint32_t col, uint32_t v)
{
    return fmix64(h ^ (((uint64_t)(col + 1) << 32) | v));
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_min(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

struct InvAcc {
    unsigned long long wsum, ns, ni, nr, oob, dig;
    int wmin;
};

__device__ __forceinline__ void inv_wave_reduce(InvAcc &v)
{
    v.wsum = wave_sum(v.wsum);
    v.ns = wave_sum(v.ns);
    v.ni = wave_sum(v.ni);
    v.nr = wave_sum(v.nr);
    v.oob = wave_sum(v.oob);
    v.dig = wave_sum(v.dig);
    v.wmin = wave_min(v.wmin);
}

// Reduce the accumulators of a 256-thread workgroup; thread 0 returns the total.
__device__ __forceinline__ void inv_block_reduce(InvAcc &v)
{
    __shared__ InvAcc part[4];
    inv_wave_reduce(v);
    const uint32_t wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t w = 1; w < blockDim.x / 64; ++w) {
            v.wsum += part[w].wsum;
            v.ns += part[w].ns;
            v.ni += part[w].ni;
            v.nr += part[w].nr;
            v.oob += part[w].oob;
            v.dig += part[w].dig;
            v.wmin = min(v.wmin, part[w].wmin);
        }
    }
}

__device__ __forceinline__ void inv_store(DevInvariants *d, const InvAcc &v)
{
    d->wealth_sum = v.wsum;
    d->n_s = v.ns;
    d->n_i = v.ni;
    d->n_r = v.nr;
    d->out_of_bounds = v.oob;
    d->digest = v.dig;
    d->wealth_min = v.wmin;
}

// Stage 1: workgroup b reduces a grid-stride share of the agents into partials[b].
__global__ __launch_bounds__(256) void k_invariants(uint32_t model, uint32_t n, int32_t L,
                                                    const int32_t *__restrict__ w,
                                                    const int32_t *__restrict__ x,
                                                    const int32_t *__restrict__ y,
                                                    const uint8_t *__restrict__ s,
                                                    DevInvariants *__restrict__ partials)
{
    InvAcc v{0, 0, 0, 0, 0, 0, 0x7fffffff};
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += stride) {
        uint64_t h = fmix64((uint64_t)a);
        bool bad = false;
        if (model == 0) {
            const int32_t wv = w[a];
            v.wsum += (unsigned long long)(long long)wv;
            v.wmin = min(v.wmin, wv);
            bad = wv < 0;
            h = mix_col(h, 0, (uint32_t)wv);
        } else {
            const int32_t px = x[a], py = y[a];
            bad = !on_grid(px, py, L);
            h = mix_col(h, 0, (uint32_t)px);
            h = mix_col(h, 1, (uint32_t)py);
            if (model == 2) {
                const uint32_t sv = s[a];
                v.ns += sv == ST_S;
                v.ni += sv == ST_I;
                v.nr += sv == ST_R;
                bad |= sv > ST_R;
                h = mix_col(h, 2, sv);
            }
        }
        v.oob += bad;
        v.dig += h;
    }
    inv_block_reduce(v);
    if (threadIdx.x == 0) inv_store(&partials[blockIdx.x], v);
}

// Stage 2: one workgroup folds the partials.
__global__ __launch_bounds__(256) void k_invariants_final(const DevInvariants *__restrict__ partials,
                                                          uint32_t count, DevInvariants *acc)
{
    InvAcc v{0, 0, 0, 0, 0, 0, 0x7fffffff};
    for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) {
        const DevInvariants &d = partials[i];
        v.wsum += d.wealth_sum;
        v.ns += d.n_s;
        v.ni += d.n_i;
        v.nr += d.n_r;
        v.oob += d.out_of_bounds;
        v.dig += d.digest;
        v.wmin = min(v.wmin, d.wealth_min);
    }
    inv_block_reduce(v);
    if (threadIdx.x == 0) inv_store(acc, v);
}
// ------------------------------------------------------------------ launchers

static inline dim3 grid_for(uint32_t items, uint32_t block) { return dim3(div_up(items, block)); }

hipError_t launch_init_wealth(int32_t *w, int32_t *inc0, int32_t *inc1, uint32_t n,
                              int32_t w_init, hipStream_t st)
{
    const uint32_t g = padded_groups(n);
    hipLaunchKernelGGL(k_init_wealth, grid_for(g, 256), dim3(256), 0, st, (int4 *)w,
                       (int4 *)inc0, (int4 *)inc1, g, n, w_init);
    return hipGetLastError();
}

hipError_t launch_init_positions(int32_t *x, int32_t *y, uint32_t n, int32_t L, uint32_t k0,
                                 uint32_t k1, hipStream_t st)
{
    const uint32_t g = padded_groups(n);
    hipLaunchKernelGGL(k_init_positions, grid_for(g, 256), dim3(256), 0, st, (int4 *)x,
                       (int4 *)y, g, L, k0, k1);
    return hipGetLastError();
}

hipError_t launch_init_states(uint8_t *s, uint32_t n, uint32_t i0, hipStream_t st)
{
    const uint32_t g = padded_groups(n);
    hipLaunchKernelGGL(k_init_states, grid_for(g, 256), dim3(256), 0, st, (uint32_t *)s, g, i0);
    return hipGetLastError();
}

// Words passed by value: kernel arguments are copied when the launch is
// enqueued, so a small host table reaches the device with no staged copy
// from pageable memory (which holds the host until the stream drains).
constexpr uint32_t WRITE_CHUNK = 960;          // 3840 bytes of kernel arguments
struct WordChunk {
    uint32_t w[WRITE_CHUNK];
};

__global__ __launch_bounds__(256) void k_write_words(uint32_t *__restrict__ dst, WordChunk c,
                                                     uint32_t count)
{
    for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) dst[i] = c.w[i];
}

hipError_t launch_write_words(uint32_t *dst, const uint32_t *src, uint64_t count, hipStream_t st)
{
    for (uint64_t o = 0; o < count; o += WRITE_CHUNK) {
        WordChunk c;
        const uint32_t k = (uint32_t)(count - o < WRITE_CHUNK ? count - o : WRITE_CHUNK);
        for (uint32_t i = 0; i < k; ++i) c.w[i] = src[o + i];
        hipLaunchKernelGGL(k_write_words, dim3(1), dim3(256), 0, st, dst + o, c, k);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_zero_words(uint32_t *p, uint64_t words, hipStream_t st)
{
    const uint64_t quads = words / 4;   // callers pass multiples of 4 words
    const uint32_t blocks = (uint32_t)((quads + 255) / 256 < 4096 ? (quads + 255) / 256 : 4096);
    if (quads == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, st, (uint4 *)p, quads);
    return hipGetLastError();
}

hipError_t launch_walk(int32_t *x, int32_t *y, uint32_t n, int32_t L, uint32_t k0, uint32_t k1,
                       uint32_t t0, uint32_t n_steps, const Tuning &tu, hipStream_t st)
{
    const uint32_t g = groups_of(n);
    hipLaunchKernelGGL(k_walk, grid_for(g, tu.block), dim3(tu.block), 0, st, (int4 *)x,
                       (int4 *)y, g, L, k0, k1, t0, n_steps);
    return hipGetLastError();
}

hipError_t launch_wealth_step(int32_t *base, int32_t *inc_cur, int32_t *inc_nxt, uint32_t n,
                              uint32_t k0, uint32_t k1, uint32_t t, const Tuning &tu,
                              hipStream_t st)
{
    const uint32_t g = groups_of(n);
    hipLaunchKernelGGL(k_wealth_step, grid_for(g, tu.block), dim3(tu.block), 0, st,
                       (int4 *)base, (int4 *)inc_cur, inc_nxt, g, n, k0, k1, t);
    return hipGetLastError();
}

hipError_t launch_wealth_fold(int32_t *base, int32_t *inc, uint32_t n, hipStream_t st)
{
    const uint32_t g = groups_of(n);
    hipLaunchKernelGGL(k_wealth_fold, grid_for(g, 256), dim3(256), 0, st, (int4 *)base,
                       (int4 *)inc, g);
    return hipGetLastError();
}

uint32_t wealth_small_max_agents() { return WEALTH_SMALL_MAX; }

uint32_t wealth_exchange_bits(uint32_t n)
{
    if (n <= (1u << 20)) return 11;            // up to 512 partitions of 2048 agents
    if (n <= (1u << 21)) return 12;            // up to 512 partitions of 4096 agents
    if (n <= (1u << 24)) return 14;            // up to 1024 partitions of 16384 agents
    if (n <= (5u << 23)) return 15;            // up to 1280 partitions of 32768 agents
    if (n <= (1u << 27)) return 16;            // 641 to 2048 partitions of 65536 agents
    return 0;                                  // too many partitions: atomic path
}

hipError_t launch_wealth_exchange(const WealthXParams &x, uint32_t t, uint32_t parity_in,
                                  uint32_t mode, uint32_t bits, hipStream_t st)
{
    if (bits == 11) {
        if (x.P > 512) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_wealth_x<11, 512, 512>), dim3(x.P), dim3(512), 0, st, x, t, parity_in,
                           mode);
    } else if (bits == 12) {
        if (x.P > 512) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_wealth_x<12, 512, 1024>), dim3(x.P), dim3(1024), 0, st, x, t,
                           parity_in, mode);
    } else if (bits == 14) {
        if (x.P > 1024) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_wealth_x<14, 1024, 1024>), dim3(x.P), dim3(1024), 0, st, x, t,
                           parity_in, mode);
    } else if (bits == 15) {
        if (x.P > 1280) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_wealth_x16<15, 1280, 1024>), dim3(x.P), dim3(1024), 0, st, x, t,
                           parity_in, mode);
    } else if (bits == 16) {
        if (x.P > 2048) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_wealth_x16<16, 2048, 1024>), dim3(x.P), dim3(1024), 0, st, x, t,
                           parity_in, mode);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_wealth_small(int32_t *w, uint32_t n, uint32_t k0, uint32_t k1, uint32_t t0,
                               uint32_t n_steps, hipStream_t st)
{
    if (n > WEALTH_SMALL_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_wealth_small, dim3(1), dim3(WEALTH_SMALL_THREADS), 0, st, w, n, k0, k1,
                       t0, n_steps);
    return hipGetLastError();
}

void sir_fill(SirParams &p)
{
    p.groups = groups_of(p.n);
    p.quads = div_up((uint32_t)p.L * (uint32_t)p.L, 4);
    p.dquads = div_up((uint32_t)p.L * (uint32_t)p.L, 16);
}

hipError_t launch_sir_head(SirParams p, uint32_t t, bool box, const Tuning &tu, hipStream_t st)
{
    sir_fill(p);
    if (box)
        hipLaunchKernelGGL(k_sir_head<true>, grid_for(p.groups, tu.block), dim3(tu.block), 0, st, p, t);
    else   // one extra workgroup for the demand-binning bookkeeping
        hipLaunchKernelGGL(k_sir_head<false>, dim3(grid_for(p.groups, tu.block).x + 1),
                           dim3(tu.block), 0, st, p, t);
    return hipGetLastError();
}

hipError_t launch_sir_body(SirParams p, uint32_t t, bool box, const Tuning &tu, hipStream_t st)
{
    sir_fill(p);
    if (box)
        hipLaunchKernelGGL(k_sir_body_box, grid_for(p.groups, tu.block), dim3(tu.block), 0, st, p, t);
    else   // one extra workgroup for the demand-binning bookkeeping
        hipLaunchKernelGGL(k_sir_body, dim3(grid_for(p.groups, tu.block).x + 1), dim3(tu.block), 0,
                           st, p, t);
    return hipGetLastError();
}

hipError_t launch_sir_tail(SirParams p, uint32_t t, uint32_t i_last, bool box, const Tuning &tu,
                           hipStream_t st)
{
    sir_fill(p);
    if (box)
        hipLaunchKernelGGL(k_sir_tail_box, grid_for(p.groups, tu.block), dim3(tu.block), 0, st, p, t);
    else
        hipLaunchKernelGGL(k_sir_tail, grid_for(p.groups, tu.block), dim3(tu.block), 0, st, p, t,
                           i_last);
    return hipGetLastError();
}

hipError_t launch_sir_box(SirParams p, uint32_t t, hipStream_t st)
{
    sir_fill(p);
    hipLaunchKernelGGL(k_sir_box, grid_for(p.quads, 256), dim3(256), 0, st, p, t);
    return hipGetLastError();
}

bool sir_exchange_shape(uint32_t n, uint32_t L, uint32_t *h_out, uint32_t *P_out, uint32_t *W_out)
{
    if (L < 3) return false;
    uint32_t h = (L + 255) / 256;
    const uint32_t hmax = XHIST / L >= 3 ? XHIST / L - 2 : 0;
    if (h > hmax) h = hmax;
    if (h == 0) return false;
    const uint32_t P = (L + h - 1) / h;
    const uint32_t W = div_up(groups_of(n), 256);
    if (P < 3 || P > XPMAX || (uint64_t)W * P > (32ull << 20)) return false;
    *h_out = h;
    *P_out = P;
    *W_out = W;
    return true;
}

hipError_t launch_sir_xbody(SirParams p, uint32_t t, bool transition, hipStream_t st)
{
    sir_fill(p);
    if (transition)
        hipLaunchKernelGGL(k_sir_xbody<true>, dim3(p.xW), dim3(256), 0, st, p, t);
    else
        hipLaunchKernelGGL(k_sir_xbody<false>, dim3(p.xW), dim3(256), 0, st, p, t);
    return hipGetLastError();
}

hipError_t launch_sir_xcount(SirParams p, hipStream_t st)
{
    sir_fill(p);
    hipLaunchKernelGGL(k_sir_xcount, dim3(p.xP), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_sir_clear(SirParams p, uint32_t mask, hipStream_t st)
{
    sir_fill(p);
    uint32_t blocks = div_up(p.quads, 256);
    if (blocks > 2048) blocks = 2048;
    if (blocks < div_up(4 * 2 * NSI_SLOTS, 256)) blocks = div_up(4 * 2 * NSI_SLOTS, 256);   // counts too
    hipLaunchKernelGGL(k_sir_clear, dim3(blocks), dim3(256), 0, st, p, mask);
    return hipGetLastError();
}

// Co-resident workgroups of 256 threads for the persistent SIR kernel with G
// groups per thread on the current device (0 if it cannot run).
template <int G>
static uint32_t persistent_capacity()
{
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop)
        return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sir_persistent<G>, 256, 0) !=
        hipSuccess)
        return 0;
    return (uint32_t)(cus * per_cu);
}

template <int G>
static hipError_t launch_persistent_g(SirParams p, SyncParams sync, uint32_t t0, uint32_t n_steps,
                                      uint32_t blocks, hipStream_t st)
{
    void *args[] = {&p, &sync, &t0, &n_steps};
    return hipLaunchCooperativeKernel((const void *)k_sir_persistent<G>, dim3(blocks), dim3(256),
                                      args, 0, st);
}

uint32_t sir_persistent_groups_per_thread(uint32_t n, uint32_t max_g, uint32_t *blocks_out)
{
    const uint32_t groups = groups_of(n);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    // Fewer workgroups make the barrier cheaper (arrivals serialise on the
    // counters); more workgroups hide more latency.  Take the smallest G that
    // fits in at most two workgroups per CU, else the smallest that fits.
    uint32_t best_g = 0, best_blocks = 0;
    static const uint32_t gs[] = {1, 2, 4, 8};
    for (uint32_t g : gs) {
        if (g > max_g) break;
        uint32_t cap = 0;
        switch (g) {
        case 1: cap = persistent_capacity<1>(); break;
        case 2: cap = persistent_capacity<2>(); break;
        case 4: cap = persistent_capacity<4>(); break;
        case 8: cap = persistent_capacity<8>(); break;
        }
        const uint32_t need = div_up(groups, 256 * g);
        const uint32_t max_blocks = (SYNC_WORDS / SYNC_STRIDE - 1) * 16;
        if (!cap || need > cap || need > max_blocks) continue;
        if (!best_g) {
            best_g = g;
            best_blocks = need;
        }
        if (need <= 2u * (uint32_t)cus) {
            best_g = g;
            best_blocks = need;
            break;
        }
    }
    if (blocks_out) *blocks_out = best_blocks;
    return best_g;
}

hipError_t launch_sir_persistent(SirParams p, uint32_t *sync_words, uint32_t *err, uint32_t t0,
                                 uint32_t n_steps, uint32_t g, uint32_t blocks, hipStream_t st)
{
    sir_fill(p);
    SyncParams sync;
    sync.words = sync_words;
    sync.err = err;
    sync.group_size = 16;
    sync.ngroups = div_up(blocks, sync.group_size);
    if ((sync.ngroups + 1) * SYNC_STRIDE > SYNC_WORDS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sync_reset, dim3(1), dim3(256), 0, st, sync_words,
                       (sync.ngroups + 1) * SYNC_STRIDE);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (g) {
    case 1: return launch_persistent_g<1>(p, sync, t0, n_steps, blocks, st);
    case 2: return launch_persistent_g<2>(p, sync, t0, n_steps, blocks, st);
    case 4: return launch_persistent_g<4>(p, sync, t0, n_steps, blocks, st);
    case 8: return launch_persistent_g<8>(p, sync, t0, n_steps, blocks, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_invariants(uint32_t model, uint32_t n, int32_t L, const int32_t *w,
                             const int32_t *x, const int32_t *y, const uint8_t *s,
                             DevInvariants *acc, DevInvariants *partials, hipStream_t st)
{
    uint32_t blocks = div_up(n, 256 * 4);
    if (blocks > INV_MAX_BLOCKS) blocks = INV_MAX_BLOCKS;
    hipLaunchKernelGGL(k_invariants, dim3(blocks), dim3(256), 0, st, model, n, L, w, x, y, s,
                       partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_invariants_final, dim3(1), dim3(256), 0, st, partials, blocks, acc);
    return hipGetLastError();
}

}  // namespace amber
