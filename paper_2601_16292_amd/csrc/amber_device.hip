// amber_device.hip -- gfx950 kernels of the columnar ABM hot path.
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
#include "amber_internal.h"

namespace amber {

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Multipliers and Weyl
// key increments as published.  The key lives in SGPRs (wavefront-uniform);
// each 32x32->64 product is one v_mad_u64_u32.
constexpr uint32_t PHILOX_M0 = 0xD2511F53u;
constexpr uint32_t PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u;
constexpr uint32_t PHILOX_W1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2,
                                        uint32_t k0, uint32_t k1)
{
    uint32_t c3 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        const uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    return make_uint4(c0, c1, c2, c3);
}

// ------------------------------------------------------------------ mappings
// Moore move from the top 3 bits of a word: index d selects (dx, dy) from the
// 8 moves in lexicographic order without (0,0).  The tables hold dx+1 and
// dy+1 as 2-bit fields at bit 2d.
constexpr uint32_t MOVE_DX1 = (0u << 0) | (0u << 2) | (0u << 4) | (1u << 6) | (1u << 8) |
                              (2u << 10) | (2u << 12) | (2u << 14);
constexpr uint32_t MOVE_DY1 = (0u << 0) | (1u << 2) | (2u << 4) | (0u << 6) | (2u << 8) |
                              (0u << 10) | (1u << 12) | (2u << 14);

// Torus step of one coordinate in [0, L) by d in {-1, 0, 1}.
__device__ __forceinline__ int32_t wrap_step(int32_t v, int32_t d, int32_t L)
{
    v += d;
    v = (v < 0) ? v + L : v;
    v = (v >= L) ? v - L : v;
    return v;
}

__device__ __forceinline__ void moore_move(uint32_t u, int32_t L, int32_t &x, int32_t &y)
{
    const uint32_t sh = (u >> 28) & 14u;   // 2 * (u >> 29)
    x = wrap_step(x, (int32_t)((MOVE_DX1 >> sh) & 3u) - 1, L);
    y = wrap_step(y, (int32_t)((MOVE_DY1 >> sh) & 3u) - 1, L);
}

// floor(u * L / 2^32)
__device__ __forceinline__ int32_t grid_coord(uint32_t u, int32_t L)
{
    return (int32_t)__umulhi(u, (uint32_t)L);
}

// floor((hi:lo) * n / 2^64) for n < 2^32.
__device__ __forceinline__ uint32_t recipient(uint32_t hi, uint32_t lo, uint32_t n)
{
    const uint64_t lo_n = (uint64_t)lo * n;
    const uint64_t mid = (uint64_t)hi * n + (lo_n >> 32);
    return (uint32_t)(mid >> 32);
}

__host__ __device__ inline uint32_t div_up(uint32_t a, uint32_t b) { return (a + b - 1) / b; }
__host__ __device__ inline uint32_t groups_of(uint32_t n) { return div_up(n, 4); }
__host__ __device__ inline uint32_t padded_groups(uint32_t n) { return div_up(n, AGENT_PAD) * (AGENT_PAD / 4); }

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
    if (q >= groups) return;
    int4 X = x[q];
    int4 Y = y[q];
    for (uint32_t i = 0; i < n_steps; ++i) {
        const uint4 r = philox(q, t0 + i, P_MOVE, k0, k1);
        moore_move(r.x, L, X.x, Y.x);
        moore_move(r.y, L, X.y, Y.y);
        moore_move(r.z, L, X.z, Y.z);
        moore_move(r.w, L, X.w, Y.w);
    }
    x[q] = X;
    y[q] = Y;
}

// ------------------------------------------------------------------ wealth
// One synchronous transfer step.  The state of agent a is base[a] +
// inc_cur[a]; the snapshot decides the donors (wealth > 0).  A donor's unit
// leaves base in place (plain store, the thread owns the row) and lands in
// inc_nxt[recipient] through an integer atomic add, so duplicates accumulate
// in any order with an identical result.  inc_cur is cleared for reuse two
// steps later.
__global__ void k_wealth_step(int4 *__restrict__ base, int4 *__restrict__ inc_cur,
                              int32_t *__restrict__ inc_nxt, uint32_t groups, uint32_t n,
                              uint32_t k0, uint32_t k1, uint32_t t)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= groups) return;
    const int4 B = base[q];
    const int4 I = inc_cur[q];
    const int32_t v0 = B.x + I.x, v1 = B.y + I.y, v2 = B.z + I.z, v3 = B.w + I.w;
    const uint32_t a = 4 * q;
    const bool d0 = v0 > 0 && a + 0 < n;
    const bool d1 = v1 > 0 && a + 1 < n;
    const bool d2 = v2 > 0 && a + 2 < n;
    const bool d3 = v3 > 0 && a + 3 < n;
    base[q] = make_int4(v0 - d0, v1 - d1, v2 - d2, v3 - d3);
    inc_cur[q] = make_int4(0, 0, 0, 0);
    if (d0 | d1) {
        const uint4 r = philox(2 * q, t, P_RECIPIENT, k0, k1);
        if (d0) atomicAdd(&inc_nxt[recipient(r.x, r.y, n)], 1);
        if (d1) atomicAdd(&inc_nxt[recipient(r.z, r.w, n)], 1);
    }
    if (d2 | d3) {
        const uint4 r = philox(2 * q + 1, t, P_RECIPIENT, k0, k1);
        if (d2) atomicAdd(&inc_nxt[recipient(r.x, r.y, n)], 1);
        if (d3) atomicAdd(&inc_nxt[recipient(r.z, r.w, n)], 1);
    }
}

__global__ void k_wealth_fold(int4 *__restrict__ base, int4 *__restrict__ inc, uint32_t groups)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= groups) return;
    const int4 B = base[q];
    const int4 I = inc[q];
    base[q] = make_int4(B.x + I.x, B.y + I.y, B.z + I.z, B.w + I.w);
    inc[q] = make_int4(0, 0, 0, 0);
}

// Small populations: one workgroup runs every step with the wealth column and
// the increments in LDS; two barriers per step separate the donor/scatter
// phase from the apply phase.  A thread owns agent pairs (one RECIPIENT
// block per pair).
constexpr uint32_t WEALTH_SMALL_THREADS = 1024;
constexpr uint32_t WEALTH_SMALL_MAX = 8192;   // 2 x 32 KB of LDS

__global__ __launch_bounds__(WEALTH_SMALL_THREADS) void k_wealth_small(
    int32_t *__restrict__ w, uint32_t n, uint32_t k0, uint32_t k1, uint32_t t0, uint32_t n_steps)
{
    __shared__ int32_t sw[WEALTH_SMALL_MAX];
    __shared__ int32_t sinc[WEALTH_SMALL_MAX];
    for (uint32_t a = threadIdx.x; a < n; a += blockDim.x) {
        sw[a] = w[a];
        sinc[a] = 0;
    }
    __syncthreads();
    const uint32_t pairs = div_up(n, 2);
    for (uint32_t i = 0; i < n_steps; ++i) {
        const uint32_t t = t0 + i;
        for (uint32_t p = threadIdx.x; p < pairs; p += blockDim.x) {
            const uint32_t a = 2 * p;
            const int32_t v0 = sw[a];
            const int32_t v1 = (a + 1 < n) ? sw[a + 1] : 0;
            const bool d0 = v0 > 0, d1 = v1 > 0;
            if (d0 | d1) {
                const uint4 r = philox(p, t, P_RECIPIENT, k0, k1);
                if (d0) {
                    sw[a] = v0 - 1;
                    atomicAdd(&sinc[recipient(r.x, r.y, n)], 1);
                }
                if (d1) {
                    sw[a + 1] = v1 - 1;
                    atomicAdd(&sinc[recipient(r.z, r.w, n)], 1);
                }
            }
        }
        __syncthreads();
        for (uint32_t a = threadIdx.x; a < n; a += blockDim.x) {
            sw[a] += sinc[a];
            sinc[a] = 0;
        }
        __syncthreads();
    }
    for (uint32_t a = threadIdx.x; a < n; a += blockDim.x) w[a] = sw[a];
}

// ------------------------------------------------------------------ SIR

// Positions come from the caller's columns; a coordinate outside [0, L) (only
// possible if the caller overwrote a column) is never used as an address.
__device__ __forceinline__ bool on_grid(int32_t x, int32_t y, int32_t L)
{
    return (uint32_t)x < (uint32_t)L && (uint32_t)y < (uint32_t)L;
}

__device__ __forceinline__ void bin_infected(uint32_t *__restrict__ count, int32_t L, bool inf,
                                             int32_t x, int32_t y)
{
    if (inf && on_grid(x, y, L)) atomicAdd(&count[(uint32_t)y * L + x], 1u);
}

// Phase 1: move every agent (same words and rule as the random walk) and
// count the agents infected at the start of the step in their post-move cell.
__global__ void k_sir_move_bin(int4 *__restrict__ x, int4 *__restrict__ y,
                               const uint32_t *__restrict__ s4, uint32_t *__restrict__ count,
                               uint32_t groups, uint32_t n, int32_t L, uint32_t k0, uint32_t k1,
                               uint32_t t)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= groups) return;
    int4 X = x[q];
    int4 Y = y[q];
    const uint32_t S = s4[q];
    const uint4 r = philox(q, t, P_MOVE, k0, k1);
    moore_move(r.x, L, X.x, Y.x);
    moore_move(r.y, L, X.y, Y.y);
    moore_move(r.z, L, X.z, Y.z);
    moore_move(r.w, L, X.w, Y.w);
    x[q] = X;
    y[q] = Y;
    const uint32_t a = 4 * q;
    bin_infected(count, L, (S & 0xffu) == ST_I && a + 0 < n, X.x, Y.x);
    bin_infected(count, L, ((S >> 8) & 0xffu) == ST_I && a + 1 < n, X.y, Y.y);
    bin_infected(count, L, ((S >> 16) & 0xffu) == ST_I && a + 2 < n, X.z, Y.z);
    bin_infected(count, L, (S >> 24) == ST_I && a + 3 < n, X.w, Y.w);
}

// Infected agents in the distinct cells of the 3x3 torus block around (cx, cy).
__device__ __forceinline__ uint32_t block_count(const uint32_t *__restrict__ count, int32_t L,
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
        return rm[xm] + rm[cx] + rm[xp] + r0[xm] + r0[cx] + r0[xp] + rp[xm] + rp[cx] + rp[xp];
    }
    // L = 1 or 2: the wrapped block covers each of the L*L cells exactly once.
    uint32_t k = 0;
    for (int32_t c = 0; c < L * L; ++c) k += count[c];
    return k;
}

// Phase 2: state transitions from the snapshot state and the counts; clears
// the other count buffer for the next step.
__global__ void k_sir_transition(const int4 *__restrict__ x, const int4 *__restrict__ y,
                                 uint32_t *__restrict__ s4, const uint32_t *__restrict__ count,
                                 uint4 *__restrict__ count_next, uint32_t count_quads,
                                 const uint32_t *__restrict__ t_inf, uint32_t k_last,
                                 uint32_t t_rec, uint32_t groups, uint32_t n, int32_t L,
                                 uint32_t k0, uint32_t k1, uint32_t t)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = q; i < count_quads; i += stride) count_next[i] = make_uint4(0, 0, 0, 0);
    if (q >= groups) return;

    const uint32_t S = s4[q];
    const uint32_t a = 4 * q;
    uint32_t st[4], k[4];
    bool any_sus = false;
    for (int j = 0; j < 4; ++j) {
        st[j] = (a + j < n) ? (S >> (8 * j)) & 0xffu : (uint32_t)ST_R;   // padding never changes
        any_sus |= st[j] == ST_S;
        k[j] = 0;
    }
    if (any_sus) {
        const int4 X = x[q];
        const int4 Y = y[q];
        if (st[0] == ST_S) k[0] = block_count(count, L, X.x, Y.x);
        if (st[1] == ST_S) k[1] = block_count(count, L, X.y, Y.y);
        if (st[2] == ST_S) k[2] = block_count(count, L, X.z, Y.z);
        if (st[3] == ST_S) k[3] = block_count(count, L, X.w, Y.w);
    }
    bool need = false;
    for (int j = 0; j < 4; ++j) need |= (st[j] == ST_S && k[j] > 0) || st[j] == ST_I;
    if (!need) return;
    const uint4 r = philox(q, t, P_EPI, k0, k1);
    const uint32_t u[4] = {r.x, r.y, r.z, r.w};
    uint32_t out = S;
    for (int j = 0; j < 4; ++j) {
        uint32_t ns = st[j];
        if (st[j] == ST_S && k[j] > 0) {
            const uint32_t thr = t_inf[k[j] < k_last ? k[j] : k_last];
            if (u[j] < thr) ns = ST_I;
        } else if (st[j] == ST_I) {
            if (u[j] < t_rec) ns = ST_R;
        }
        if (ns != st[j]) out = (out & ~(0xffu << (8 * j))) | (ns << (8 * j));
    }
    if (out != S) s4[q] = out;
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

__global__ void k_inv_clear(DevInvariants *acc)
{
    if (threadIdx.x == 0) {
        acc->wealth_sum = 0;
        acc->n_s = acc->n_i = acc->n_r = 0;
        acc->out_of_bounds = 0;
        acc->digest = 0;
        acc->wealth_min = 0x7fffffff;
    }
}

__global__ void k_invariants(uint32_t model, uint32_t n, int32_t L, const int32_t *__restrict__ w,
                             const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                             const uint8_t *__restrict__ s, DevInvariants *acc)
{
    unsigned long long wsum = 0, ns = 0, ni = 0, nr = 0, oob = 0, dig = 0;
    int wmin = 0x7fffffff;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += stride) {
        uint64_t h = fmix64((uint64_t)a);
        bool bad = false;
        if (model == 0) {
            const int32_t v = w[a];
            wsum += (unsigned long long)(long long)v;
            wmin = min(wmin, v);
            bad = v < 0;
            h = mix_col(h, 0, (uint32_t)v);
        } else {
            const int32_t px = x[a], py = y[a];
            bad = px < 0 || px >= L || py < 0 || py >= L;
            h = mix_col(h, 0, (uint32_t)px);
            h = mix_col(h, 1, (uint32_t)py);
            if (model == 2) {
                const uint32_t sv = s[a];
                ns += sv == ST_S;
                ni += sv == ST_I;
                nr += sv == ST_R;
                bad |= sv > ST_R;
                h = mix_col(h, 2, sv);
            }
        }
        oob += bad;
        dig += h;
    }
    wsum = wave_sum(wsum);
    ns = wave_sum(ns);
    ni = wave_sum(ni);
    nr = wave_sum(nr);
    oob = wave_sum(oob);
    dig = wave_sum(dig);
    wmin = wave_min(wmin);
    if ((threadIdx.x & 63) == 0) {
        if (wsum) atomicAdd(&acc->wealth_sum, wsum);
        if (ns) atomicAdd(&acc->n_s, ns);
        if (ni) atomicAdd(&acc->n_i, ni);
        if (nr) atomicAdd(&acc->n_r, nr);
        if (oob) atomicAdd(&acc->out_of_bounds, oob);
        atomicAdd(&acc->digest, dig);
        if (model == 0) atomicMin(&acc->wealth_min, wmin);
    }
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

hipError_t launch_wealth_small(int32_t *w, uint32_t n, uint32_t k0, uint32_t k1, uint32_t t0,
                               uint32_t n_steps, hipStream_t st)
{
    if (n > WEALTH_SMALL_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_wealth_small, dim3(1), dim3(WEALTH_SMALL_THREADS), 0, st, w, n, k0, k1,
                       t0, n_steps);
    return hipGetLastError();
}

hipError_t launch_sir_step(const SirParams &p, uint32_t t, const Tuning &tu, hipStream_t st)
{
    const uint32_t g = groups_of(p.n);
    const uint32_t cells = (uint32_t)p.L * (uint32_t)p.L;
    const uint32_t quads = div_up(cells, 4);
    uint32_t *cur = p.count[t & 1];
    uint32_t *nxt = p.count[(t + 1) & 1];
    hipLaunchKernelGGL(k_sir_move_bin, grid_for(g, tu.block), dim3(tu.block), 0, st,
                       (int4 *)p.x, (int4 *)p.y, (const uint32_t *)p.s, cur, g, p.n, p.L,
                       p.k0, p.k1, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sir_transition, grid_for(g, tu.block), dim3(tu.block), 0, st,
                       (const int4 *)p.x, (const int4 *)p.y, (uint32_t *)p.s, cur, (uint4 *)nxt,
                       quads, p.t_inf, p.table_len - 1, p.t_rec, g, p.n, p.L, p.k0, p.k1, t);
    return hipGetLastError();
}

hipError_t launch_invariants(uint32_t model, uint32_t n, int32_t L, const int32_t *w,
                             const int32_t *x, const int32_t *y, const uint8_t *s,
                             DevInvariants *acc, hipStream_t st)
{
    hipLaunchKernelGGL(k_inv_clear, dim3(1), dim3(64), 0, st, acc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t blocks = div_up(n, 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_invariants, dim3(blocks), dim3(256), 0, st, model, n, L, w, x, y, s, acc);
    return hipGetLastError();
}

}  // namespace amber
