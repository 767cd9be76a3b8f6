// amber_tiled.hip -- SIR steps on a tile-sorted working copy of the agents
// (count mode 4).
//
// The grid modes pay one random global atomic per infected agent (binning)
// and random gathers per susceptible agent (neighbour counts).  Here the
// agents of a call are grouped by the grid tile that holds them, so one
// workgroup sees every agent of its tile: it bins and sums counts in LDS and
// touches global memory only with streaming loads and stores.  Agents move at
// most one cell per step (the torus Moore move), so an agent leaves its tile
// only for one of the 8 tiles around it, and a tile's next record list is
// its stayers plus what its neighbours send its way.
//
// One launch per step, one workgroup per tile:
//  1. The tile's input is 9 chunks of records: for each tile offset
//     (ddx, ddy), the group that tile (ti - ddx, tj - ddy) sent this way.
//  2. Infected counts of the previous step on the tile and the one-cell ring
//     around it go to LDS: the interior counts that each tile stores for its
//     own cells, plus the ring partial counts of the 9 tiles around (each
//     tile stores the infected agents it moved onto the ring around it).
//  3. Per agent: the transition of the previous step from the 3 x 3 sum in
//     LDS, then the move of this step.  Infected agents are binned into an
//     LDS histogram of the tile and its ring, and the record goes to the
//     group of its destination tile inside the tile's output range (one
//     atomic per tile allocates that range).
//  4. The histogram's interior is stored to the count grid and its ring to
//     the tile's ring array, every cell, so nothing is ever cleared.
// With every tile at least 2 cells wide, all agents that can reach a cell
// within distance 1 of a tile start inside the tile's 3 x 3 block of tiles,
// which is what steps 1 and 2 read.
//
// The arithmetic per agent is the one of the other modes (same Philox words,
// thresholds and integer counts), and sums do not depend on order, so the
// results are identical to theirs.

#include "amber_device_common.h"

namespace amber {
namespace {

constexpr uint32_t STAY = 4;                     // group of the offset (0, 0)
constexpr uint32_t TILE_LDS_BINS = 32768;        // initial sort: tiles counted in LDS
constexpr uint32_t SORT_PER = 8;                 // initial sort: agents per thread
constexpr uint32_t STEP_MAXA = 8;                // records a thread holds per round

__device__ __forceinline__ uint32_t tile_w(const TileParams &p, uint32_t i)
{
    return i + 1 == p.nT ? (uint32_t)p.L - (p.nT - 1) * p.T : p.T;
}

__device__ __forceinline__ uint32_t tile_of(const TileParams &p, int32_t v)
{
    const uint32_t i = (uint32_t)v >> p.tshift;
    return i < p.nT ? i : p.nT - 1;
}

// Ring of a w x h tile: the row above (w + 2 cells, corners included), the
// row below, then the column left and the column right (h cells each).
__device__ __forceinline__ uint32_t ring_size(uint32_t w, uint32_t h) { return 2 * (w + 2) + 2 * h; }

__device__ __forceinline__ void ring_cell(uint32_t r, uint32_t w, uint32_t h, int32_t &lx,
                                          int32_t &ly)
{
    const uint32_t row = w + 2;
    if (r < row) {
        lx = (int32_t)r - 1;
        ly = -1;
    } else if (r < 2 * row) {
        lx = (int32_t)(r - row) - 1;
        ly = (int32_t)h;
    } else if (r < 2 * row + h) {
        lx = -1;
        ly = (int32_t)(r - 2 * row);
    } else {
        lx = (int32_t)w;
        ly = (int32_t)(r - 2 * row - h);
    }
}

// Word j of a Philox block, by value selects (an indexed read would make the
// compiler keep the block in memory).
__device__ __forceinline__ uint32_t word_of(uint4 r, uint32_t j)
{
    const uint32_t odd = 0u - (j & 1u), high = 0u - ((j >> 1) & 1u);
    const uint32_t lo = (r.x & ~odd) | (r.y & odd);
    const uint32_t hi = (r.z & ~odd) | (r.w & odd);
    return (lo & ~high) | (hi & high);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Adds the active lanes of the wavefront to ctr[key] with one LDS atomic per
// distinct key and returns each lane's rank among the lanes of its key.
// Every lane of the wavefront must call it.
__device__ __forceinline__ uint32_t wave_add(uint32_t key, bool active, uint32_t *ctr)
{
    uint64_t pending = __ballot(active);
    uint32_t rank = 0;
    const uint32_t lane = __lane_id();
    while (pending) {
        const uint32_t leader = (uint32_t)__builtin_ctzll(pending);
        const uint32_t k = (uint32_t)__shfl((int)key, (int)leader);
        const uint64_t same = __ballot(active && key == k);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctr[k], (uint32_t)__popcll(same));
        base = (uint32_t)__shfl((int)base, (int)leader);
        if (active && key == k) rank = base + lanes_below(same);
        pending &= ~same;
    }
    return rank;
}

// Record v of the tile's input (chunk d holds virtual indices
// [pre[d], pre[d+1])).
__device__ __forceinline__ uint2 load_rec(const uint2 *__restrict__ rec, const uint32_t *start,
                                          const uint32_t *pre, uint32_t v)
{
    uint32_t d = 0;
#pragma unroll
    for (int k = 1; k < 9; ++k) d += v >= pre[k] ? 1u : 0u;
    return rec[start[d] + (v - pre[d])];
}

// Move of step t for agent id at local (lx, ly): returns the new local
// position (+1, 10 bits each) and the destination group (bits 20..23).
__device__ __forceinline__ uint32_t move_of(const TileParams &p, uint32_t id, uint32_t pk,
                                            uint32_t t, uint32_t w, uint32_t h)
{
    const uint32_t u = word_of(philox(id >> 2, t, P_MOVE, p.k0, p.k1), id & 3u);
    const uint32_t sh = (u >> 28) & 14u;
    const int32_t nx = (int32_t)(pk & 1023u) + (int32_t)((MOVE_DX1 >> sh) & 3u) - 1;
    const int32_t ny = (int32_t)((pk >> 10) & 1023u) + (int32_t)((MOVE_DY1 >> sh) & 3u) - 1;
    const uint32_t gx = nx < 0 ? 0u : (nx >= (int32_t)w ? 2u : 1u);
    const uint32_t gy = ny < 0 ? 0u : (ny >= (int32_t)h ? 2u : 1u);
    return (uint32_t)(nx + 1) | ((uint32_t)(ny + 1) << 10) | ((gy * 3 + gx) << 20);
}

// Transition of step t_prev for an agent at local (lx, ly) of the tile, with
// the previous step's counts of the tile and its ring in reg (row stride RW,
// cell (lx, ly) at (ly + 1) * RW + lx + 1).
template <uint32_t RW>
__device__ __forceinline__ uint32_t tile_transition(const TileParams &p, const uint32_t *reg,
                                                    uint32_t id, uint32_t s, uint32_t lx,
                                                    uint32_t ly, uint32_t t_prev)
{
    if (s == ST_R) return s;
    uint32_t k = 0;
    if (s == ST_S) {
        const uint32_t *c = reg + ly * RW + lx;
        k = c[0] + c[1] + c[2] + c[RW] + c[RW + 1] + c[RW + 2] + c[2 * RW] + c[2 * RW + 1] +
            c[2 * RW + 2];
        if (k == 0) return s;
    }
    const uint32_t u = word_of(philox(id >> 2, t_prev, P_EPI, p.k0, p.k1), id & 3u);
    if (s == ST_S) {
        const uint32_t kl = p.table_len - 1;
        return u < p.t_inf[k < kl ? k : kl] ? (uint32_t)ST_I : (uint32_t)ST_S;
    }
    return u < p.t_rec ? (uint32_t)ST_R : (uint32_t)ST_I;
}

// One step on one tile.  TRANS: apply the transition of step t - 1 first
// (not on the first launch of a call).  MOVE: move and bin step t and write
// the next records (not on the last launch, which writes the columns).
// Input generation gen, output generation gen ^ 1.
template <uint32_t T, bool TRANS, bool MOVE>
__global__ void __launch_bounds__(1024) k_tile_step(TileParams p, uint32_t t, uint32_t gen)
{
    constexpr uint32_t RW = T + 3;                 // widest tile (T + 1) plus its ring
    __shared__ uint32_t reg[TRANS ? RW * RW : 1];  // counts of step t - 1
    __shared__ uint32_t hist[MOVE ? RW * RW : 1];  // infected of step t
    __shared__ uint32_t c_start[9], c_cnt[9], c_pre[10], gcnt[9], gcur[9], goff[9];
    __shared__ uint32_t s_base;
    const uint32_t tid = threadIdx.x, NT = blockDim.x;
    const uint32_t tile = blockIdx.x;
    const uint32_t ti = tile % p.nT, tj = tile / p.nT;
    const int32_t x0 = (int32_t)(ti * T), y0 = (int32_t)(tj * T);
    const uint32_t w = tile_w(p, ti), h = tile_w(p, tj);

    if (tid < 9) {
        // chunk tid: what tile (ti - ddx, tj - ddy) sent with offset (ddx, ddy)
        const uint32_t si = (ti + p.nT + 1 - tid % 3) % p.nT;
        const uint32_t sj = (tj + p.nT + 1 - tid / 3) % p.nT;
        const uint32_t *H = p.hdr[gen] + (size_t)(sj * p.nT + si) * TILE_HDR;
        uint32_t off = H[0];
        for (uint32_t g = 0; g < tid; ++g) off += H[1 + g];
        c_start[tid] = off;
        c_cnt[tid] = H[1 + tid];
        gcnt[tid] = 0;
        gcur[tid] = 0;
    }
    if (MOVE)
        for (uint32_t k = tid; k < RW * RW; k += NT) hist[k] = 0;
    if (TRANS) {
        const uint32_t *C = p.C[gen ^ 1];
        const uint32_t rw = w + 2, cells = rw * (h + 2);
        for (uint32_t k = tid; k < cells; k += NT) {
            const uint32_t ry = k / rw, rx = k - ry * rw;
            int32_t gx = x0 + (int32_t)rx - 1, gy = y0 + (int32_t)ry - 1;
            gx = gx < 0 ? gx + p.L : (gx >= p.L ? gx - p.L : gx);
            gy = gy < 0 ? gy + p.L : (gy >= p.L ? gy - p.L : gy);
            reg[ry * RW + rx] = C[(size_t)gy * (uint32_t)p.L + (uint32_t)gx];
        }
    }
    __syncthreads();
    if (tid == 0) {
        // the chunks must lie inside the record buffer and sum to at most n;
        // if not, the tile takes no records and the error word says so
        uint32_t acc = 0;
        bool ok = true;
        for (int d = 0; d < 9; ++d) {
            c_pre[d] = acc;
            acc += c_cnt[d];
            ok = ok && c_cnt[d] <= p.n && c_start[d] <= p.n - c_cnt[d];
        }
        if (!ok || acc > p.n) {
            acc = 0;
            for (int d = 0; d < 9; ++d) c_pre[d] = 0;
            __hip_atomic_fetch_or(p.err, ERR_TILE_LISTS, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
        }
        c_pre[9] = acc;
    }
    if (TRANS) {
        // ring partial counts of the 9 tiles around (this one included)
        const uint32_t *R = p.ring[gen ^ 1];
        for (uint32_t k = tid; k < 9 * p.rs; k += NT) {
            const uint32_t a = k / p.rs, r = k - a * p.rs;
            const uint32_t ai = (ti + p.nT + a % 3 - 1) % p.nT;
            const uint32_t aj = (tj + p.nT + a / 3 - 1) % p.nT;
            const uint32_t aw = tile_w(p, ai), ah = tile_w(p, aj);
            if (r >= ring_size(aw, ah)) continue;
            const uint32_t v = R[(size_t)(aj * p.nT + ai) * p.rs + r];
            if (v == 0) continue;
            int32_t lx, ly;
            ring_cell(r, aw, ah, lx, ly);
            int32_t bx = (int32_t)(ai * T) + lx - x0, by = (int32_t)(aj * T) + ly - y0;
            if (bx < -1) bx += p.L;
            else if (bx > (int32_t)w) bx -= p.L;
            if (by < -1) by += p.L;
            else if (by > (int32_t)h) by -= p.L;
            if (bx >= -1 && bx <= (int32_t)w && by >= -1 && by <= (int32_t)h)
                atomicAdd(&reg[(uint32_t)(by + 1) * RW + (uint32_t)(bx + 1)], v);
        }
    }
    __syncthreads();
    const uint32_t n_in = c_pre[9];
    const uint2 *in = p.rec[gen];

    if (!MOVE) {
        // last launch of the call: transition, then back to the columns
        for (uint32_t v = tid; v < n_in; v += NT) {
            const uint2 r = load_rec(in, c_start, c_pre, v);
            const uint32_t lx = r.y & 1023u, ly = (r.y >> 10) & 1023u;
            uint32_t s = (r.y >> 20) & 3u;
            if (r.x >= p.n || lx >= w || ly >= h) {
                __hip_atomic_fetch_or(p.err, ERR_TILE_LISTS, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                continue;
            }
            if (TRANS) s = tile_transition<RW>(p, reg, r.x, s, lx, ly, t - 1);
            p.x[r.x] = x0 + (int32_t)lx;
            p.y[r.x] = y0 + (int32_t)ly;
            p.s[r.x] = (uint8_t)s;
        }
        return;
    }

    // pass 1: group sizes (records stay in registers when they fit one round)
    const uint32_t cap = NT * STEP_MAXA;
    uint32_t rid[STEP_MAXA], rpk[STEP_MAXA], rmv[STEP_MAXA];
    for (uint32_t r0 = 0; r0 < n_in; r0 += cap) {
#pragma unroll
        for (uint32_t j = 0; j < STEP_MAXA; ++j) {
            const uint32_t v = r0 + tid + j * NT;
            const bool act = v < n_in;
            uint32_t g = STAY;
            if (act) {
                const uint2 r = load_rec(in, c_start, c_pre, v);
                rid[j] = r.x;
                rpk[j] = r.y;
                rmv[j] = move_of(p, r.x, r.y, t, w, h);
                g = rmv[j] >> 20;
                if ((r.y & 1023u) >= w || ((r.y >> 10) & 1023u) >= h)
                    __hip_atomic_fetch_or(p.err, ERR_TILE_LISTS, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
            }
            wave_add(g, act, gcnt);
        }
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (int g = 0; g < 9; ++g) {
            goff[g] = acc;
            acc += gcnt[g];
        }
        uint32_t base = atomicAdd(p.ctr + 64 * (gen ^ 1), n_in);
        if (base > p.n - n_in) {       // more records than agents: write none
            __hip_atomic_fetch_or(p.err, ERR_TILE_LISTS, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            base = 0xffffffffu;
        }
        s_base = base;
        uint32_t *H = p.hdr[gen ^ 1] + (size_t)tile * TILE_HDR;
        H[0] = base;
        for (int g = 0; g < 9; ++g) H[1 + g] = gcnt[g];
        if (tile == 0) p.ctr[64 * gen] = 0;     // allocator of the next launch's output
    }
    __syncthreads();

    // pass 2: transition, bin, write
    const bool one = n_in <= cap;
    const uint32_t base = s_base;
    const bool store = base != 0xffffffffu;
    uint2 *out = p.rec[gen ^ 1];
    const uint32_t wl = tile_w(p, (ti + p.nT - 1) % p.nT);   // width of the tile to the left
    const uint32_t hb = tile_w(p, (tj + p.nT - 1) % p.nT);   // height of the tile above
    for (uint32_t r0 = 0; r0 < n_in; r0 += cap) {
#pragma unroll
        for (uint32_t j = 0; j < STEP_MAXA; ++j) {
            const uint32_t v = r0 + tid + j * NT;
            const bool act = v < n_in;
            uint32_t g = STAY, pk = 0;
            if (act) {
                if (!one) {
                    const uint2 r = load_rec(in, c_start, c_pre, v);
                    rid[j] = r.x;
                    rpk[j] = r.y;
                    rmv[j] = move_of(p, r.x, r.y, t, w, h);
                }
                uint32_t s = (rpk[j] >> 20) & 3u;
                if (TRANS)
                    s = tile_transition<RW>(p, reg, rid[j], s, rpk[j] & 1023u,
                                            (rpk[j] >> 10) & 1023u, t - 1);
                const uint32_t m = rmv[j];
                const uint32_t cx = m & 1023u, cy = (m >> 10) & 1023u;   // new local + 1
                g = m >> 20;
                if (s == ST_I && cx <= w + 1 && cy <= h + 1) atomicAdd(&hist[cy * RW + cx], 1u);
                const uint32_t gx = g % 3, gy = g / 3;
                const uint32_t dx = gx == 0 ? wl - 1 : (gx == 2 ? 0u : cx - 1);
                const uint32_t dy = gy == 0 ? hb - 1 : (gy == 2 ? 0u : cy - 1);
                pk = dx | (dy << 10) | (s << 20);
            }
            const uint32_t rank = wave_add(g, act, gcur);
            if (act && store) out[base + goff[g] + rank] = make_uint2(rid[j], pk);
        }
    }
    __syncthreads();

    // counts of step t: interior to the grid, ring to the tile's ring array
    uint32_t *C = p.C[gen];
    for (uint32_t k = tid; k < w * h; k += NT) {
        const uint32_t ly = k / w, lx = k - ly * w;
        C[(size_t)((uint32_t)y0 + ly) * (uint32_t)p.L + (uint32_t)x0 + lx] =
            hist[(ly + 1) * RW + lx + 1];
    }
    uint32_t *R = p.ring[gen] + (size_t)tile * p.rs;
    const uint32_t rsz = ring_size(w, h);
    for (uint32_t r = tid; r < rsz; r += NT) {
        int32_t lx, ly;
        ring_cell(r, w, h, lx, ly);
        R[r] = hist[(uint32_t)(ly + 1) * RW + (uint32_t)(lx + 1)];
    }
}

// ------------------------------------------------------------------ initial sort
// Counting sort of the columns into generation 0: agents per tile, an
// exclusive scan into record ranges, then the scatter.  With at most
// TILE_LDS_BINS tiles a workgroup counts its agents in LDS first and takes
// one global atomic per tile it touches.

__device__ __forceinline__ uint32_t agent_tile(const TileParams &p, uint32_t a)
{
    return tile_of(p, p.y[a]) * p.nT + tile_of(p, p.x[a]);
}

template <bool LDS>
__global__ void __launch_bounds__(1024) k_tile_hist(TileParams p)
{
    __shared__ uint32_t h[LDS ? TILE_LDS_BINS : 1];
    const uint32_t tid = threadIdx.x, NT = blockDim.x, nt = p.nT * p.nT;
    const uint32_t a0 = blockIdx.x * NT * SORT_PER;
    if (LDS) {
        for (uint32_t b = tid; b < nt; b += NT) h[b] = 0;
        __syncthreads();
    }
    for (uint32_t j = 0; j < SORT_PER; ++j) {
        const uint32_t a = a0 + j * NT + tid;
        if (a >= p.n) break;
        const uint32_t b = agent_tile(p, a);
        if (LDS) atomicAdd(&h[b], 1u);
        else atomicAdd(&p.cursor[b], 1u);
    }
    if (LDS) {
        __syncthreads();
        for (uint32_t b = tid; b < nt; b += NT)
            if (h[b]) atomicAdd(&p.cursor[b], h[b]);
    }
}

// One workgroup: cursor[] (counts) -> record bases, generation-0 headers.
__global__ void __launch_bounds__(1024) k_tile_scan(TileParams p)
{
    __shared__ uint32_t part[1024];
    __shared__ uint32_t carry;
    const uint32_t tid = threadIdx.x, nt = p.nT * p.nT;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (uint32_t c0 = 0; c0 < nt; c0 += 4 * 1024) {
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = c0 + tid * 4 + j;
            v[j] = i < nt ? p.cursor[i] : 0u;
            sum += v[j];
        }
        part[tid] = sum;
        __syncthreads();
        for (uint32_t off = 1; off < 1024; off <<= 1) {
            const uint32_t add = tid >= off ? part[tid - off] : 0u;
            __syncthreads();
            part[tid] += add;
            __syncthreads();
        }
        uint32_t b = carry + part[tid] - sum;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = c0 + tid * 4 + j;
            if (i < nt) {
                uint32_t *H = p.hdr[0] + (size_t)i * TILE_HDR;
                H[0] = b;
                for (uint32_t g = 0; g < 9; ++g) H[1 + g] = g == STAY ? v[j] : 0u;
                p.cursor[i] = b;
            }
            b += v[j];
        }
        __syncthreads();
        if (tid == 1023) carry += part[1023];
        __syncthreads();
    }
    if (tid == 0) {
        p.ctr[0] = 0;
        p.ctr[64] = 0;
    }
}

template <bool LDS>
__global__ void __launch_bounds__(1024) k_tile_scatter(TileParams p)
{
    __shared__ uint32_t h[LDS ? TILE_LDS_BINS : 1];
    const uint32_t tid = threadIdx.x, NT = blockDim.x, nt = p.nT * p.nT;
    const uint32_t a0 = blockIdx.x * NT * SORT_PER;
    uint32_t bin[SORT_PER], rank[SORT_PER];
    if (LDS) {
        for (uint32_t b = tid; b < nt; b += NT) h[b] = 0;
        __syncthreads();
#pragma unroll
        for (uint32_t j = 0; j < SORT_PER; ++j) {
            const uint32_t a = a0 + j * NT + tid;
            if (a < p.n) {
                bin[j] = agent_tile(p, a);
                rank[j] = atomicAdd(&h[bin[j]], 1u);
            }
        }
        __syncthreads();
        for (uint32_t b = tid; b < nt; b += NT)
            if (h[b]) h[b] = atomicAdd(&p.cursor[b], h[b]);   // count -> first slot
        __syncthreads();
    }
#pragma unroll
    for (uint32_t j = 0; j < SORT_PER; ++j) {
        const uint32_t a = a0 + j * NT + tid;
        if (a >= p.n) continue;
        const int32_t x = p.x[a], y = p.y[a];
        const uint32_t tx = tile_of(p, x), ty = tile_of(p, y);
        const uint32_t slot = LDS ? h[bin[j]] + rank[j] : atomicAdd(&p.cursor[ty * p.nT + tx], 1u);
        const uint32_t lx = (uint32_t)x - tx * p.T, ly = (uint32_t)y - ty * p.T;
        p.rec[0][slot] = make_uint2(a, lx | (ly << 10) | ((uint32_t)p.s[a] << 20));
    }
}

template <uint32_t T>
hipError_t step_launch(const TileParams &p, uint32_t t, uint32_t gen, uint32_t phase,
                       uint32_t block, hipStream_t st)
{
    const dim3 grid(p.nT * p.nT), thr(block);
    if (phase == 0) hipLaunchKernelGGL((k_tile_step<T, false, true>), grid, thr, 0, st, p, t, gen);
    else if (phase == 1) hipLaunchKernelGGL((k_tile_step<T, true, true>), grid, thr, 0, st, p, t, gen);
    else hipLaunchKernelGGL((k_tile_step<T, true, false>), grid, thr, 0, st, p, t, gen);
    return hipGetLastError();
}

}  // namespace

uint32_t sir_tile_count(uint32_t L, uint32_t T)
{
    return L >= 2 * T + 2 ? (L - 2) / T + 1 : 0u;
}

uint64_t sir_tile_ring_words(uint32_t L)
{
    const uint64_t nt = sir_tile_count(L, TILE_MIN);
    return nt * nt * (4ull * TILE_MIN + 8);
}

hipError_t launch_sir_tile_sort(const TileParams &p, hipStream_t st)
{
    const uint32_t nt = p.nT * p.nT;
    hipError_t e = launch_zero_words(p.cursor, (nt + 3u) & ~3u, st);
    if (e != hipSuccess) return e;
    const uint32_t per_block = 1024 * SORT_PER;
    const dim3 grid((p.n + per_block - 1) / per_block), thr(1024);
    if (nt <= TILE_LDS_BINS) hipLaunchKernelGGL(k_tile_hist<true>, grid, thr, 0, st, p);
    else hipLaunchKernelGGL(k_tile_hist<false>, grid, thr, 0, st, p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (nt <= TILE_LDS_BINS) hipLaunchKernelGGL(k_tile_scatter<true>, grid, thr, 0, st, p);
    else hipLaunchKernelGGL(k_tile_scatter<false>, grid, thr, 0, st, p);
    return hipGetLastError();
}

hipError_t launch_sir_tile_step(const TileParams &p, uint32_t t0, uint32_t i, uint32_t n,
                                uint32_t block, hipStream_t st)
{
    const uint32_t phase = i == 0 ? 0u : (i == n ? 2u : 1u);
    if (p.T == 32) return step_launch<32>(p, t0 + i, i & 1u, phase, block, st);
    if (p.T == 64) return step_launch<64>(p, t0 + i, i & 1u, phase, block, st);
    return hipErrorInvalidValue;
}

}  // namespace amber
