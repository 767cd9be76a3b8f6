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
//     A tile's list holds its own stayers first, so the input's first
//     entries are its stay chunk and the chunk search is for the few
//     records that moved in.
//  2. Infected counts of the previous step on the tile and the one-cell ring
//     around it go to LDS: inside the tile, the infected records of its own
//     input (a record holds its position after the previous move and its
//     state at the start of that step); on the ring, the border cells that
//     each tile stores from its grid plus the ring partial counts of the 9
//     tiles around (each tile stores the infected agents it moved onto the
//     ring around it).
//  3. Per agent: the transition of the previous step from the 3 x 3 sum in
//     LDS, then the move of this step.  Infected agents are binned into an
//     LDS histogram of the tile and its ring, and the record goes to the
//     group of its destination tile inside the tile's output range (one
//     atomic per tile allocates that range).
//  4. The histogram's border cells are stored to the count grid and its ring
//     to the tile's ring array, every cell, so nothing is cleared during a
//     call.
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
// compiler keep the block in memory): three bitwise selects m ? a : b, each
// one v_bitop3_b32 (truth table 0xE4 for operands a, b, m), on the all-ones
// or zero masks of bits 0 and 1 of j.
__device__ __forceinline__ uint32_t word_of(uint4 r, uint32_t j)
{
    const uint32_t odd = (uint32_t)((int32_t)(j << 31) >> 31);
    const uint32_t high = (uint32_t)((int32_t)(j << 30) >> 31);
    const uint32_t lo = __builtin_amdgcn_bitop3_b32(r.y, r.x, odd, 0xE4);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32(r.w, r.z, odd, 0xE4);
    return __builtin_amdgcn_bitop3_b32(hi, lo, high, 0xE4);
}

// A tile's record list holds its nine groups in the order STAY, 0, 1, 2, 3,
// 5, 6, 7, 8 (group_rank gives a group's place, group_at the group in a
// place): the records that stayed come first, so an input entry below the
// stay count needs no chunk search.
__device__ __forceinline__ uint32_t group_rank(uint32_t g)
{
    return g == STAY ? 0u : (g < STAY ? g + 1 : g);
}
__device__ __forceinline__ uint32_t group_at(uint32_t k)
{
    return k == 0 ? STAY : (k <= STAY ? k - 1 : k);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Slot of index u of a tile's record list (slots [fix, fix + cap), then the
// overflow range at ovf).
__device__ __forceinline__ uint32_t rec_slot(uint32_t u, uint32_t cap, uint32_t fix, uint32_t ovf)
{
    return u < cap ? fix + u : ovf + (u - cap);
}

// Move of step t for agent id at local (lx, ly): returns the new local
// position (+1, 10 bits each), the destination group (bits 20..23) and its
// tile offsets + 1 in x (bits 24..25) and y (bits 26..27).
__device__ __forceinline__ uint32_t move_of(const TileParams &p, uint32_t id, uint32_t pk,
                                            uint32_t t, uint32_t w, uint32_t h)
{
    const uint32_t u = word_of(philox(id >> 2, t, P_MOVE, p.k0, p.k1), id & 3u);
    const uint32_t sh = (u >> 28) & 14u;
    const int32_t nx = (int32_t)(pk & 1023u) + (int32_t)((MOVE_DX1 >> sh) & 3u) - 1;
    const int32_t ny = (int32_t)((pk >> 10) & 1023u) + (int32_t)((MOVE_DY1 >> sh) & 3u) - 1;
    const uint32_t gx = nx < 0 ? 0u : (nx >= (int32_t)w ? 2u : 1u);
    const uint32_t gy = ny < 0 ? 0u : (ny >= (int32_t)h ? 2u : 1u);
    return (uint32_t)(nx + 1) | ((uint32_t)(ny + 1) << 10) | ((gy * 3 + gx) << 20) | (gx << 24) |
           (gy << 26);
}

// Transition of step t_prev for an agent at local (lx, ly) of the tile, with
// the previous step's counts of the tile and its ring in reg (row stride RW,
// cell (lx, ly) at (ly + 1) * RW + lx + 1).
// The first TINF_LDS thresholds are read from an LDS copy (tinf), the rest
// from the table in memory.
constexpr uint32_t TINF_LDS = 64;
template <uint32_t RW>
__device__ __forceinline__ uint32_t tile_transition(const TileParams &p, const uint32_t *reg,
                                                    const uint32_t *tinf, uint32_t id, uint32_t s,
                                                    uint32_t lx, uint32_t ly, uint32_t t_prev)
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
        const uint32_t kl = p.table_len - 1, kk = k < kl ? k : kl;
        // an LDS read, and a global one only past the copy (volatile, so that
        // the two are not merged into one flat load through a chosen pointer,
        // which waits on both)
        uint32_t thr = tinf[kk < TINF_LDS ? kk : 0u];
        if (kk >= TINF_LDS) thr = *(const volatile uint32_t *)(p.t_inf + kk);
        return u < thr ? (uint32_t)ST_I : (uint32_t)ST_S;
    }
    return u < p.t_rec ? (uint32_t)ST_R : (uint32_t)ST_I;
}

// Buffers of one launch: input generation gen, output generation gen ^ 1;
// counts are read from the previous launch and written for the next.
struct StepIO {
    const uint2 *rec_in;
    uint2 *rec_out;
    const uint32_t *hdr_in;
    uint32_t *hdr_out;
    const uint32_t *C_in;
    uint32_t *C_out;
    const uint32_t *ring_in;
    uint32_t *ring_out;
    uint32_t *ovf_out;         // overflow allocator of the output generation
    uint32_t *ovf_reset;       // allocator the previous launch used: back to zero
};

// Ring entry k of the 9-tile neighbourhood: the ring word it reads and the
// region entry (row stride RW) it adds to, for the tile (ti, tj) of size
// w x h.  Only words that count cells on the tile's ring are listed (the
// cells inside the tile are counted from its own input records): the tile's
// own ring (2(w+2) + 2h words), then 24 single words of the 8 neighbours'
// rings, each a ring cell next to one of the tile's corners.
struct RingSeg {
    const uint32_t *src;
    uint32_t dst;
};

template <uint32_t RW>
__device__ __forceinline__ RingSeg ring_entry(const uint32_t *R, uint32_t rs, uint32_t nT,
                                              uint32_t k, uint32_t ti, uint32_t tj, uint32_t li,
                                              uint32_t ri, uint32_t uj, uint32_t dj, uint32_t w,
                                              uint32_t h, uint32_t wl, uint32_t wr, uint32_t hu,
                                              uint32_t hd)
{
    auto ring = [&](uint32_t i, uint32_t j) { return R + (size_t)(j * nT + i) * rs; };
    const uint32_t n_self = 2 * (w + 2) + 2 * h;
    if (k < n_self) {
        int32_t lx, ly;
        ring_cell(k, w, h, lx, ly);
        return {ring(ti, tj) + k, (uint32_t)(ly + 1) * RW + (uint32_t)(lx + 1)};
    }
    const uint32_t b = (h + 1) * RW;        // bottom ring row
    switch (k - n_self) {
    // the tile above: the two ends of the row below it; the tile below: of
    // the row above it
    case 0: return {ring(ti, uj) + w + 2, RW};
    case 1: return {ring(ti, uj) + 2 * w + 3, RW + w + 1};
    case 2: return {ring(ti, dj), h * RW};
    case 3: return {ring(ti, dj) + w + 1, h * RW + w + 1};
    // the tiles left and right: the cells of their top and bottom ring rows
    // next to the tile
    case 4: return {ring(li, tj) + wl, 0};
    case 5: return {ring(li, tj) + wl + 1, 1};
    case 6: return {ring(li, tj) + wl + 2 + wl, b};
    case 7: return {ring(li, tj) + wl + 2 + wl + 1, b + 1};
    case 8: return {ring(ri, tj), w};
    case 9: return {ring(ri, tj) + 1, w + 1};
    case 10: return {ring(ri, tj) + wr + 2, b + w};
    case 11: return {ring(ri, tj) + wr + 3, b + w + 1};
    // the tiles above and below: the cells of their side ring columns next
    // to the tile
    case 12: return {ring(ti, uj) + 2 * (w + 2) + hu - 1, 0};
    case 13: return {ring(ti, uj) + 2 * (w + 2) + 2 * hu - 1, w + 1};
    case 14: return {ring(ti, dj) + 2 * (w + 2), b};
    case 15: return {ring(ti, dj) + 2 * (w + 2) + hd, b + w + 1};
    // the four diagonal tiles: their ring cells on this tile's ring
    case 16: return {ring(li, uj) + wl + 2 + wl, RW};
    case 17: return {ring(li, uj) + 2 * (wl + 2) + 2 * hu - 1, 1};
    case 18: return {ring(ri, uj) + wr + 3, RW + w + 1};
    case 19: return {ring(ri, uj) + 2 * (wr + 2) + hu - 1, w};
    case 20: return {ring(li, dj) + wl, h * RW};
    case 21: return {ring(li, dj) + 2 * (wl + 2) + hd, b + 1};
    case 22: return {ring(ri, dj) + 1, h * RW + w + 1};
    default: return {ring(ri, dj) + 2 * (wr + 2), b + w};
    }
}

// One step on one tile.  TRANS: apply the transition of step t - 1 first
// (not on the first launch of a call).  MOVE: move and bin step t and write
// the next records (not on the last launch, which writes the columns).
// Input generation gen, output generation gen ^ 1.
//
// Output slots: every wavefront counts its records per destination group
// (pass 1); the counts become per-wavefront bases inside each group, and
// pass 2 hands out consecutive slots from those bases: ballot ranks for the
// records that stay, LDS atomics for the few that leave.
// Global loads of one phase are all issued before any of them is used.
template <uint32_t T, bool TRANS, bool MOVE>
__global__ void __launch_bounds__(1024) k_tile_step(TileParams p, StepIO io, uint32_t t)
{
    constexpr uint32_t RW = T + 3;                 // widest tile (T + 1) plus its ring
    constexpr uint32_t MAXW = 16;                  // wavefronts per workgroup
    __shared__ uint32_t reg[TRANS ? RW * RW : 1];  // counts of step t - 1
    __shared__ uint32_t hist[MOVE ? RW * RW : 1];  // infected of step t
    __shared__ uint32_t wcnt[MOVE ? MAXW * 9 : 1]; // per-wavefront group counts
    __shared__ uint32_t wbase[MOVE ? MAXW * 9 : 1];// per-wavefront group bases
    __shared__ uint32_t c_start[9], c_fix[9], c_ovf[9], c_cnt[9], gtot[9];
    __shared__ uint32_t s_ovf, s_store, s_sus;
    __shared__ uint32_t tinf[TRANS ? TINF_LDS : 1];   // first thresholds of the table
    const uint32_t tid = threadIdx.x, NT = blockDim.x;
    const uint32_t lane = tid & 63u, nw = NT >> 6;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wavefront-uniform
    const uint32_t nT = p.nT, tile = xcd_partition(blockIdx.x, gridDim.x);
    const uint32_t tj = tile / nT, ti = tile - tj * nT;
    const uint32_t last = (uint32_t)p.L - (nT - 1) * T;
    const uint32_t li = ti ? ti - 1 : nT - 1, ri = ti + 1 < nT ? ti + 1 : 0u;
    const uint32_t uj = tj ? tj - 1 : nT - 1, dj = tj + 1 < nT ? tj + 1 : 0u;
    const uint32_t w = ti + 1 == nT ? last : T, h = tj + 1 == nT ? last : T;
    const int32_t x0 = (int32_t)(ti * T), y0 = (int32_t)(tj * T);

    if (tid < 9) {
        // chunk tid: what tile (ti - ddx, tj - ddy) sent with offset
        // (ddx, ddy) = (tid % 3 - 1, tid / 3 - 1): its group tid
        const uint32_t cx = tid % 3, cy = tid / 3;
        const uint32_t si = cx == 0 ? ri : (cx == 1 ? ti : li);
        const uint32_t sj = cy == 0 ? dj : (cy == 1 ? tj : uj);
        const uint32_t src = sj * nT + si;
        const uint32_t *H = io.hdr_in + (size_t)src * TILE_HDR;
        uint32_t hv[TILE_HDR];
#pragma unroll
        for (uint32_t i = 0; i < TILE_HDR; ++i) hv[i] = H[i];
        uint32_t off = 0, cnt = 0;
#pragma unroll
        for (uint32_t g = 0; g < 9; ++g) {
            off += group_rank(g) < group_rank(tid) ? hv[1 + g] : 0u;
            cnt = g == tid ? hv[1 + g] : cnt;
        }
        c_start[tid] = off;
        c_fix[tid] = src * p.cap;
        c_ovf[tid] = hv[0];
        c_cnt[tid] = cnt;
    }
    if (MOVE) {
        for (uint32_t k = tid; k < RW * RW; k += NT) hist[k] = 0;
        for (uint32_t k = tid; k < nw * 9; k += NT) wcnt[k] = 0;
        if (tid < 9) gtot[tid] = 0;
    }
    if (TRANS && tid < TINF_LDS && tid < p.table_len) tinf[tid] = p.t_inf[tid];
    // Counts of the previous step.  Inside the tile they are the infected
    // records of the tile's own input (each record carries its position and
    // its state at the start of that step, which is what was binned), counted
    // in LDS during the first pass.  On the ring around the tile they come
    // from memory: the border cells of the neighbouring tiles' grids plus the
    // ring partial counts of the 9 tiles that land there (ring_entry).
    // Neither depends on the headers:
    // those loads go out together with the header loads, the ring cells into
    // LDS before the barrier, the first RING_PRE partial words of each thread
    // into registers (added after the first pass).
    constexpr uint32_t RING_PRE = 4;
    uint32_t ring_v[RING_PRE], ring_dst[RING_PRE];
    const uint32_t wl = li + 1 == nT ? last : T, wr = ri + 1 == nT ? last : T;
    const uint32_t hu = uj + 1 == nT ? last : T, hd = dj + 1 == nT ? last : T;
    const uint32_t ring_total = 2 * (w + 2) + 2 * h + 24;
    if (TRANS) {
#pragma unroll
        for (uint32_t i = 0; i < RING_PRE; ++i) {
            const uint32_t k = tid + i * NT;
            ring_v[i] = 0;
            ring_dst[i] = 0;
            if (k < ring_total) {
                const RingSeg e = ring_entry<RW>(io.ring_in, p.rs, nT, k, ti, tj, li, ri, uj,
                                                 dj, w, h, wl, wr, hu, hd);
                ring_v[i] = *e.src;
                ring_dst[i] = e.dst;
            }
        }
        const uint32_t *C = io.C_in;
        const uint32_t rsz = ring_size(w, h);
        for (uint32_t r = tid; r < rsz; r += NT) {
            int32_t lx, ly;
            ring_cell(r, w, h, lx, ly);
            int32_t gx = x0 + lx, gy = y0 + ly;
            gx = gx < 0 ? gx + p.L : (gx >= p.L ? gx - p.L : gx);
            gy = gy < 0 ? gy + p.L : (gy >= p.L ? gy - p.L : gy);
            reg[(uint32_t)(ly + 1) * RW + (uint32_t)(lx + 1)] = C[(size_t)gy * (uint32_t)p.L + gx];
        }
        for (uint32_t ry = wave; ry < h; ry += nw)
            for (uint32_t rx = lane; rx < w; rx += 64) reg[(ry + 1) * RW + rx + 1] = 0;
    }
    __syncthreads();

    // chunk prefix (every thread) and its check: the chunks must lie inside
    // the record buffer and sum to at most n, else the tile takes no records
    uint32_t pre[10];
    bool ok = true;
    pre[0] = 0;
#pragma unroll
    for (uint32_t k = 0; k < 9; ++k) {           // entry order: the chunks in group order
        const uint32_t d = group_at(k);
        const uint32_t c = c_cnt[d], st = c_start[d];
        pre[k + 1] = pre[k] + c;
        ok = ok && c <= p.n && st <= p.n - c;
        if (ok && c && st + c > p.cap)     // the chunk reaches the overflow range
            ok = c_ovf[d] >= p.ovf0 && c_ovf[d] - p.ovf0 <= p.n - (st + c - p.cap);
    }
    ok = ok && pre[9] <= p.n;
    const uint32_t n_in = ok ? pre[9] : 0u;
    if (!ok && tid == 0)
        __hip_atomic_fetch_or(p.err, ERR_TILE_LISTS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint2 *in = io.rec_in;
    // slot of entry v of the tile's input (the 9 chunks one after another,
    // in list order: the stay chunk first)
    auto slot_of = [&](uint32_t v) {
        uint32_t d = STAY, pd = 0;
        if (v >= pre[1]) {                          // a record that moved in (few)
#pragma unroll
            for (uint32_t k = 1; k < 9; ++k)
                if (v >= pre[k]) {
                    d = group_at(k);
                    pd = pre[k];
                }
        }
        return rec_slot(c_start[d] + (v - pd), p.cap, c_fix[d], c_ovf[d]);
    };

    if (MOVE && tid == 0) {
        // records beyond the tile's slots go to an overflow range (rare; one
        // atomic per overflowing tile)
        const uint32_t over = n_in > p.cap ? n_in - p.cap : 0u;
        uint32_t ovf = 0, store = 1;
        if (over) {
            const uint32_t b = atomicAdd(io.ovf_out, over);
            if (b > p.n - over) {    // more records than agents: write none
                __hip_atomic_fetch_or(p.err, ERR_TILE_LISTS, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                store = 0;
            }
            ovf = p.ovf0 + b;
        }
        s_ovf = ovf;
        s_store = store;
        if (tile == 0) *io.ovf_reset = 0;      // overflow allocator of the next launch
    }

    const uint32_t round_cap = NT * STEP_MAXA;
    const bool one = n_in <= round_cap;
    uint32_t rid[STEP_MAXA], rpk[STEP_MAXA], rmv[STEP_MAXA];
    // Every slot first, then every load, unconditionally (an entry past the
    // input reads slot 0 and is never used): the round's loads are then in
    // flight together.  Loads under a branch each waited for all earlier
    // ones.
    auto fetch = [&](uint32_t r0) {
        uint32_t slot[STEP_MAXA];
#pragma unroll
        for (uint32_t j = 0; j < STEP_MAXA; ++j) {
            const uint32_t v = r0 + j * NT + tid;
            slot[j] = v < n_in ? slot_of(v) : 0u;
        }
#pragma unroll
        for (uint32_t j = 0; j < STEP_MAXA; ++j) {
            const uint2 r = in[slot[j]];
            rid[j] = r.x;
            rpk[j] = r.y;
        }
    };

    // an input record infected at the start of the previous step adds one to
    // its cell of the previous step's counts (positions outside the tile are
    // a corrupt list, flagged in the first pass, and not counted)
    auto count_in = [&](uint32_t pk) {
        const uint32_t lx = pk & 1023u, ly = (pk >> 10) & 1023u;
        if (((pk >> 20) & 3u) == ST_I && lx < w && ly < h)
            atomicAdd(&reg[(ly + 1) * RW + lx + 1], 1u);
    };

    if (MOVE) {
        // pass 1: records per destination group and wavefront
        uint32_t *mine = wcnt + wave * 9;
        uint32_t stay = 0;                          // wavefront-uniform
        for (uint32_t r0 = 0; r0 < n_in; r0 += round_cap) {
            fetch(r0);
#pragma unroll
            for (uint32_t j = 0; j < STEP_MAXA; ++j) {
                if (r0 + j * NT + wave * 64 >= n_in) break;     // whole wavefront past the end
                const bool act = r0 + j * NT + tid < n_in;
                uint32_t g = STAY;
                if (act) {
                    rmv[j] = move_of(p, rid[j], rpk[j], t, w, h);
                    g = (rmv[j] >> 20) & 15u;
                    if ((rpk[j] & 1023u) >= w || ((rpk[j] >> 10) & 1023u) >= h)
                        __hip_atomic_fetch_or(p.err, ERR_TILE_LISTS, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                }
                stay += (uint32_t)__popcll(__ballot(act && g == STAY));
                // the few records that leave the tile: one LDS add each, to the
                // wavefront's count and to the group's total
                if (act && g != STAY) {
                    atomicAdd(&mine[g], 1u);
                    atomicAdd(&gtot[g], 1u);
                }
                if (TRANS && act) count_in(rpk[j]);
            }
        }
        if (lane == 0) {
            mine[STAY] = stay;
            atomicAdd(&gtot[STAY], stay);
        }
    } else {
        // the tail counts every round's infected records, then holds the
        // first round while the ring counts come in
        for (uint32_t r0 = 0; r0 < n_in; r0 += round_cap) {
            fetch(r0);
#pragma unroll
            for (uint32_t j = 0; j < STEP_MAXA; ++j)
                if (r0 + j * NT + tid < n_in) count_in(rpk[j]);
        }
        if (!one) fetch(0);
    }
    __syncthreads();

    if (TRANS) {
        // ring partial counts: the words loaded before the first barrier,
        // then any beyond them
#pragma unroll
        for (uint32_t i = 0; i < RING_PRE; ++i)
            if (ring_v[i]) atomicAdd(&reg[ring_dst[i]], ring_v[i]);
        for (uint32_t k = tid + RING_PRE * NT; k < ring_total; k += NT) {
            const RingSeg e = ring_entry<RW>(io.ring_in, p.rs, nT, k, ti, tj, li, ri, uj,
                                             dj, w, h, wl, wr, hu, hd);
            const uint32_t v = *e.src;
            if (v) atomicAdd(&reg[e.dst], v);
        }
    }
    if (MOVE) {
        // per-wavefront bases inside each group of the tile's list, and the
        // tile's header
        if (tid < nw * 9) {
            const uint32_t k = tid / 9, g = tid - k * 9;
            uint32_t b = 0;
            for (uint32_t q = 0; q < 9; ++q) b += group_rank(q) < group_rank(g) ? gtot[q] : 0u;
            for (uint32_t q = 0; q < k; ++q) b += wcnt[q * 9 + g];
            wbase[tid] = b;
        }
        if (tid == 0) {
            uint32_t *H = io.hdr_out + (size_t)tile * TILE_HDR;
            H[0] = s_ovf;
            for (int g = 0; g < 9; ++g) H[1 + g] = gtot[g];
            s_sus = 0;
        }
    }
    __syncthreads();

    if (!MOVE) {
        // last launch of the call: transition, then one 8-byte word per agent,
        // {x | y << 16, state}, into the free record generation at the agent's
        // id; k_tile_unpack then splits it into the columns with streaming
        // stores (three scattered stores per agent would each cost a partial
        // memory line)
        uint2 *const packed = io.rec_out;
        for (uint32_t r0 = 0; r0 < n_in; r0 += round_cap) {
            if (r0) fetch(r0);
#pragma unroll
            for (uint32_t j = 0; j < STEP_MAXA; ++j) {
                const uint32_t v = r0 + j * NT + tid;
                if (v >= n_in) break;
                const uint32_t lx = rpk[j] & 1023u, ly = (rpk[j] >> 10) & 1023u;
                if (rid[j] >= p.n || lx >= w || ly >= h) {
                    __hip_atomic_fetch_or(p.err, ERR_TILE_LISTS, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                    continue;
                }
                uint32_t s = (rpk[j] >> 20) & 3u;
                if (TRANS) s = tile_transition<RW>(p, reg, tinf, rid[j], s, lx, ly, t - 1);
                packed[rid[j]] = make_uint2((uint32_t)(x0 + (int32_t)lx) |
                                                ((uint32_t)(y0 + (int32_t)ly) << 16),
                                            s);
            }
        }
        return;
    }

    // pass 2: transition, bin, write
    const bool store = s_store != 0;
    const uint32_t fix = tile * p.cap, ovf = s_ovf;
    uint2 *out = io.rec_out;
    const uint32_t hb = hu;                         // height of the tile above
    uint32_t *mine = wbase + wave * 9;
    uint32_t stay_run = mine[STAY];
    uint32_t wsus = 0;                              // susceptible records of this wavefront
    for (uint32_t r0 = 0; r0 < n_in; r0 += round_cap) {
        if (!one) {
            fetch(r0);
#pragma unroll
            for (uint32_t j = 0; j < STEP_MAXA; ++j)
                if (r0 + j * NT + tid < n_in) rmv[j] = move_of(p, rid[j], rpk[j], t, w, h);
        }
#pragma unroll
        for (uint32_t j = 0; j < STEP_MAXA; ++j) {
            if (r0 + j * NT + wave * 64 >= n_in) break;
            const bool act = r0 + j * NT + tid < n_in;
            uint32_t g = STAY, pk = 0;
            bool sus = false;
            if (act) {
                uint32_t s = (rpk[j] >> 20) & 3u;
                if (TRANS)
                    s = tile_transition<RW>(p, reg, tinf, rid[j], s, rpk[j] & 1023u,
                                            (rpk[j] >> 10) & 1023u, t - 1);
                sus = s == ST_S;
                const uint32_t m = rmv[j];
                const uint32_t cx = m & 1023u, cy = (m >> 10) & 1023u;   // new local + 1
                g = (m >> 20) & 15u;
                if (s == ST_I && cx <= w + 1 && cy <= h + 1) atomicAdd(&hist[cy * RW + cx], 1u);
                const uint32_t gx = (m >> 24) & 3u, gy = (m >> 26) & 3u;
                const uint32_t dx = gx == 0 ? wl - 1 : (gx == 2 ? 0u : cx - 1);
                const uint32_t dy = gy == 0 ? hb - 1 : (gy == 2 ? 0u : cy - 1);
                pk = dx | (dy << 10) | (s << 20);
            }
            uint32_t slot = 0;
            const uint64_t ms = __ballot(act && g == STAY);
            if (act && g == STAY) slot = stay_run + lanes_below(ms);
            stay_run += (uint32_t)__popcll(ms);
            // a record that leaves takes the next slot of its wavefront's range
            // in its group (in the order the LDS grants them)
            if (act && g != STAY) slot = atomicAdd(&mine[g], 1u);
            if (act && store) out[rec_slot(slot, p.cap, fix, ovf)] = make_uint2(rid[j], pk);
            if (TRANS) wsus += (uint32_t)__popcll(__ballot(sus));
        }
    }
    if (TRANS && p.scnt && lane == 0 && wsus) atomicAdd(&s_sus, wsus);
    __syncthreads();
    if (TRANS && p.scnt && tid == 0) p.scnt[tile] = s_sus;

    // counts of step t: the tile's border cells to the grid (the only ones a
    // neighbour reads: they lie on its ring), the ring to the tile's ring
    // array
    uint32_t *C = io.C_out;
    const uint32_t nb = 2 * w + 2 * (h - 2);
    for (uint32_t b = tid; b < nb; b += NT) {
        uint32_t lx, ly;
        if (b < 2 * w) {
            lx = b < w ? b : b - w;
            ly = b < w ? 0u : h - 1;
        } else {
            const uint32_t c = b - 2 * w;
            lx = c < h - 2 ? 0u : w - 1;
            ly = 1 + (c < h - 2 ? c : c - (h - 2));
        }
        C[(size_t)((uint32_t)y0 + ly) * (uint32_t)p.L + (uint32_t)x0 + lx] =
            hist[(ly + 1) * RW + lx + 1];
    }
    uint32_t *R = io.ring_out + (size_t)tile * p.rs;
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

// One workgroup: cursor[] (counts) -> generation-0 headers (the overflow
// ranges of tiles with more records than slots are laid out in tile order),
// cursor[] back to zero for the ranks.
__global__ void __launch_bounds__(1024) k_tile_scan(TileParams p)
{
    __shared__ uint32_t part[1024];
    __shared__ uint32_t carry;
    const uint32_t tid = threadIdx.x, nt = p.nT * p.nT;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (uint32_t c0 = 0; c0 < nt; c0 += 4 * 1024) {
        uint32_t v[4], sum = 0;
        uint32_t cnt[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = c0 + tid * 4 + j;
            cnt[j] = i < nt ? p.cursor[i] : 0u;
            v[j] = cnt[j] > p.cap ? cnt[j] - p.cap : 0u;     // records past the tile's slots
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
                H[0] = p.ovf0 + b;
                for (uint32_t g = 0; g < 9; ++g) H[1 + g] = g == STAY ? cnt[j] : 0u;
                p.cursor[i] = 0;
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
            if (h[b]) h[b] = atomicAdd(&p.cursor[b], h[b]);   // count -> first rank
        __syncthreads();
    }
#pragma unroll
    for (uint32_t j = 0; j < SORT_PER; ++j) {
        const uint32_t a = a0 + j * NT + tid;
        if (a >= p.n) continue;
        const int32_t x = p.x[a], y = p.y[a];
        const uint32_t tx = tile_of(p, x), ty = tile_of(p, y), b = ty * p.nT + tx;
        const uint32_t r = LDS ? h[bin[j]] + rank[j] : atomicAdd(&p.cursor[b], 1u);
        const uint32_t slot = rec_slot(r, p.cap, b * p.cap, p.hdr[0][(size_t)b * TILE_HDR]);
        const uint32_t lx = (uint32_t)x - tx * p.T, ly = (uint32_t)y - ty * p.T;
        p.rec[0][slot] = make_uint2(a, lx | (ly << 10) | ((uint32_t)p.s[a] << 20));
    }
}

// Columns from the tail's packed words (agent order): one thread per 4
// agents; a last partial group writes only its agents below n.  x and y fit
// 16 bits since L*L < 2^31.  With p.mark set (a gather segment follows) it
// also marks the cells its susceptible agents read at step p.mark_t: the
// gather segment's first launch then bins only infected agents on marked
// cells, as its later launches do (see sir_body_demand).
__global__ void __launch_bounds__(256) k_tile_unpack(const uint2 *__restrict__ packed,
                                                     TileParams p)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t a = 4 * q;
    const uint32_t n = p.n;
    if (a >= n) return;
    if (p.mark && q == 0) {
        p.mark_flags[0] = 1u;
        p.mark_flags[1] = 1u;
    }
    int32_t xs[4] = {0, 0, 0, 0}, ys[4] = {0, 0, 0, 0};
    uint32_t ss[4] = {ST_R, ST_R, ST_R, ST_R};
    if (a + 4 <= n) {
        const uint4 u0 = ((const uint4 *)packed)[2 * q], u1 = ((const uint4 *)packed)[2 * q + 1];
        xs[0] = (int32_t)(u0.x & 0xffffu);
        xs[1] = (int32_t)(u0.z & 0xffffu);
        xs[2] = (int32_t)(u1.x & 0xffffu);
        xs[3] = (int32_t)(u1.z & 0xffffu);
        ys[0] = (int32_t)(u0.x >> 16);
        ys[1] = (int32_t)(u0.z >> 16);
        ys[2] = (int32_t)(u1.x >> 16);
        ys[3] = (int32_t)(u1.z >> 16);
        ss[0] = u0.y;
        ss[1] = u0.w;
        ss[2] = u1.y;
        ss[3] = u1.w;
        ((int4 *)p.x)[q] = make_int4(xs[0], xs[1], xs[2], xs[3]);
        ((int4 *)p.y)[q] = make_int4(ys[0], ys[1], ys[2], ys[3]);
        ((uint32_t *)p.s)[q] = ss[0] | (ss[1] << 8) | (ss[2] << 16) | (ss[3] << 24);
    } else {
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {      // constant indices: the arrays stay in registers
            if (a + j >= n) continue;
            const uint2 u = packed[a + j];
            xs[j] = (int32_t)(u.x & 0xffffu);
            ys[j] = (int32_t)(u.x >> 16);
            ss[j] = u.y;
            p.x[a + j] = xs[j];
            p.y[a + j] = ys[j];
            p.s[a + j] = (uint8_t)u.y;
        }
    }
    if (!p.mark) return;
    bool any = false;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) any |= a + j < n && ss[j] == ST_S;
    if (!any) return;
    const uint4 r = philox(q, p.mark_t, P_MOVE, p.k0, p.k1);
    const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        if (a + j >= n || ss[j] != ST_S) continue;
        int32_t x2 = xs[j], y2 = ys[j];
        moore_move(u[j], p.L, x2, y2);
        mark_demand(p.mark, p.L, x2, y2);
        if (p.mark_cside) mark_coarse(p.mark_coarse, p.mark_cside, p.L, x2, y2);
    }
}

template <uint32_t T>
hipError_t step_launch(const TileParams &p, uint32_t t, uint32_t gen, uint32_t phase,
                       uint32_t block, hipStream_t st)
{
    StepIO io;
    io.rec_in = p.rec[gen];
    io.rec_out = p.rec[gen ^ 1];
    io.hdr_in = p.hdr[gen];
    io.hdr_out = p.hdr[gen ^ 1];
    io.C_in = p.C[gen ^ 1];        // counts of the previous launch
    io.C_out = p.C[gen];
    io.ring_in = p.ring[gen ^ 1];
    io.ring_out = p.ring[gen];
    io.ovf_out = p.ctr + 64 * (gen ^ 1);
    io.ovf_reset = p.ctr + 64 * gen;
    const dim3 grid(p.nT * p.nT), thr(block);
    if (phase == 0) hipLaunchKernelGGL((k_tile_step<T, false, true>), grid, thr, 0, st, p, io, t);
    else if (phase == 1) hipLaunchKernelGGL((k_tile_step<T, true, true>), grid, thr, 0, st, p, io, t);
    else hipLaunchKernelGGL((k_tile_step<T, true, false>), grid, thr, 0, st, p, io, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || phase != 2) return e;
    const uint32_t groups = (p.n + 3) / 4;
    hipLaunchKernelGGL(k_tile_unpack, dim3((groups + 255) / 256), dim3(256), 0, st, io.rec_out,
                       p);
    return hipGetLastError();
}

}  // namespace

uint32_t sir_tile_count(uint32_t L, uint32_t T)
{
    return L >= 2 * T + 2 ? (L - 2) / T + 1 : 0u;
}

uint32_t sir_tile_cap(uint32_t n, uint32_t nt)
{
    const uint64_t mean = ((uint64_t)n + nt - 1) / nt;
    return (uint32_t)((2 * mean + 64 + 63) / 64 * 64);
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

__global__ void __launch_bounds__(1024) k_sum_words(const uint32_t *__restrict__ a, uint32_t n,
                                                   uint32_t *dst)
{
    __shared__ uint32_t part[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    uint32_t v = 0;
    for (uint32_t i = tid; i < n; i += 1024) v += a[i];
    for (uint32_t off = 32; off; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) part[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        uint32_t s = 0;
        for (uint32_t k = 0; k < 16; ++k) s += part[k];
        __hip_atomic_store(dst, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

hipError_t launch_sum_words(const uint32_t *a, uint32_t n, uint32_t *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_words, dim3(1), dim3(1024), 0, st, a, n, dst);
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
