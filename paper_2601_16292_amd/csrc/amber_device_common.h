// amber_device_common.h -- device helpers shared by the single-run kernels
// (amber_device.hip) and the batched kernels (amber_batch.hip).
#pragma once

#include "amber_internal.h"

namespace amber {

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Multipliers and Weyl
// key increments as published.  The key lives in SGPRs (wavefront-uniform);
// each 32x32->64 product is one v_mad_u64_u32.  From the third round on both
// words are lane-varying and each three-way XOR is one v_bitop3_b32 (truth
// table 0x96); in the first two rounds the counter's constant and uniform
// words leave parts of the XORs to scalar code, so plain XORs stay there.
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
        const uint32_t n0 = r < 2 ? (uint32_t)(p1 >> 32) ^ c1 ^ k0
                                  : __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = r < 2 ? (uint32_t)(p0 >> 32) ^ c3 ^ k1
                                  : __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
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

// ------------------------------------------------------------------ per-group bodies
// Each body handles agent group q (agents 4q..4q+3) of one run.

// Random walk: steps t0 .. t0+n_steps-1 with positions in registers.
__device__ __forceinline__ void walk_group(int4 *__restrict__ x, int4 *__restrict__ y, uint32_t q,
                                           int32_t L, uint32_t k0, uint32_t k1, uint32_t t0,
                                           uint32_t n_steps)
{
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

// Wealth: one synchronous transfer step.  The state of agent a is base[a] +
// inc_cur[a]; the snapshot decides the donors (wealth > 0).  A donor's unit
// leaves base in place (plain store, the thread owns the row) and lands in
// inc_nxt[recipient] through an integer atomic add, so duplicates accumulate
// in any order with an identical result.  inc_cur is cleared for reuse two
// steps later.
__device__ __forceinline__ void wealth_step_group(int4 *__restrict__ base, int4 *__restrict__ inc_cur,
                                                  int32_t *__restrict__ inc_nxt, uint32_t q,
                                                  uint32_t n, uint32_t k0, uint32_t k1, uint32_t t)
{
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

__device__ __forceinline__ void wealth_fold_group(int4 *__restrict__ base, int4 *__restrict__ inc,
                                                  uint32_t q)
{
    const int4 B = base[q];
    const int4 I = inc[q];
    base[q] = make_int4(B.x + I.x, B.y + I.y, B.z + I.z, B.w + I.w);
    inc[q] = make_int4(0, 0, 0, 0);
}

// ------------------------------------------------------------------ block scan

// Exclusive prefix sum of in[0..n) into out[0..n) by a workgroup of THREADS
// threads (a multiple of 64, at most 1024), n <= THREADS * PER (each thread
// scans up to PER consecutive entries); T is a 32- or 16-bit unsigned type
// whose range holds every sum.  in and out may alias.  Ends with a barrier.
template <uint32_t THREADS, uint32_t PER, typename T>
__device__ __forceinline__ void block_exclusive_scan(const T *in, T *out, uint32_t n)
{
    constexpr uint32_t WAVES = THREADS / 64;
    __shared__ uint32_t wave_total[WAVES];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t per = (n + THREADS - 1) / THREADS;
    const uint32_t start = tid * per;
    uint32_t part[PER], sum = 0;
#pragma unroll
    for (uint32_t e = 0; e < PER; ++e) {
        const uint32_t idx = start + e;
        const uint32_t v = (e < per && idx < n) ? in[idx] : 0u;
        part[e] = sum;
        sum += v;
    }
    uint32_t incl = sum;
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wave_total[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        uint32_t wt = lane < WAVES ? wave_total[lane] : 0u;
        uint32_t wi = wt;
        for (uint32_t off = 1; off < WAVES; off <<= 1) {
            const uint32_t v = __shfl_up(wi, off, 64);
            if (lane >= off) wi += v;
        }
        if (lane < WAVES) wave_total[lane] = wi - wt;
    }
    __syncthreads();
    const uint32_t base = incl - sum + wave_total[wave];
#pragma unroll
    for (uint32_t e = 0; e < PER; ++e) {
        const uint32_t idx = start + e;
        if (e < per && idx < n) out[idx] = (T)(base + part[e]);
    }
    __syncthreads();
}

// ------------------------------------------------------------------ XCD-aware work mapping
// Item of workgroup b out of P items: workgroups are dealt to the 8 XCDs in
// turn (b mod 8), so this gives each XCD a run of consecutive items.
// Neighbouring items that read each other's data (wealth owners reading
// neighbouring table words and record pieces, tiles reading their
// neighbours' records and rings) then share that XCD's L2.  A bijection on
// [0, P) for any P; only speed depends on the dealing order.
__device__ __forceinline__ uint32_t xcd_partition(uint32_t b, uint32_t P)
{
    const uint32_t xcd = b & 7u, j = b >> 3;
    uint32_t start = 0;
    for (uint32_t y = 0; y < xcd; ++y) start += (P - y + 7) >> 3;   // items dealt to XCD y
    return start + j;
}

// ------------------------------------------------------------------ wealth, partition exchange
// The population is cut into partitions of XR = 2^XB consecutive agents and
// one workgroup of NT threads (512 or 1024) owns each partition.  The kernel of step t
//   (1) folds into its agents the units sent to them at step t-1: the
//       producers left their recipient ids sorted by destination partition,
//       so the owner reads only its share and counts it in an LDS histogram;
//   (2) decides its donors on the resulting snapshot, takes their unit, and
//       draws their recipients;
//   (3) counting-sorts those recipient ids by destination partition in LDS
//       and writes them to its own output segment with contiguous stores,
//       plus one (offset, count) word per destination.
// No global atomics are used, and the column is read and written once per
// step.  Records and tables are double-buffered by step parity; a call ends
// with a fold-only launch, so the column holds the state at every call
// boundary.

// Writes the producer's recipient ids to its output segment, grouped by
// destination: record (g, j) goes to position off[dest] + rank.  The ids are
// first placed in LDS (stage, at least `total` words, free at this point),
// then copied out with contiguous 16-byte stores, so that every memory line
// of the segment is written whole by one wavefront.
template <int G, int XB, int NT>
__device__ __forceinline__ void wealth_write_records(uint32_t *rec_out, uint32_t *stage,
                                                     const uint32_t (&rcp)[G][4],
                                                     const uint32_t (&rank)[G][4],
                                                     const uint32_t *off, uint32_t total)
{
#pragma unroll
    for (uint32_t g = 0; g < G; ++g)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (rcp[g][j] != 0xffffffffu) stage[off[rcp[g][j] >> XB] + rank[g][j]] = rcp[g][j];
    __syncthreads();
    for (uint32_t i = 4 * threadIdx.x; i < total; i += 4 * NT) {
        if (i + 4 <= total) {
            *(uint4 *)(rec_out + i) = *(const uint4 *)(stage + i);
        } else {
            for (uint32_t k = i; k < total; ++k) rec_out[k] = stage[k];
        }
    }
}

template <int XB, int PMAX, int NT>
__device__ __forceinline__ void wealth_exchange_partition(const WealthXParams &x, uint32_t p,
                                                          uint32_t t, uint32_t parity_in,
                                                          bool consume, bool produce,
                                                          int32_t *hist, uint32_t *pcount,
                                                          uint32_t *poff)
{
    constexpr uint32_t XR = 1u << XB;
    constexpr uint32_t G = XR / (4 * NT);      // 4-agent groups per thread
    const uint32_t tid = threadIdx.x;
    const uint32_t P = x.P;
    const uint32_t groups = groups_of(x.n);
    static_assert(PMAX <= NT, "one source per thread in the fold");
    // Fold: thread s (< P) reads source s's table entry, then its few records
    // for this partition.  The table entry is loaded before the barrier that
    // orders the histogram clear.
    const uint32_t *tab = x.tab[parity_in];
    const uint32_t e = consume && tid < P ? tab[(size_t)tid * P + p] : 0u;
    for (uint32_t i = tid; i < XR; i += NT) hist[i] = 0;
    __syncthreads();
    // Fold: the source's records [off, end) (agent ids; h is the histogram
    // shifted by the partition's first id), read with aligned 16-byte loads,
    // two per round, so a piece of a few records costs one or two loads at
    // any offset.  A segment is 16-byte aligned and a piece never passes its
    // end (a multiple of 4 words), so every load stays inside it; words
    // outside the piece are read and ignored.  The recipient draws do not
    // depend on who gives: they are made while the first window is in
    // flight.
    const uint32_t off = e >> 16, end = off + (e & 0xffffu);
    const uint32_t *seg = x.rec[parity_in] + (size_t)tid * XR;
    uint32_t k = off & ~3u;
    const bool first = consume && tid < P && k < end;
    uint4 u0 = make_uint4(0, 0, 0, 0);
    if (first) u0 = *(const uint4 *)(seg + k);
    uint32_t rcp[G][4], rank[G][4];
    if (produce) {
#pragma unroll
        for (uint32_t g = 0; g < G; ++g) {
            const uint32_t q = p * (XR / 4) + g * NT + tid;
            const uint4 r0 = philox(2 * q, t, P_RECIPIENT, x.k0, x.k1);
            const uint4 r1 = philox(2 * q + 1, t, P_RECIPIENT, x.k0, x.k1);
            rcp[g][0] = recipient(r0.x, r0.y, x.n);
            rcp[g][1] = recipient(r0.z, r0.w, x.n);
            rcp[g][2] = recipient(r1.x, r1.y, x.n);
            rcp[g][3] = recipient(r1.z, r1.w, x.n);
        }
    }
    if (first) {
        int32_t *h = hist - (size_t)p * XR;
        for (;;) {
            const uint4 u1 = k + 4 < end ? *(const uint4 *)(seg + k + 4) : make_uint4(0, 0, 0, 0);
            const uint32_t v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
            for (uint32_t j = 0; j < 8; ++j)
                if (k + j >= off && k + j < end) atomicAdd(&h[v[j]], 1);
            k += 8;
            if (k >= end) break;
            u0 = *(const uint4 *)(seg + k);
        }
    }
    for (uint32_t i = tid; i < P; i += NT) pcount[i] = 0;
    __syncthreads();
    int4 V[G];
#pragma unroll
    for (uint32_t g = 0; g < G; ++g) {
        const uint32_t local = g * NT + tid;                 // group within the partition
        const uint32_t q = p * (XR / 4) + local;
        V[g] = make_int4(0, 0, 0, 0);
        if (q < groups) {
            const int4 W = ((const int4 *)x.w)[q];
            V[g] = make_int4(W.x + hist[4 * local], W.y + hist[4 * local + 1],
                             W.z + hist[4 * local + 2], W.w + hist[4 * local + 3]);
        }
        if (!produce) {
            if (q < groups) ((int4 *)x.w)[q] = V[g];
            continue;
        }
        const uint32_t a = 4 * q;
        const int32_t v[4] = {V[g].x, V[g].y, V[g].z, V[g].w};
        bool d[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            d[j] = q < groups && v[j] > 0 && a + j < x.n;
            rcp[g][j] = d[j] ? rcp[g][j] : 0xffffffffu;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            rank[g][j] = d[j] ? atomicAdd(&pcount[rcp[g][j] >> XB], 1u) : 0u;
        if (q < groups)
            ((int4 *)x.w)[q] = make_int4(v[0] - d[0], v[1] - d[1], v[2] - d[2], v[3] - d[3]);
    }
    if (!produce) return;
    __syncthreads();
    block_exclusive_scan<NT, (PMAX + NT - 1) / NT>(pcount, poff, P);
    // the fold histogram (XR words) is dead: it stages the at most XR records
    wealth_write_records<G, XB, NT>(x.rec[parity_in ^ 1u] + (size_t)p * XR, (uint32_t *)hist,
                                    rcp, rank, poff, poff[P - 1] + pcount[P - 1]);
    uint32_t *tab_out = x.tab[parity_in ^ 1u] + (size_t)p * P;
    for (uint32_t d = tid; d < P; d += NT) tab_out[d] = (poff[d] << 16) | pcount[d];
}

// The same exchange with 16-bit fold counters and 16-bit records, for
// partitions of XR = 2^XB agents, XB = 15 or 16 (populations above 2^24).
// A record is the recipient's index within its destination partition (the
// segment it sits in names the source, its table entry the destination), so
// it takes two bytes.  LDS holds
//   h2[XR / 2]     the fold histogram, two 16-bit counters per word (agent 2i
//                  in the low half); after the produce loop, the stage of the
//                  outgoing records;
//   c32[PMAX + 2]  per-destination counts, then offsets (entry P = total),
//                  then placement cursors.
// With 2^16-agent partitions the table has a quarter of the entries of
// 2^15-agent ones and every owner reads half as many pieces, each twice as
// long: scattered reads bound the fold, so fewer and longer pieces win.
//
// A table entry is off << 16 | (cnt - 1) for a non-empty piece, all ones for
// an empty one (off + cnt <= XR, so a non-empty piece never encodes as all
// ones).
//
// A 16-bit fold counter wraps only if one agent receives 65536 units in one
// step.  Every add returns the word's previous value, so a wrap is seen;
// the owner then clears the histogram and folds again in two passes over
// half the partition each, with 32-bit counters added into the wealth
// column (`wide` takes that form from the start).
//
// Within one destination the records are placed in the order the LDS
// atomics grant the cursors; the owner only counts them, so the result does
// not depend on that order.
constexpr uint32_t WX16_EMPTY = 0xffffffffu;

// Adds the records of one source's piece [off, end) found in the aligned
// 8-record window u at position k to the 16-bit histogram; returns nonzero
// if a counter wrapped.  Branch-free: a record outside the piece adds 0 (to
// the word its bits name, masked into the partition).
template <int XB>
__device__ __forceinline__ uint32_t wealth_fold16_window(uint32_t *h2, const uint4 &u, uint32_t k,
                                                         uint32_t off, uint32_t end)
{
    const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
    const int32_t lo = (int32_t)(off - k), hi = (int32_t)(end - k);
    uint32_t wrap = 0;
#pragma unroll
    for (int32_t j = 0; j < 8; ++j) {
        const uint32_t v = (wd[j >> 1] >> (16 * (j & 1))) & ((1u << XB) - 1u);
        const uint32_t sh = 16 * (v & 1u);
        const uint32_t one = (j >= lo && j < hi) ? 1u : 0u;
        const uint32_t old = atomicAdd(&h2[v >> 1], one << sh);
        wrap |= (((old >> sh) & 0xffffu) + one) >> 16;
    }
    return wrap;
}

// The wide fold: the records of the piece whose index falls in half `half`
// of the partition, counted in 32-bit words (h32 spans XR / 2 agents).
template <int XB>
__device__ __forceinline__ void wealth_fold_wide(uint32_t *h32, const uint16_t *seg, uint32_t off,
                                                 uint32_t cnt, uint32_t half)
{
    const uint32_t end = off + cnt;
    for (uint32_t k = off; k < end; ++k) {
        const uint32_t v = seg[k];
        if ((v >> (XB - 1)) == half) atomicAdd(&h32[v & ((1u << (XB - 1)) - 1u)], 1u);
    }
}

template <int XB, int PMAX, int NT>
__device__ __forceinline__ void wealth_exchange_partition16(const WealthXParams &x, uint32_t p,
                                                            uint32_t t, uint32_t parity_in,
                                                            bool consume, bool produce,
                                                            bool wide, uint32_t *h2,
                                                            uint32_t *c32, uint32_t *flag)
{
    constexpr uint32_t XR = 1u << XB;
    constexpr uint32_t G = XR / (4 * NT);                   // 4-agent groups per thread
    constexpr uint32_t LPS = 4;                              // lanes per source in the fold
    constexpr uint32_t SPT = (PMAX + NT / LPS - 1) / (NT / LPS);   // sources per lane
    // Groups whose recipients are drawn during the fold (the rest in the
    // produce loop).  Each holds 4 more registers through the fold; with
    // 2^15-agent partitions two workgroups share a CU only within 64.
    constexpr uint32_t GF = (XB == 16 ? 3u : 4u) < G ? (XB == 16 ? 3u : 4u) : G;
    static_assert(G >= 1 && XB >= 4 && XB <= 16, "16-bit records");
    const uint32_t tid = threadIdx.x;
    const uint32_t P = x.P;
    const uint32_t groups = groups_of(x.n);
    // Table entries of this partition's sources; the clears happen before
    // the barrier.
    const uint32_t *tab = x.tab[parity_in];
    uint32_t e[SPT];
#pragma unroll
    for (uint32_t c = 0; c < SPT; ++c) {
        const uint32_t s = c * (NT / LPS) + tid / LPS;
        e[c] = consume && s < P ? tab[(size_t)s * P + p] : WX16_EMPTY;
    }
    for (uint32_t i = tid; i < XR / 2; i += NT) h2[i] = 0;
    for (uint32_t i = tid; i < PMAX + 2; i += NT) c32[i] = 0;
    if (tid == 0) *flag = 0;
    // The recipient draws do not depend on who gives, so a thread draws
    // those of its first GF agent groups while its table and piece loads
    // are in flight (slot 0 before the barrier, slot c + 1 with source c):
    // the Philox arithmetic fills the wait on the scattered loads.
    uint32_t rcp[G][4];
    auto draw = [&](uint32_t slot) {
#pragma unroll
        for (uint32_t g = 0; g < GF; ++g) {
            if (g * (SPT + 1) / GF != slot) continue;
            const uint32_t q = p * (XR / 4) + g * NT + tid;
            const uint4 r0 = philox(2 * q, t, P_RECIPIENT, x.k0, x.k1);
            const uint4 r1 = philox(2 * q + 1, t, P_RECIPIENT, x.k0, x.k1);
            rcp[g][0] = recipient(r0.x, r0.y, x.n);
            rcp[g][1] = recipient(r0.z, r0.w, x.n);
            rcp[g][2] = recipient(r1.x, r1.y, x.n);
            rcp[g][3] = recipient(r1.z, r1.w, x.n);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    if (produce) draw(0);
    __syncthreads();
    const uint16_t *rec = (const uint16_t *)x.rec[parity_in];
    uint32_t wrap = 0;
    // LPS neighbouring lanes share a source: lane w of them takes the
    // piece's aligned windows w, w + LPS, ...; their loads fall in the same
    // lines and are served together.
#pragma unroll
    for (uint32_t c = 0; c < SPT; ++c) {
        const bool has = !wide && e[c] != WX16_EMPTY;
        const uint32_t off = e[c] >> 16, end = off + (e[c] & 0xffffu) + 1;
        const uint16_t *seg = rec + (size_t)(c * (NT / LPS) + tid / LPS) * XR;
        uint32_t k = (off & ~7u) + 8 * (tid % LPS);
        const bool first = has && k < end;
        uint4 u = make_uint4(0, 0, 0, 0);
        if (first) u = *(const uint4 *)(seg + k);
        if (produce) draw(c + 1);
        if (first) {
            wrap |= wealth_fold16_window<XB>(h2, u, k, off, end);
            for (k += 8 * LPS; k < end; k += 8 * LPS)
                wrap |= wealth_fold16_window<XB>(h2, *(const uint4 *)(seg + k), k, off, end);
        }
    }
    if (wrap) *flag = 1;
    __syncthreads();
    if (wide || *flag) {               // a counter wrapped (or asked for): 32-bit, by halves
        for (uint32_t half = 0; half < 2; ++half) {
            for (uint32_t i = tid; i < XR / 2; i += NT) h2[i] = 0;
            __syncthreads();
#pragma unroll
            for (uint32_t c = 0; c < SPT; ++c)
                if (e[c] != WX16_EMPTY && tid % LPS == 0)
                    wealth_fold_wide<XB>(h2, rec + (size_t)(c * (NT / LPS) + tid / LPS) * XR,
                                         e[c] >> 16, (e[c] & 0xffffu) + 1, half);
            __syncthreads();
            for (uint32_t i = tid; i < XR / 8; i += NT) {
                const uint32_t q = p * (XR / 4) + half * (XR / 8) + i;
                if (q < groups) {
                    const int4 W = ((const int4 *)x.w)[q];
                    ((int4 *)x.w)[q] = make_int4(W.x + (int32_t)h2[4 * i], W.y + (int32_t)h2[4 * i + 1],
                                                 W.z + (int32_t)h2[4 * i + 2],
                                                 W.w + (int32_t)h2[4 * i + 3]);
                }
            }
            __syncthreads();
        }
        for (uint32_t i = tid; i < XR / 2; i += NT) h2[i] = 0;
        __syncthreads();
    }
#pragma unroll
    for (uint32_t g = 0; g < G; ++g) {
        const uint32_t local = g * NT + tid;                 // group within the partition
        const uint32_t q = p * (XR / 4) + local;
        int4 V = make_int4(0, 0, 0, 0);
        if (q < groups) {
            const int4 W = ((const int4 *)x.w)[q];
            const uint2 h = *(const uint2 *)(h2 + 2 * local);
            V = make_int4(W.x + (int32_t)(h.x & 0xffffu), W.y + (int32_t)(h.x >> 16),
                          W.z + (int32_t)(h.y & 0xffffu), W.w + (int32_t)(h.y >> 16));
        }
        if (!produce) {
            if (q < groups) ((int4 *)x.w)[q] = V;
            continue;
        }
        const uint32_t a = 4 * q;
        const int32_t v[4] = {V.x, V.y, V.z, V.w};
        bool d[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) d[j] = q < groups && v[j] > 0 && a + j < x.n;
        if (g >= GF) {
            const uint4 r0 = philox(2 * q, t, P_RECIPIENT, x.k0, x.k1);
            const uint4 r1 = philox(2 * q + 1, t, P_RECIPIENT, x.k0, x.k1);
            rcp[g][0] = recipient(r0.x, r0.y, x.n);
            rcp[g][1] = recipient(r0.z, r0.w, x.n);
            rcp[g][2] = recipient(r1.x, r1.y, x.n);
            rcp[g][3] = recipient(r1.z, r1.w, x.n);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) rcp[g][j] = d[j] ? rcp[g][j] : 0xffffffffu;
        // a non-donor adds 0 to a word of its own lane (no same-word conflicts)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            atomicAdd(&c32[d[j] ? rcp[g][j] >> XB : (tid & 63u)], d[j] ? 1u : 0u);
        if (q < groups)
            ((int4 *)x.w)[q] = make_int4(v[0] - d[0], v[1] - d[1], v[2] - d[2], v[3] - d[3]);
        __builtin_amdgcn_sched_barrier(0);   // one group at a time: fewer live registers
    }
    if (!produce) return;
    __syncthreads();
    block_exclusive_scan<NT, (PMAX + NT) / NT>(c32, c32, P + 1);   // entry P: the total
    const uint32_t n_rec = c32[P];
    uint32_t *tab_out = x.tab[parity_in ^ 1u] + (size_t)p * P;
    for (uint32_t dd = tid; dd < P; dd += NT) {
        const uint32_t o = c32[dd], cnt = c32[dd + 1] - o;
        tab_out[dd] = cnt ? (o << 16) | (cnt - 1) : WX16_EMPTY;
    }
    __syncthreads();
    // place each record at its destination's cursor in the stage (the dead
    // histogram), then copy the stage out with 16-byte stores; the stage's
    // words past n_rec are stale and never read
    uint16_t *stage = (uint16_t *)h2;
#pragma unroll
    for (uint32_t g = 0; g < G; ++g)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (rcp[g][j] != 0xffffffffu)
                stage[atomicAdd(&c32[rcp[g][j] >> XB], 1u)] = (uint16_t)(rcp[g][j] & (XR - 1));
    __syncthreads();
    uint16_t *rec_out = (uint16_t *)x.rec[parity_in ^ 1u] + (size_t)p * XR;
    for (uint32_t i = 8 * tid; i < n_rec; i += 8 * NT)
        *(uint4 *)(rec_out + i) = *(const uint4 *)(stage + i);
}

// Small populations: one workgroup runs every step with the wealth column and
// the increments in LDS; two barriers per step separate the donor/scatter
// phase from the apply phase.  A thread owns agent pairs (one RECIPIENT
// block per pair).
constexpr uint32_t WEALTH_SMALL_THREADS = 1024;
constexpr uint32_t WEALTH_SMALL_MAX = 8192;   // 2 x 32 KB of LDS

__device__ __forceinline__ void wealth_small_run(int32_t *__restrict__ w, int32_t *sw, int32_t *sinc,
                                                 uint32_t n, uint32_t k0, uint32_t k1, uint32_t t0,
                                                 uint32_t n_steps)
{
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
// Step t maps (positions, states) at the start of step t to the next state:
//   move(t)       every agent moves by its MOVE word (the random-walk rule);
//   bin(t)        C_t[c] = number of agents infected at the start of step t
//                 whose post-move cell is c (integer atomic adds);
//   transition(t) S -> I iff EPI word < T_inf[min(k, k_sat)] with k the infected
//                 count of the distinct cells of the 3x3 torus block, I -> R iff
//                 EPI word < T_rec, from C_t and the start-of-step state.
//
// Workspace grids: count[0..2], each L*L uint32, all zero at every call
// boundary.  Inside a call (first step t_base) the grids are used by the
// step's offset i = t - t_base, so every launch form starts from the same
// state and forms can be mixed between calls on one handle:
//   gather mode  C_t = count[i % 3]; transition(t) sums the 3x3 block of C_t
//                (9 cells, read as three 3-cell rows);
//   box mode     C_t = count[i % 2]; a stencil kernel writes the box-summed
//                K = count[2] (K[c] = k of any agent in cell c), so
//                transition(t) reads one cell of K.
// The last kernels of a call leave the used grids zero again.
//
// Pipelined form (any N): "head" = move+bin(t0); "body"(t) = transition(t-1)
// then move+bin(t), with the positions and states of its 4 agents held in
// registers between the halves, so each column is read and written once per
// step; "tail" = transition(t_last).  n steps cost n+1 launches (box mode adds
// one stencil launch per step).
//
// Persistent form (N up to what the chip holds in registers): one cooperative
// launch; each thread keeps its agents' positions and states in registers for
// every step, and one grid barrier per step separates bin(t) from
// transition(t).

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

__device__ __forceinline__ void sir_move4(const SirParams &p, uint32_t q, uint32_t t, int4 &X,
                                          int4 &Y)
{
    const uint4 r = philox(q, t, P_MOVE, p.k0, p.k1);
    moore_move(r.x, p.L, X.x, Y.x);
    moore_move(r.y, p.L, X.y, Y.y);
    moore_move(r.z, p.L, X.z, Y.z);
    moore_move(r.w, p.L, X.w, Y.w);
}

// Bin the infected among agents 4q..4q+3 (state word S) at (X, Y).
__device__ __forceinline__ void sir_bin4(const SirParams &p, uint32_t *__restrict__ count,
                                         uint32_t q, uint32_t S, const int4 &X, const int4 &Y)
{
    const uint32_t a = 4 * q;
    bin_infected(count, p.L, (S & 0xffu) == ST_I && a + 0 < p.n, X.x, Y.x);
    bin_infected(count, p.L, ((S >> 8) & 0xffu) == ST_I && a + 1 < p.n, X.y, Y.y);
    bin_infected(count, p.L, ((S >> 16) & 0xffu) == ST_I && a + 2 < p.n, X.z, Y.z);
    bin_infected(count, p.L, (S >> 24) == ST_I && a + 3 < p.n, X.w, Y.w);
}

// Three consecutive cells x-1, x, x+1 of one row, 1 <= x <= L-2: one
// dword-aligned 12-byte load.
struct __attribute__((packed, aligned(4))) Cells3 {
    uint32_t a, b, c;
};

__device__ __forceinline__ uint32_t row3(const uint32_t *__restrict__ row, int32_t x, int32_t L)
{
    if (x >= 1 && x <= L - 2) {
        const Cells3 v = *(const Cells3 *)(row + x - 1);
        return v.a + v.b + v.c;
    }
    const int32_t xm = x == 0 ? L - 1 : x - 1;
    const int32_t xp = x == L - 1 ? 0 : x + 1;
    return row[xm] + row[x] + row[xp];
}

// Infected agents in the distinct cells of the 3x3 torus block around (cx, cy).
__device__ __forceinline__ uint32_t block_count(const uint32_t *__restrict__ count, int32_t L,
                                                int32_t cx, int32_t cy)
{
    if (!on_grid(cx, cy, L)) return 0;
    if (L >= 3) {
        const int32_t ym = cy == 0 ? L - 1 : cy - 1;
        const int32_t yp = cy == L - 1 ? 0 : cy + 1;
        return row3(count + (uint32_t)ym * L, cx, L) + row3(count + (uint32_t)cy * L, cx, L) +
               row3(count + (uint32_t)yp * L, cx, L);
    }
    // L = 1 or 2: the wrapped block covers each of the L*L cells exactly once.
    uint32_t k = 0;
    for (int32_t c = 0; c < L * L; ++c) k += count[c];
    return k;
}

// k of an agent at (cx, cy): from the count grid (gather mode) or from the
// box-summed grid (box mode).
template <bool BOX>
__device__ __forceinline__ uint32_t neighbour_k(const uint32_t *__restrict__ g, int32_t L,
                                                int32_t cx, int32_t cy)
{
    if (BOX) return on_grid(cx, cy, L) ? g[(uint32_t)cy * L + cx] : 0u;
    return block_count(g, L, cx, cy);
}

// k of the susceptible agents among 4 (0 for the others).  Every load of the
// four agents is issued before any result is used, so a wavefront waits for
// one memory round trip instead of one per agent; a non-susceptible agent
// reads its own cell (a valid address) and its sum is discarded.  Gather
// mode reads each of the three rows as one 12-byte load starting at
// clamp(x-1, 0, L-3); an agent on the first or last column (1 in L/2 of
// agents) adds the wrapped cell with one more load.
template <bool BOX>
__device__ __forceinline__ void neighbour_k4(const uint32_t *__restrict__ g, int32_t L,
                                             const uint32_t st[4], const int4 &X, const int4 &Y,
                                             uint32_t k[4])
{
    const int32_t xs[4] = {X.x, X.y, X.z, X.w};
    const int32_t ys[4] = {Y.x, Y.y, Y.z, Y.w};
    bool use[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) use[j] = st[j] == ST_S && on_grid(xs[j], ys[j], L);
    if (BOX) {
        uint32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t c = use[j] ? (uint32_t)ys[j] * L + (uint32_t)xs[j] : 0u;
            v[j] = g[c];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) k[j] = use[j] ? v[j] : 0u;
        return;
    }
    if (L < 3) {
#pragma unroll
        for (int j = 0; j < 4; ++j) k[j] = use[j] ? block_count(g, L, xs[j], ys[j]) : 0u;
        return;
    }
    Cells3 r[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int32_t x = use[j] ? xs[j] : 1, y = use[j] ? ys[j] : 1;
        const int32_t s0 = x == 0 ? 0 : (x == L - 1 ? L - 3 : x - 1);
        const int32_t ym = y == 0 ? L - 1 : y - 1;
        const int32_t yp = y == L - 1 ? 0 : y + 1;
        r[j][0] = *(const Cells3 *)(g + (uint32_t)ym * L + s0);
        r[j][1] = *(const Cells3 *)(g + (uint32_t)y * L + s0);
        r[j][2] = *(const Cells3 *)(g + (uint32_t)yp * L + s0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t sum = 0;
        const int32_t x = xs[j];
        if (!use[j]) {
            k[j] = 0;
            continue;
        }
        if (x != 0 && x != L - 1) {
#pragma unroll
            for (int rr = 0; rr < 3; ++rr) sum += r[j][rr].a + r[j][rr].b + r[j][rr].c;
        } else {
            // first column: rows hold cells 0,1,2 and the wrapped cell is L-1;
            // last column: rows hold L-3,L-2,L-1 and the wrapped cell is 0
            const int32_t y = ys[j];
            const int32_t ym = y == 0 ? L - 1 : y - 1;
            const int32_t yp = y == L - 1 ? 0 : y + 1;
            const uint32_t wrap = x == 0 ? (uint32_t)(L - 1) : 0u;
            const uint32_t rows[3] = {(uint32_t)ym, (uint32_t)y, (uint32_t)yp};
#pragma unroll
            for (int rr = 0; rr < 3; ++rr) {
                const uint32_t pair = x == 0 ? r[j][rr].a + r[j][rr].b : r[j][rr].b + r[j][rr].c;
                sum += pair + g[rows[rr] * L + wrap];
            }
        }
        k[j] = sum;
    }
}

// transition(t) of agents 4q..4q+3: returns the new state word.
template <bool BOX>
__device__ __forceinline__ uint32_t sir_transition4(const SirParams &p,
                                                    const uint32_t *__restrict__ count,
                                                    uint32_t q, uint32_t t, uint32_t S,
                                                    const int4 &X, const int4 &Y)
{
    const uint32_t a = 4 * q;
    uint32_t st[4], k[4] = {0, 0, 0, 0};
    bool any_sus = false, need = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        st[j] = (a + j < p.n) ? (S >> (8 * j)) & 0xffu : (uint32_t)ST_R;   // padding never changes
        any_sus |= st[j] == ST_S;
    }
    if (any_sus) neighbour_k4<BOX>(count, p.L, st, X, Y, k);
#pragma unroll
    for (int j = 0; j < 4; ++j) need |= (st[j] == ST_S && k[j] > 0) || st[j] == ST_I;
    if (!need) return S;
    // the four thresholds are loaded unconditionally, before the Philox
    // block, so the loads are in flight together while it is computed
    const uint32_t k_last = p.table_len - 1;
    uint32_t thr[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) thr[j] = p.t_inf[k[j] < k_last ? k[j] : k_last];
    const uint4 r = philox(q, t, P_EPI, p.k0, p.k1);
    const uint32_t u[4] = {r.x, r.y, r.z, r.w};
    uint32_t out = S;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t ns = st[j];
        if (st[j] == ST_S && k[j] > 0) {
            if (u[j] < thr[j]) ns = ST_I;
        } else if (st[j] == ST_I) {
            if (u[j] < p.t_rec) ns = ST_R;
        }
        out = (out & ~(0xffu << (8 * j))) | (ns << (8 * j));
    }
    return out;
}

__device__ __forceinline__ void zero_quads(uint32_t *__restrict__ p, uint32_t quads, uint32_t i,
                                           uint32_t stride)
{
    uint4 *p4 = (uint4 *)p;
    for (; i < quads; i += stride) p4[i] = make_uint4(0, 0, 0, 0);
}

// Count grid of step t: gather mode rotates three grids, box mode two.
__device__ __forceinline__ uint32_t *grid_of(const SirParams &p, uint32_t t)
{
    return p.count[(t - p.t_base) % 3];
}
__device__ __forceinline__ uint32_t *cgrid_box(const SirParams &p, uint32_t t)
{
    return p.count[(t - p.t_base) & 1];
}
__device__ __forceinline__ uint32_t *kgrid_box(const SirParams &p) { return p.count[2]; }

// Grid a transition(t) reads in each mode.
template <bool BOX>
__device__ __forceinline__ const uint32_t *kin(const SirParams &p, uint32_t t)
{
    return BOX ? kgrid_box(p) : grid_of(p, t);
}
// Grid bin(t) adds into in each mode.
template <bool BOX>
__device__ __forceinline__ uint32_t *bin_target(const SirParams &p, uint32_t t)
{
    return BOX ? cgrid_box(p, t) : grid_of(p, t);
}

// head(t): move + bin(t) of group q.
// Column accesses of the per-step SIR kernels are streaming: marked
// non-temporal so they do not push the count grid (gathered at random) out
// of the L2.
typedef int32_t i32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int4 load_nt4(const int32_t *p, uint32_t q)
{
    const i32x4_t v = __builtin_nontemporal_load((const i32x4_t *)p + q);
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void store_nt4(int32_t *p, uint32_t q, const int4 &v)
{
    const i32x4_t w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, (i32x4_t *)p + q);
}
__device__ __forceinline__ uint32_t load_nt1(const uint8_t *p, uint32_t q)
{
    return __builtin_nontemporal_load((const uint32_t *)p + q);
}
__device__ __forceinline__ void store_nt1(uint8_t *p, uint32_t q, uint32_t v)
{
    __builtin_nontemporal_store(v, (uint32_t *)p + q);
}

template <bool BOX>
__device__ __forceinline__ void sir_head_group(const SirParams &p, uint32_t q, uint32_t t)
{
    int4 X = load_nt4(p.x, q);
    int4 Y = load_nt4(p.y, q);
    const uint32_t S = load_nt1(p.s, q);
    sir_move4(p, q, t, X, Y);
    store_nt4(p.x, q, X);
    store_nt4(p.y, q, Y);
    sir_bin4(p, bin_target<BOX>(p, t), q, S, X, Y);
}

// body(t): transition(t-1), then move + bin(t) of group q.
template <bool BOX>
__device__ __forceinline__ void sir_body_group(const SirParams &p, uint32_t q, uint32_t t)
{
    int4 X = load_nt4(p.x, q);
    int4 Y = load_nt4(p.y, q);
    const uint32_t S = load_nt1(p.s, q);
    const uint32_t S2 = sir_transition4<BOX>(p, kin<BOX>(p, t - 1), q, t - 1, S, X, Y);
    sir_move4(p, q, t, X, Y);
    store_nt4(p.x, q, X);
    store_nt4(p.y, q, Y);
    if (S2 != S) store_nt1(p.s, q, S2);
    sir_bin4(p, bin_target<BOX>(p, t), q, S2, X, Y);
}

// tail(t): transition(t) of group q.
template <bool BOX>
__device__ __forceinline__ void sir_tail_group(const SirParams &p, uint32_t q, uint32_t t)
{
    const int4 X = load_nt4(p.x, q);
    const int4 Y = load_nt4(p.y, q);
    const uint32_t S = load_nt1(p.s, q);
    const uint32_t S2 = sir_transition4<BOX>(p, kin<BOX>(p, t), q, t, S, X, Y);
    if (S2 != S) store_nt1(p.s, q, S2);
}

// ------------------------------------------------------------------ SIR, demand-driven binning
// The gather mode bins an infected agent into the count grid only where some
// susceptible agent will read the count.  Susceptible agents never come
// back, and an agent's move of step t+1 is a function of its id and t+1
// only, so launch i of a call (call-relative, step t) can draw the move of
// step t+1 of each of its susceptible agents and mark, in demand map
// (i+1) % 3, the 3 x 3 block that agent reads at step t+1.  Launch i+1 then
// bins only the infected agents whose cell is marked.  Marking costs one
// extra move draw per group of four agents holding a susceptible one and 9
// byte stores per susceptible agent; it saves one global atomic per
// infected agent off the marked cells.
//
// Flag F_j of step j is decided by launch j-2 from the complete S and I
// counts of step j-3: 1 = targeted binning (sir_targeted), 2 = no
// susceptible agent left, 0 = neither.  Launch j-1 marks iff F_j = 1 and
// launch j bins on marked cells iff F_j = 1, so the two always agree;
// F_0 = F_1 = F_2 = 0, except after a tiled segment of the same call: the
// tiled mode's last launch then marks map 0 for the head and sets F_0 =
// F_1 = 1, and the head's bookkeeping F_2 = 1 (any F_j = 1 is exact as
// long as the marks of launch j-1 cover the cells read at step j).  Every
// count that is read is exact; counts nobody reads are not produced.
//
// Susceptible agents never come back, so once F_j = 2 no count is read
// again in the call, and F stays 2.  The agents' remaining steps are then
// independent of each other: the first launch with F = 2 runs every
// remaining step of the call for its agents in registers (recoveries and
// moves, and the tail's transition), and the later launches do nothing.
// They bin, mark, count and clear nothing; the tail clears all three count
// grids for the next call (sir_demand_dirty).

// Targeted binning pays a dependent byte load per infected agent, and the
// marking a move draw and 9 byte stores per susceptible agent, for the
// atomics it saves off the marked cells (about a fraction exp(-9 S / L^2)
// of them).  Measured at N = L^2 = 1e6, it pays once the atomics are many
// (at least a tenth of the agents infected) and 3 S <= L^2, i.e. while up
// to about 95 % of the cells are marked.
__device__ __forceinline__ bool sir_targeted(uint32_t ns, uint32_t ni, uint32_t n, int32_t L)
{
    return 3ull * ns <= (uint64_t)L * (uint64_t)L && 10ull * ni >= (uint64_t)n;
}

// Counts of call-relative step j: slot k of S at [k * NSI_STRIDE], of I at
// [(NSI_SLOTS + k) * NSI_STRIDE].
__device__ __forceinline__ uint32_t *sir_counts_of(const SirParams &p, uint32_t j)
{
    return p.nsi + (j & 3u) * 2 * NSI_SLOTS * NSI_STRIDE;
}

// Bookkeeping of launch i, run by one extra workgroup that holds no agents
// (so the latency of reading the counts stays off the agents' path):
// publish F_{i+2} and zero the counts of step i+1 (last read by launch i-1).
__device__ __forceinline__ void sir_demand_book(const SirParams &p, uint32_t i)
{
    if (threadIdx.x < 64) {
        // launch 0: F_2 follows F_0 (1 only after a tiled segment)
        uint32_t flag = i == 0 && p.nsi[NSI_FLAGS] == 1u ? 1u : 0u;
        if (i >= 1) {
            const uint32_t *c = sir_counts_of(p, i - 1);
            uint32_t a = c[threadIdx.x * NSI_STRIDE];
            uint32_t b = c[(NSI_SLOTS + threadIdx.x) * NSI_STRIDE];
            for (int off = 32; off >= 1; off >>= 1) {
                a += __shfl_xor(a, off, 64);
                b += __shfl_xor(b, off, 64);
            }
            flag = a == 0 ? 2u : sir_targeted(a, b, p.n, p.L) ? 1u : 0u;
        }
        if (threadIdx.x == 0) p.nsi[NSI_FLAGS + ((i + 2) & 3u)] = flag;
    }
    for (uint32_t k = threadIdx.x; k < 2 * NSI_SLOTS; k += blockDim.x)
        sir_counts_of(p, i + 1)[k * NSI_STRIDE] = 0;
}

// Modes of body launch i >= 1: bit 0 = mark demand map (i+1) % 3
// (F_{i+1} = 1), bit 1 = bin only marked cells (F_i = 1), bit 2 = no
// susceptible agent left (F_i = 2), bit 3 = an earlier launch has already
// run the call's remaining steps (F_{i-1} = 2).  Slot (i-1) & 3 is next
// written by launch i+1.
__device__ __forceinline__ uint32_t sir_demand_modes(const SirParams &p, uint32_t i)
{
    const uint32_t mark = p.nsi[NSI_FLAGS + ((i + 1) & 3u)];
    const uint32_t cur = p.nsi[NSI_FLAGS + (i & 3u)];
    const uint32_t prev = p.nsi[NSI_FLAGS + ((i - 1) & 3u)];
    return (mark == 1u ? 1u : 0u) | (cur == 1u ? 2u : 0u) | (cur == 2u ? 4u : 0u) |
           (prev == 2u ? 8u : 0u);
}

// Whether the call ran out of susceptible agents: F of the last body launch
// enqueued (call-relative index i) is 2.  Then a body launch has run the
// tail's transition too, and some launches skipped their grid clears.  F_i
// is not overwritten before the call ends (launch i writes F_{i+2}).  The
// host stops enqueueing body launches early only after the launch that runs
// the remaining steps has started, so F_i = 2 then.
__device__ __forceinline__ bool sir_demand_dirty(const SirParams &p, uint32_t i)
{
    return p.nsi[NSI_FLAGS + (i & 3u)] == 2u;
}

// Adds the S and I agents of the group's states (packed S) to the counts of
// step i: wavefront sums from ballots into per-wavefront LDS words (s_wc,
// 2 per wavefront), a workgroup sum after one barrier, then one atomic per
// workgroup and kind into one of NSI_SLOTS lines.  Every thread of the
// workgroup must call it.
__device__ __forceinline__ void sir_count_states(const SirParams &p, uint32_t i, uint32_t q,
                                                 uint32_t S, bool valid, uint32_t *s_wc,
                                                 uint32_t block)
{
    uint32_t cs = 0, ci = 0;
    if (valid) {
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint32_t st = (S >> (8 * k)) & 0xffu;
            const bool in = 4 * q + k < p.n;
            cs += in && st == ST_S;
            ci += in && st == ST_I;
        }
    }
    uint32_t ws = 0, wi = 0;
#pragma unroll
    for (uint32_t b = 0; b < 3; ++b) {
        ws += (uint32_t)__popcll(__ballot((cs >> b) & 1u)) << b;
        wi += (uint32_t)__popcll(__ballot((ci >> b) & 1u)) << b;
    }
    if ((threadIdx.x & 63u) == 0) {
        s_wc[2 * (threadIdx.x >> 6)] = ws;
        s_wc[2 * (threadIdx.x >> 6) + 1] = wi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t ts = 0, ti = 0;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
            ts += s_wc[2 * w];
            ti += s_wc[2 * w + 1];
        }
        const uint32_t slot = block % NSI_SLOTS;
        uint32_t *c = sir_counts_of(p, i);
        if (ts) atomicAdd(&c[slot * NSI_STRIDE], ts);
        if (ti) atomicAdd(&c[(NSI_SLOTS + slot) * NSI_STRIDE], ti);
    }
}

// Coarse demand map that follows fine map m: one byte per 8 x 8 block of
// cells, marked whenever a cell of the block is.  On grids larger than an
// L2, an infected agent reads its block's byte (a small map that stays in
// the L2) and its cell's byte only on a marked block: once few susceptible
// agents are left, most of the random reads of the big fine map go.
__device__ __forceinline__ uint8_t *coarse_of(const SirParams &p, const uint8_t *m)
{
    const size_t cells = (size_t)(uint32_t)p.L * (uint32_t)p.L;
    return (uint8_t *)m + ((cells + 255) & ~(size_t)255);
}

__device__ __forceinline__ uint32_t coarse_quads(const SirParams &p)
{
    return (p.cside * p.cside + 15) / 16;
}

// Marks the coarse blocks of the wrapped 3 x 3 block around (x, y): the
// blocks of the three columns and three rows (the middle one only when it
// differs from both ends).
__device__ __forceinline__ void mark_coarse(uint8_t *__restrict__ c, uint32_t cs, int32_t L,
                                            int32_t x, int32_t y)
{
    if (!on_grid(x, y, L)) return;
    const uint32_t bx[3] = {(uint32_t)wrap_step(x, -1, L) >> 3, (uint32_t)x >> 3,
                            (uint32_t)wrap_step(x, 1, L) >> 3};
    const uint32_t by[3] = {(uint32_t)wrap_step(y, -1, L) >> 3, (uint32_t)y >> 3,
                            (uint32_t)wrap_step(y, 1, L) >> 3};
    const bool midx = bx[1] != bx[0] && bx[1] != bx[2], midy = by[1] != by[0] && by[1] != by[2];
    for (uint32_t j = 0; j < 3; ++j) {
        if (j == 1 && !midy) continue;
        for (uint32_t k = 0; k < 3; ++k) {
            if (k == 1 && !midx) continue;
            c[by[j] * cs + bx[k]] = 1;
        }
    }
}

// Marks the wrapped 3 x 3 block around (x, y): the cells a susceptible agent
// at (x, y) reads.
__device__ __forceinline__ void mark_demand(uint8_t *__restrict__ d, int32_t L, int32_t x, int32_t y)
{
    if (!on_grid(x, y, L)) return;
    for (int32_t dy = -1; dy <= 1; ++dy) {
        uint8_t *row = d + (size_t)wrap_step(y, dy, L) * (uint32_t)L;
        for (int32_t dx = -1; dx <= 1; ++dx) row[wrap_step(x, dx, L)] = 1;
    }
}

// Binning (all infected agents, or only those on marked cells) and marking
// of one group after its transition and move of step t.
__device__ __forceinline__ void sir_bin_mark4(const SirParams &p, uint32_t *__restrict__ count,
                                              uint32_t q, uint32_t t, uint32_t S, const int4 &X,
                                              const int4 &Y, uint32_t mode,
                                              const uint8_t *__restrict__ dcur,
                                              uint8_t *__restrict__ dnext)
{
    const uint32_t a = 4 * q;
    const int32_t xs[4] = {X.x, X.y, X.z, X.w}, ys[4] = {Y.x, Y.y, Y.z, Y.w};
    bool mark = false;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
        mark |= (mode & 1u) && a + k < p.n && ((S >> (8 * k)) & 0xffu) == ST_S;
    uint4 r = make_uint4(0, 0, 0, 0);
    if (mark) r = philox(q, t + 1, P_MOVE, p.k0, p.k1);     // the moves of step t+1
    const uint32_t u[4] = {r.x, r.y, r.z, r.w};
    const uint8_t *ccur = p.cside && (mode & 2u) ? coarse_of(p, dcur) : nullptr;
    uint8_t *cnext = p.cside && (mode & 1u) ? coarse_of(p, dnext) : nullptr;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t st = (S >> (8 * k)) & 0xffu;
        if (a + k >= p.n || !on_grid(xs[k], ys[k], p.L)) continue;
        const uint32_t c = (uint32_t)ys[k] * (uint32_t)p.L + (uint32_t)xs[k];
        if (st == ST_I &&
            (!(mode & 2u) ||
             ((!ccur || ccur[((uint32_t)ys[k] >> 3) * p.cside + ((uint32_t)xs[k] >> 3)]) &&
              dcur[c])))
            atomicAdd(&count[c], 1u);
        if (st == ST_S && (mode & 1u)) {
            int32_t x2 = xs[k], y2 = ys[k];
            moore_move(u[k], p.L, x2, y2);
            mark_demand(dnext, p.L, x2, y2);
            if (cnext) mark_coarse(cnext, p.cside, p.L, x2, y2);
        }
    }
}

// Recoveries of steps u0 .. u1 of the group's infected agents (bit j of inf
// = agent 4q+j), with no susceptible agent left: an infected agent recovers
// at the first of its draws below t_rec, and nothing else reads the draws.
// The lanes of a wavefront share the draws.  Each round, the na groups that
// still hold infected agents and steps get m = floor(64 / na) lanes each,
// one lane per consecutive step, and each agent takes the first of its m
// draws that hits.  A group then needs a draw only while it holds an
// infected agent, and the wavefront runs about as many rounds as the sum of
// those draws over 64.  While more than 32 groups draw, m would be 1 and the
// sharing would only move each group's draw to another lane: each lane then
// draws its own group's next step, with none of the lane exchanges.  Returns
// the bits of the agents still infected.  Every lane of the wavefront must
// call it.
__device__ __forceinline__ uint32_t sir_recover_wave(const SirParams &p, uint32_t q, uint32_t inf,
                                                     uint32_t u0, uint32_t u1)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t below = (1ull << lane) - 1;
    uint32_t left = u1 - u0 + 1;                   // draws this group may still take
    for (;;) {
        const bool active = inf != 0 && left != 0;
        const uint64_t A = __ballot(active);
        if (A == 0) break;
        const uint32_t na = (uint32_t)__popcll(A);
        if (na > 32) {                                          // wavefront-uniform
            if (active) {
                const uint4 r = philox(q, u1 + 1 - left, P_EPI, p.k0, p.k1);
                inf &= ~((r.x < p.t_rec ? 1u : 0u) | (r.y < p.t_rec ? 2u : 0u) |
                         (r.z < p.t_rec ? 4u : 0u) | (r.w < p.t_rec ? 8u : 0u));
                left -= 1;
            }
            continue;
        }
        const uint32_t m = 64u / na;                            // lanes per group
        // rank of the active lanes 0 .. na-1 in lane order (the inactive ones
        // after them), and lane_of[r] = the lane of rank r
        const uint32_t rank = active ? (uint32_t)__popcll(A & below)
                                     : na + (uint32_t)__popcll(~A & below);
        const uint32_t lane_of = (uint32_t)__builtin_amdgcn_ds_permute((int)(rank * 4), (int)lane);
        const uint32_t slot = lane / m, off = lane - slot * m;
        const uint32_t owner = (uint32_t)__builtin_amdgcn_ds_bpermute(
            (int)((slot < na ? slot : 0u) * 4), (int)lane_of);
        const uint32_t oq = __shfl(q, (int)owner);
        const uint32_t oinf = __shfl(inf, (int)owner);
        const uint32_t oleft = __shfl(left, (int)owner);
        uint32_t hit = 0;
        if (slot < na && off < oleft) {
            const uint4 r = philox(oq, u1 + 1 - oleft + off, P_EPI, p.k0, p.k1);
            hit = (r.x < p.t_rec ? 1u : 0u) | (r.y < p.t_rec ? 2u : 0u) |
                  (r.z < p.t_rec ? 4u : 0u) | (r.w < p.t_rec ? 8u : 0u);
            hit &= oinf;
        }
        const uint64_t seg = m == 64 ? ~0ull : ((1ull << m) - 1);
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint64_t B = __ballot((hit >> j) & 1u);
            if (active && ((B >> (rank * m)) & seg)) inf &= ~(1u << j);
        }
        if (active) left = left > m ? left - m : 0u;
    }
    return inf;
}

// The launch that finishes a call with no susceptible agent left: for the
// group of this thread (valid = it holds agents), the moves of steps
// t .. t_last and the recoveries of steps t-1 .. t_last, in registers.
// Moves and recoveries are independent then.  Every lane of the wavefront
// must call it.
__device__ __forceinline__ void sir_finish_group(const SirParams &p, uint32_t q, bool valid,
                                                 uint32_t t)
{
    int4 X = make_int4(0, 0, 0, 0), Y = make_int4(0, 0, 0, 0);
    uint32_t S0 = 0, inf0 = 0;
    if (valid) {
        X = load_nt4(p.x, q);
        Y = load_nt4(p.y, q);
        S0 = load_nt1(p.s, q);
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j)
            if (4 * q + j < p.n && ((S0 >> (8 * j)) & 0xffu) == ST_I) inf0 |= 1u << j;
        const uint32_t steps = p.t_last - t + 1;
        for (uint32_t k = 0; k < steps; ++k) sir_move4(p, q, t + k, X, Y);
    }
    const uint32_t inf = sir_recover_wave(p, q, inf0, t - 1, p.t_last);
    if (!valid) return;
    uint32_t S = S0;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
        if ((inf0 & ~inf) & (1u << j)) S = (S & ~(0xffu << (8 * j))) | ((uint32_t)ST_R << (8 * j));
    store_nt4(p.x, q, X);
    store_nt4(p.y, q, Y);
    if (S != S0) store_nt1(p.s, q, S);
}

// Gather-mode head (launch 0 of a call) and body (launch i >= 1) for the
// workgroup's agent groups, with demand-driven binning: q is the group of
// this thread, threads the number of agent threads of the run's launch (the
// stride of the demand-map clear), block the workgroup's index within the
// run.  Every thread of the workgroup must call them (they end with a
// workgroup barrier).
__device__ __forceinline__ void sir_head_demand(const SirParams &p, uint32_t q, uint32_t threads,
                                                uint32_t t, uint32_t block, uint32_t *s_wc)
{
    zero_quads((uint32_t *)p.dmap[2], p.dquads, q, threads);
    if (p.cside) zero_quads((uint32_t *)coarse_of(p, p.dmap[2]), coarse_quads(p), q, threads);
    // F_0 and F_1 are 0 unless a tiled segment of the call handed over
    const uint32_t mode = sir_demand_modes(p, 0) & 3u;
    uint32_t S = 0;
    if (q < p.groups) {
        int4 X = load_nt4(p.x, q);
        int4 Y = load_nt4(p.y, q);
        S = load_nt1(p.s, q);
        sir_move4(p, q, t, X, Y);
        store_nt4(p.x, q, X);
        store_nt4(p.y, q, Y);
        sir_bin_mark4(p, grid_of(p, t), q, t, S, X, Y, mode, p.dmap[0], p.dmap[1]);
    }
    sir_count_states(p, 0, q, S, q < p.groups, s_wc, block);
}

__device__ __forceinline__ void sir_body_demand(const SirParams &p, uint32_t q, uint32_t threads,
                                                uint32_t t, uint32_t i, uint32_t block,
                                                uint32_t *s_wc)
{
    const uint32_t mode = sir_demand_modes(p, i);
    if (mode & 4u) {                               // the same in every workgroup
        if (mode & 8u) return;
        // steps t .. t_last, then the tail's transition(t_last); no grid is read
        if (q == 0 && p.stop_word)                 // the host may stop enqueueing launches
            __hip_atomic_store(p.stop_word, p.stop_seq, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        sir_finish_group(p, q, q < p.groups, t);
        return;
    }
    zero_quads(grid_of(p, t + 1), p.quads, q, threads);
    zero_quads((uint32_t *)p.dmap[(i + 2) % 3], p.dquads, q, threads);
    if (p.cside)
        zero_quads((uint32_t *)coarse_of(p, p.dmap[(i + 2) % 3]), coarse_quads(p), q, threads);
    uint32_t S2 = 0;
    if (q < p.groups) {
        int4 X = load_nt4(p.x, q);
        int4 Y = load_nt4(p.y, q);
        const uint32_t S = load_nt1(p.s, q);
        S2 = sir_transition4<false>(p, grid_of(p, t - 1), q, t - 1, S, X, Y);
        sir_move4(p, q, t, X, Y);
        store_nt4(p.x, q, X);
        store_nt4(p.y, q, Y);
        if (S2 != S) store_nt1(p.s, q, S2);
        sir_bin_mark4(p, grid_of(p, t), q, t, S2, X, Y, mode, p.dmap[i % 3],
                      p.dmap[(i + 1) % 3]);
    }
    sir_count_states(p, i, q, S2, q < p.groups, s_wc, block);
}

// End of a call: the demand-binning counts and flags start the next call at
// zero (thread k of the run's first workgroup of a clear launch).
__device__ __forceinline__ void sir_demand_reset(const SirParams &p, uint32_t k, uint32_t threads)
{
    if (!p.nsi) return;
    for (uint32_t j = k; j < 4 * 2 * NSI_SLOTS; j += threads) p.nsi[j * NSI_STRIDE] = 0;
    if (k < 4) p.nsi[NSI_FLAGS + k] = 0;
}

// ------------------------------------------------------------------ SIR, exchange count mode
// Binning without global atomics.  The grid is cut into bands of xh rows
// (xP >= 3 bands).  The body kernel (256 threads, 1024 agents per workgroup)
// emits, for every agent infected at the start of step t, a record holding
// its post-move cell; a record on the first or last row of its band is also
// sent to the neighbouring band, which needs that row as a halo.  The records
// are counting-sorted by destination band in LDS and written to the
// workgroup's own segment (at most 3 per agent) with one (offset, count)
// word per band.  The count kernel (one workgroup per band) folds the records
// sent to its band into an LDS histogram of the band's rows plus one halo row
// on each side, and writes the band's rows of the box-summed grid K.  K is
// rewritten every step, so nothing has to be cleared between steps.

constexpr uint32_t XSEG = XSEG_WORDS;         // record slots per producer workgroup
constexpr uint32_t XCHUNK = 1024;            // sources per fold round in the count kernel

template <bool TRANSITION>
__device__ __forceinline__ void sir_exchange_produce(const SirParams &p, uint32_t wg, uint32_t t,
                                                     uint32_t *pcount, uint32_t *poff)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t q = wg * 256 + tid;
    const uint32_t P = p.xP, h = p.xh;
    for (uint32_t i = tid; i < P; i += 256) pcount[i] = 0;
    __syncthreads();
    uint32_t rc[12], rd[12], rr[12];
    uint32_t nrec = 0;
    if (q < p.groups) {
        int4 X = ((const int4 *)p.x)[q];
        int4 Y = ((const int4 *)p.y)[q];
        const uint32_t S = ((const uint32_t *)p.s)[q];
        uint32_t S2 = S;
        if (TRANSITION) S2 = sir_transition4<true>(p, kgrid_box(p), q, t - 1, S, X, Y);
        sir_move4(p, q, t, X, Y);
        ((int4 *)p.x)[q] = X;
        ((int4 *)p.y)[q] = Y;
        if (S2 != S) ((uint32_t *)p.s)[q] = S2;
        const int32_t xs[4] = {X.x, X.y, X.z, X.w};
        const int32_t ys[4] = {Y.x, Y.y, Y.z, Y.w};
        const uint32_t a = 4 * q;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (((S2 >> (8 * j)) & 0xffu) != ST_I || a + j >= p.n || !on_grid(xs[j], ys[j], p.L))
                continue;
            const uint32_t y = (uint32_t)ys[j];
            const uint32_t c = y * (uint32_t)p.L + (uint32_t)xs[j];
            const uint32_t d = y / h;
            const uint32_t first = d * h;
            const uint32_t last = min(first + h, (uint32_t)p.L) - 1;
            rc[nrec] = c;
            rd[nrec++] = d;
            if (y == first) {
                rc[nrec] = c;
                rd[nrec++] = d == 0 ? P - 1 : d - 1;
            }
            if (y == last) {
                rc[nrec] = c;
                rd[nrec++] = d + 1 == P ? 0 : d + 1;
            }
        }
    }
    for (uint32_t k = 0; k < nrec; ++k) rr[k] = atomicAdd(&pcount[rd[k]], 1u);
    __syncthreads();
    block_exclusive_scan<256, 8>(pcount, poff, P);
    uint32_t *rec = p.xrec + (size_t)wg * XSEG;
    for (uint32_t k = 0; k < nrec; ++k) rec[poff[rd[k]] + rr[k]] = rc[k];
    uint32_t *tab = p.xtab + (size_t)wg * P;
    for (uint32_t d = tid; d < P; d += 256) tab[d] = (poff[d] << 16) | pcount[d];
}

// Count kernel body for band b (256 threads).  hist holds (xh + 2) * L counters.
__device__ __forceinline__ void sir_exchange_count(const SirParams &p, uint32_t b, uint32_t *hist,
                                                   uint32_t *scnt, uint32_t *soff, uint32_t *sraw)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t L = (uint32_t)p.L, h = p.xh, P = p.xP, W = p.xW;
    const uint32_t y0 = b * h;
    const uint32_t hb = min(h, L - y0);               // rows of this band
    const uint32_t top = (y0 + L - 1) % L;            // halo row above the band
    const uint32_t slots = (hb + 2) * L;
    for (uint32_t i = tid; i < slots; i += 256) hist[i] = 0;
    for (uint32_t w0 = 0; w0 < W; w0 += XCHUNK) {
        const uint32_t nsrc = min(XCHUNK, W - w0);
        __syncthreads();                              // previous round done with scnt/soff/sraw
        for (uint32_t i = tid; i < nsrc; i += 256) {
            const uint32_t e = p.xtab[(size_t)(w0 + i) * P + b];
            sraw[i] = e;
            scnt[i] = e & 0xffffu;
        }
        __syncthreads();
        block_exclusive_scan<256, 4>(scnt, soff, nsrc);
        const uint32_t total = soff[nsrc - 1] + (sraw[nsrc - 1] & 0xffffu);
        for (uint32_t i = tid; i < total; i += 256) {
            uint32_t lo = 0, hi = nsrc;               // last source with soff[s] <= i
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (soff[mid] <= i) lo = mid;
                else hi = mid;
            }
            const uint32_t c = p.xrec[(size_t)(w0 + lo) * XSEG + (sraw[lo] >> 16) + (i - soff[lo])];
            const uint32_t y = c / L, x = c - y * L;
            const uint32_t r = (y + L - top) % L;     // slot row, < hb + 2 by construction
            if (r < hb + 2) atomicAdd(&hist[r * L + x], 1u);
        }
    }
    __syncthreads();
    uint32_t *K = kgrid_box(p) + (size_t)y0 * L;
    for (uint32_t i = tid; i < hb * L; i += 256) {
        const uint32_t j = i / L + 1, x = i - (j - 1) * L;
        const uint32_t xm = x == 0 ? L - 1 : x - 1;
        const uint32_t xp = x + 1 == L ? 0 : x + 1;
        uint32_t k = 0;
#pragma unroll
        for (uint32_t rr = 0; rr < 3; ++rr) {
            const uint32_t *row = hist + (j - 1 + rr) * L;
            k += row[xm] + row[x] + row[xp];
        }
        K[i] = k;
    }
}

// box(t) for cells 4i..4i+3: K = 3x3 torus box sum of C_t (each distinct
// cell once), written as one 16-byte store; cells past L*L (grid padding)
// get 0.
__device__ __forceinline__ void sir_box_quad(const SirParams &p, const uint32_t *__restrict__ C,
                                             uint32_t *__restrict__ K, uint32_t i)
{
    const uint32_t cells = (uint32_t)p.L * (uint32_t)p.L;
    uint32_t v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t c = 4 * i + j;
        v[j] = c < cells ? block_count(C, p.L, (int32_t)(c % (uint32_t)p.L),
                                       (int32_t)(c / (uint32_t)p.L))
                         : 0u;
    }
    ((uint4 *)K)[i] = make_uint4(v[0], v[1], v[2], v[3]);
}

}  // namespace amber
