// amber_views.hip -- the view primitives on arbitrary int32 / float32 columns.
//
// The three views of the method's view API (Sec. 3.3), as the listings of
// Sec. 3.1.1 use them:
//   full view      every row:                 v <- a*v + b
//   filtered view  rows where p CMP thr:      v <- a*v + b (p read before
//                  the update, as one snapshot)
//   scatter view   for j in list order:       col[ids[j]] += vals[j]
//                  (duplicate ids accumulate; ids outside the column skipped)
// int32 arithmetic wraps modulo 2^32, so every order of the scatter's
// integer additions gives the same column and one atomic add per entry is
// exact.  float32 updates are one fused multiply-add; float32 scatter adds
// round after every addition in list order, so the entries are first put in
// order of (id, position in the list) by a stable LSD radix sort on the id,
// and each id's run of entries is then added in that order by one thread.
//
// Column accesses are streamed and coalesced: four consecutive rows per
// thread, as one 16-byte access per column when the pointers allow it.
#include <type_traits>

#include "amber_device_common.h"

namespace amber {
namespace {

enum : uint32_t { CMP_LT = 0, CMP_LE, CMP_EQ, CMP_NE, CMP_GE, CMP_GT };

template <typename P>
__device__ __forceinline__ bool compare(P v, uint32_t cmp, P thr)
{
    switch (cmp) {
    case CMP_LT: return v < thr;
    case CMP_LE: return v <= thr;
    case CMP_EQ: return v == thr;
    case CMP_NE: return v != thr;
    case CMP_GE: return v >= thr;
    default: return v > thr;
    }
}

__device__ __forceinline__ int32_t affine(int32_t v, int32_t a, int32_t b)
{
    return (int32_t)((uint32_t)a * (uint32_t)v + (uint32_t)b);
}

__device__ __forceinline__ float affine(float v, float a, float b)
{
    return __builtin_fmaf(a, v, b);
}

// One thread per four consecutive rows; VEC: 16-byte accesses (pointers
// 16-byte aligned), else four scalar accesses.  pred NULL: full view.
template <typename T, typename P, bool VEC>
__global__ __launch_bounds__(256) void k_view_update(T *__restrict__ col, uint64_t n, T a, T b,
                                                     const P *__restrict__ pred, uint32_t cmp,
                                                     P thr)
{
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t r0 = 4 * q;
    if (r0 >= n) return;
    if (VEC && r0 + 4 <= n) {
        using V = typename std::conditional<std::is_same<T, float>::value, float4, int4>::type;
        V v = reinterpret_cast<V *>(col)[q];
        bool take[4] = {true, true, true, true};
        if (pred) {
            using W = typename std::conditional<std::is_same<P, float>::value, float4, int4>::type;
            const W p = reinterpret_cast<const W *>(pred)[q];
            take[0] = compare<P>(p.x, cmp, thr);
            take[1] = compare<P>(p.y, cmp, thr);
            take[2] = compare<P>(p.z, cmp, thr);
            take[3] = compare<P>(p.w, cmp, thr);
        }
        if (take[0]) v.x = affine(v.x, a, b);
        if (take[1]) v.y = affine(v.y, a, b);
        if (take[2]) v.z = affine(v.z, a, b);
        if (take[3]) v.w = affine(v.w, a, b);
        reinterpret_cast<V *>(col)[q] = v;
        return;
    }
    const uint64_t r1 = r0 + 4 < n ? r0 + 4 : n;
    for (uint64_t r = r0; r < r1; ++r) {
        if (pred && !compare<P>(pred[r], cmp, thr)) continue;
        col[r] = affine(col[r], a, b);
    }
}

__global__ __launch_bounds__(256) void k_scatter_add_i32(int32_t *__restrict__ col, uint64_t n,
                                                         const uint32_t *__restrict__ ids,
                                                         const int32_t *__restrict__ vals,
                                                         int32_t scalar, uint64_t m)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
        const uint32_t id = ids[j];
        if (id < n) atomicAdd(col + id, vals ? vals[j] : scalar);
    }
}

// ---------------------------------------------------------------- radix sort

constexpr uint32_t RS_THREADS = 256;
constexpr uint32_t RS_PER_THREAD = 8;
constexpr uint32_t RS_TILE = RS_THREADS * RS_PER_THREAD;   // entries per block
constexpr uint32_t RS_BITS = 4;
constexpr uint32_t RS_DIGITS = 1u << RS_BITS;

// Key of entry j before the first pass: its id, or n for an id outside the
// column (those sort last and are skipped).
__device__ __forceinline__ uint32_t first_key(const uint32_t *ids, uint64_t j, uint64_t n)
{
    const uint32_t id = ids[j];
    return id < n ? id : (uint32_t)n;
}

// Digit counts of one tile of entries: hist[d * blocks + b].
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t *__restrict__ keys_in,
                                                         const uint32_t *__restrict__ ids,
                                                         uint64_t n, uint64_t m, uint32_t shift,
                                                         uint32_t *__restrict__ hist)
{
    __shared__ uint32_t cnt[RS_DIGITS];
    if (threadIdx.x < RS_DIGITS) cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    for (uint32_t k = threadIdx.x; k < RS_TILE; k += RS_THREADS) {
        const uint64_t j = base + k;
        if (j >= m) break;
        const uint32_t key = keys_in ? keys_in[j] : first_key(ids, j, n);
        atomicAdd(&cnt[(key >> shift) & (RS_DIGITS - 1)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < RS_DIGITS) hist[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan, in place, of `count` words in digit-major order (one
// workgroup; each thread scans a contiguous chunk, then the chunk sums).
__global__ __launch_bounds__(1024) void k_rs_scan(uint32_t *__restrict__ hist, uint64_t count)
{
    __shared__ uint32_t part[1024];
    const uint64_t per = (count + blockDim.x - 1) / blockDim.x;
    const uint64_t lo = threadIdx.x * per;
    const uint64_t hi = lo + per < count ? lo + per : count;
    uint32_t s = 0;
    for (uint64_t i = lo; i < hi; ++i) s += hist[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t t = 0; t < blockDim.x; ++t) {
            const uint32_t v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (uint64_t i = lo; i < hi; ++i) {
        const uint32_t v = hist[i];
        hist[i] = run;
        run += v;
    }
}

// The digit counts of a big sort are scanned in three launches: the sum of
// every 4096-word tile, a one-workgroup scan of those sums, then each tile's
// own scan plus its tile's offset.
constexpr uint32_t SCAN_TILE = 4096;

__global__ __launch_bounds__(1024) void k_scan_tile_sums(const uint32_t *__restrict__ d,
                                                         uint64_t count, uint32_t *__restrict__ sums)
{
    __shared__ uint32_t red[16];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
    for (uint32_t i = threadIdx.x; i < SCAN_TILE; i += 1024)
        if (base + i < count) s += d[base + i];
    for (uint32_t off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63u) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t w = 0; w < 16; ++w) t += red[w];
        sums[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_scan_tiles(uint32_t *__restrict__ d, uint64_t count,
                                                     const uint32_t *__restrict__ offs)
{
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    const uint32_t n = (uint32_t)(count - base < SCAN_TILE ? count - base : SCAN_TILE);
    block_exclusive_scan<1024, SCAN_TILE / 1024>(d + base, d + base, n);
    const uint32_t add = offs[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < n; i += 1024) d[base + i] += add;
}

// Stable scatter of one tile by one digit.  Thread t holds the tile's
// entries t*8 .. t*8+7 in list order; an entry's destination is the digit's
// global offset for this tile, plus the entries of that digit held by
// earlier threads, plus those earlier in its own eight.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint32_t *__restrict__ keys_in,
                                                            const uint32_t *__restrict__ pos_in,
                                                            const uint32_t *__restrict__ ids,
                                                            uint64_t n, uint64_t m, uint32_t shift,
                                                            const uint32_t *__restrict__ offs,
                                                            uint32_t *__restrict__ keys_out,
                                                            uint32_t *__restrict__ pos_out)
{
    __shared__ uint32_t cnt[RS_DIGITS][RS_THREADS];
    __shared__ uint32_t seg[RS_DIGITS][16];
    __shared__ uint32_t goff[RS_DIGITS];
    const uint32_t t = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x * RS_TILE + (uint64_t)t * RS_PER_THREAD;
    uint32_t key[RS_PER_THREAD], pos[RS_PER_THREAD];
    uint32_t c[RS_DIGITS];
#pragma unroll
    for (uint32_t d = 0; d < RS_DIGITS; ++d) c[d] = 0;
#pragma unroll
    for (uint32_t k = 0; k < RS_PER_THREAD; ++k) {
        const uint64_t j = base + k;
        key[k] = 0xffffffffu;
        pos[k] = 0;
        if (j < m) {
            key[k] = keys_in ? keys_in[j] : first_key(ids, j, n);
            pos[k] = pos_in ? pos_in[j] : (uint32_t)j;
            const uint32_t d = (key[k] >> shift) & (RS_DIGITS - 1);
#pragma unroll
            for (uint32_t e = 0; e < RS_DIGITS; ++e) c[e] += (e == d);
        }
    }
    if (t < RS_DIGITS) goff[t] = offs[(uint64_t)t * gridDim.x + blockIdx.x];
#pragma unroll
    for (uint32_t d = 0; d < RS_DIGITS; ++d) cnt[d][t] = c[d];
    __syncthreads();
    // exclusive prefix of each digit's row over the threads: thread t scans
    // 16 entries of row t/16, then the row's 16 segment sums are scanned
    const uint32_t row = t >> 4, s0 = (t & 15) * 16;
    uint32_t run = 0;
    for (uint32_t i = 0; i < 16; ++i) {
        const uint32_t v = cnt[row][s0 + i];
        cnt[row][s0 + i] = run;
        run += v;
    }
    seg[row][t & 15] = run;
    __syncthreads();
    if (t < RS_DIGITS) {
        uint32_t r = 0;
        for (uint32_t i = 0; i < 16; ++i) {
            const uint32_t v = seg[t][i];
            seg[t][i] = r;
            r += v;
        }
    }
    __syncthreads();
    for (uint32_t i = 0; i < 16; ++i) cnt[row][s0 + i] += seg[row][t & 15];
    __syncthreads();
#pragma unroll
    for (uint32_t d = 0; d < RS_DIGITS; ++d) c[d] = 0;
#pragma unroll
    for (uint32_t k = 0; k < RS_PER_THREAD; ++k) {
        if (base + k >= m) break;
        const uint32_t d = (key[k] >> shift) & (RS_DIGITS - 1);
        uint32_t before = 0;
#pragma unroll
        for (uint32_t e = 0; e < RS_DIGITS; ++e) before += (e == d) ? c[e] : 0u;
        const uint32_t dest = goff[d] + cnt[d][t] + before;
        keys_out[dest] = key[k];
        pos_out[dest] = pos[k];
#pragma unroll
        for (uint32_t e = 0; e < RS_DIGITS; ++e) c[e] += (e == d);
    }
}

// After the sort: the first entry of each id's run adds the run's values to
// the column, one after the other in list order, with float32 rounding.
__global__ __launch_bounds__(256) void k_segment_add_f32(float *__restrict__ col, uint64_t n,
                                                         const uint32_t *__restrict__ keys,
                                                         const uint32_t *__restrict__ pos,
                                                         const float *__restrict__ vals,
                                                         float scalar, uint64_t m)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += stride) {
        const uint32_t id = keys[k];
        if (id >= n || (k > 0 && keys[k - 1] == id)) continue;
        float v = col[id];
        for (uint64_t e = k; e < m && keys[e] == id; ++e) v = v + (vals ? vals[pos[e]] : scalar);
        col[id] = v;
    }
}

// After the sort: the last entry of each id's run (the latest in the log)
// writes its value.
__global__ __launch_bounds__(256) void k_write_last(uint32_t *__restrict__ col, uint64_t n,
                                                    const uint32_t *__restrict__ keys,
                                                    const uint32_t *__restrict__ pos,
                                                    const uint32_t *__restrict__ vals, uint64_t m)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += stride) {
        const uint32_t id = keys[k];
        if (id < n && (k + 1 == m || keys[k + 1] != id)) col[id] = vals[pos[k]];
    }
}

uint32_t launch_grid(uint64_t items, uint32_t block, uint32_t cap)
{
    const uint64_t g = (items + block - 1) / block;
    return (uint32_t)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

// Radix-sort workspace: two generations of keys and positions (4 words per
// entry) plus the digit counts of every tile.
uint64_t view_scatter_f32_workspace(uint64_t m)
{
    const uint64_t blocks = (m + RS_TILE - 1) / RS_TILE;
    const uint64_t counts = RS_DIGITS * (blocks ? blocks : 1);
    return 16 * m + 4 * counts + 4 * ((counts + SCAN_TILE - 1) / SCAN_TILE) + 256;
}

namespace {
template <typename T, typename P>
void view_launch(bool vec, uint64_t n, hipStream_t st, void *col, T a, T b, const void *pred,
                 uint32_t cmp, P thr)
{
    const dim3 grid((unsigned)((n + 4 * 256 - 1) / (4 * 256))), blk(256);
    if (vec)
        hipLaunchKernelGGL((k_view_update<T, P, true>), grid, blk, 0, st, (T *)col, n, a, b,
                           (const P *)pred, cmp, thr);
    else
        hipLaunchKernelGGL((k_view_update<T, P, false>), grid, blk, 0, st, (T *)col, n, a, b,
                           (const P *)pred, cmp, thr);
}
}  // namespace

hipError_t launch_view_update(void *col, uint32_t dtype, uint64_t n, ViewValue a, ViewValue b,
                              const void *pred, uint32_t pred_dtype, uint32_t cmp, ViewValue thr,
                              hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const bool vec = ((uintptr_t)col & 15u) == 0 && ((uintptr_t)pred & 15u) == 0;
    const bool pf = pred && pred_dtype == VIEW_F32;
    if (dtype == VIEW_I32) {
        if (pf) view_launch<int32_t, float>(vec, n, st, col, a.i, b.i, pred, cmp, thr.f);
        else view_launch<int32_t, int32_t>(vec, n, st, col, a.i, b.i, pred, cmp, thr.i);
    } else {
        if (pf) view_launch<float, float>(vec, n, st, col, a.f, b.f, pred, cmp, thr.f);
        else view_launch<float, int32_t>(vec, n, st, col, a.f, b.f, pred, cmp, thr.i);
    }
    return hipGetLastError();
}

hipError_t radix_sort_ids(const uint32_t *ids, uint64_t n, uint64_t m, void *ws, hipStream_t st,
                          const uint32_t **keys_out, const uint32_t **pos_out)
{
    const uint32_t blocks = (uint32_t)((m + RS_TILE - 1) / RS_TILE);
    uint32_t *keys[2] = {(uint32_t *)ws, (uint32_t *)ws + m};
    uint32_t *pos[2] = {(uint32_t *)ws + 2 * m, (uint32_t *)ws + 3 * m};
    uint32_t *hist = (uint32_t *)ws + 4 * m;
    uint32_t *tile_sums = hist + (uint64_t)RS_DIGITS * blocks;
    uint32_t bits = 1;                                   // keys lie in [0, n]
    while (bits < 32 && (n >> bits) != 0) ++bits;
    const uint32_t passes = (bits + RS_BITS - 1) / RS_BITS;
    for (uint32_t p = 0; p < passes; ++p) {
        const uint32_t shift = p * RS_BITS;
        const uint32_t *kin = p ? keys[(p - 1) & 1] : nullptr;
        const uint32_t *pin = p ? pos[(p - 1) & 1] : nullptr;
        hipLaunchKernelGGL(k_rs_hist, dim3(blocks), dim3(RS_THREADS), 0, st, kin, ids, n, m, shift,
                           hist);
        const uint64_t counts = (uint64_t)RS_DIGITS * blocks;
        if (counts <= SCAN_TILE) {
            hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(1024), 0, st, hist, counts);
        } else {
            const uint32_t tiles = (uint32_t)((counts + SCAN_TILE - 1) / SCAN_TILE);
            hipLaunchKernelGGL(k_scan_tile_sums, dim3(tiles), dim3(1024), 0, st, hist, counts,
                               tile_sums);
            hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(1024), 0, st, tile_sums, (uint64_t)tiles);
            hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(1024), 0, st, hist, counts,
                               tile_sums);
        }
        hipLaunchKernelGGL(k_rs_scatter, dim3(blocks), dim3(RS_THREADS), 0, st, kin, pin, ids, n, m,
                           shift, hist, keys[p & 1], pos[p & 1]);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    *keys_out = keys[(passes - 1) & 1];
    *pos_out = pos[(passes - 1) & 1];
    return hipSuccess;
}

hipError_t launch_view_scatter_add(void *col, uint32_t dtype, uint64_t n, const uint32_t *ids,
                                   uint64_t m, const void *vals, ViewValue scalar, void *ws,
                                   hipStream_t st)
{
    if (m == 0) return hipSuccess;
    if (dtype == VIEW_I32) {
        hipLaunchKernelGGL(k_scatter_add_i32, dim3(launch_grid(m, 256, 8192)), dim3(256), 0, st,
                           (int32_t *)col, n, ids, (const int32_t *)vals, scalar.i, m);
        return hipGetLastError();
    }
    const uint32_t *keys = nullptr, *pos = nullptr;
    const hipError_t e = radix_sort_ids(ids, n, m, ws, st, &keys, &pos);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_segment_add_f32, dim3(launch_grid(m, 256, 8192)), dim3(256), 0, st,
                       (float *)col, n, keys, pos, (const float *)vals, scalar.f, m);
    return hipGetLastError();
}

hipError_t launch_view_write_log(uint32_t *col, uint64_t n, const uint32_t *ids, uint64_t m,
                                 const uint32_t *vals, void *ws, hipStream_t st)
{
    if (m == 0) return hipSuccess;
    const uint32_t *keys = nullptr, *pos = nullptr;
    const hipError_t e = radix_sort_ids(ids, n, m, ws, st, &keys, &pos);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_write_last, dim3(launch_grid(m, 256, 8192)), dim3(256), 0, st, col, n,
                       keys, pos, vals, m);
    return hipGetLastError();
}

}  // namespace amber
