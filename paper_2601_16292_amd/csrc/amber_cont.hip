// amber_cont.hip -- the paper's continuous-space benchmark models (Sec. 5.1.2)
// in a W x W world with float32 coordinates.
//
//   walk  x <- min(max(x + dx, 0), W), y likewise; dx, dy uniform on [-1, 1)
//         from the agent's two STEP words of the step (2 words per agent, so
//         one Philox block serves two agents).
//   SIR   the walk's move, then each susceptible agent counts the agents
//         infected at the start of the step within distance r of its new
//         position, (xa - xb)^2 + (ya - yb)^2 <= r^2 in float32 with one
//         rounding per operation, and becomes infected with probability
//         1 - (1 - p)^k (exact uint32 thresholds); infected agents count days
//         and recover after `recover` of them.
//
// The paper's contact search is an all-pairs test.  Here the infected
// agents of a step are counting-sorted into a cell list of side r (cell
// coordinate floor(x / r) evaluated in double precision, which is the exact
// floor of the real quotient), so every infected agent within distance r of
// an agent lies in the 3 x 3 cells around it, and only those are tested.
// The count k is a sum, independent of the order of the list, so the result
// equals the all-pairs definition bit for bit.
//
// Every float operation of the model is written with the round-to-nearest
// intrinsics, so the compiler fuses none of them.
#include "amber_device_common.h"

namespace amber {
namespace {

__device__ __forceinline__ float unit_delta(uint32_t u)
{
    return __fsub_rn(__fmul_rn((float)(u >> 8), 0x1p-23f), 1.0f);
}

__device__ __forceinline__ float clamp_w(float v, float W)
{
    return v < 0.0f ? 0.0f : (v > W ? W : v);
}

__device__ __forceinline__ uint32_t cell_axis(float v, float r, uint32_t nc)
{
    const double q = floor((double)v / (double)r);
    const uint32_t c = q < 0.0 ? 0u : (uint32_t)q;
    return c < nc ? c : nc - 1;
}

// Agents 2q and 2q + 1 share one Philox block (two words per agent): words
// 0, 1 are agent 2q's pair and words 2, 3 agent 2q + 1's.  Init uses the
// INIT_POS block (q, 0, 0, 0), a step t the STEP block (q, t, 5, 0).
__global__ __launch_bounds__(256) void k_cont_init(float *__restrict__ x, float *__restrict__ y,
                                                   uint32_t n, float W, uint32_t k0, uint32_t k1)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t a = 2 * q;
    if (a >= n) return;
    const uint4 r = philox(q, 0, P_INIT_POS, k0, k1);
    x[a] = __fmul_rn(__fmul_rn((float)(r.x >> 8), 0x1p-24f), W);
    y[a] = __fmul_rn(__fmul_rn((float)(r.y >> 8), 0x1p-24f), W);
    if (a + 1 < n) {
        x[a + 1] = __fmul_rn(__fmul_rn((float)(r.z >> 8), 0x1p-24f), W);
        y[a + 1] = __fmul_rn(__fmul_rn((float)(r.w >> 8), 0x1p-24f), W);
    }
}

__global__ __launch_bounds__(256) void k_cont_states(uint8_t *__restrict__ s,
                                                     uint8_t *__restrict__ days, uint32_t n,
                                                     uint32_t i0)
{
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    s[a] = a < i0 ? (uint8_t)ST_I : (uint8_t)ST_S;
    days[a] = 0;
}

__global__ __launch_bounds__(256) void k_cont_walk(float *__restrict__ x, float *__restrict__ y,
                                                   uint32_t n, float W, uint32_t k0, uint32_t k1,
                                                   uint32_t t0, uint32_t n_steps)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t a = 2 * q;
    if (a >= n) return;
    const bool two = a + 1 < n;
    float x0 = x[a], y0 = y[a], x1 = two ? x[a + 1] : 0.0f, y1 = two ? y[a + 1] : 0.0f;
    for (uint32_t i = 0; i < n_steps; ++i) {
        const uint4 r = philox(q, t0 + i, P_STEP, k0, k1);
        x0 = clamp_w(__fadd_rn(x0, unit_delta(r.x)), W);
        y0 = clamp_w(__fadd_rn(y0, unit_delta(r.y)), W);
        x1 = clamp_w(__fadd_rn(x1, unit_delta(r.z)), W);
        y1 = clamp_w(__fadd_rn(y1, unit_delta(r.w)), W);
    }
    x[a] = x0;
    y[a] = y0;
    if (two) {
        x[a + 1] = x1;
        y[a + 1] = y1;
    }
}

struct ContSir {
    float *x, *y;
    uint8_t *s, *days;
    uint32_t n, nc, k0, k1, table_len, recover;
    float W, r;
    const uint32_t *t_inf;
    uint32_t *cnt;        // nc * nc + 1 cell counts, then offsets
    uint32_t *cursor;     // nc * nc placement cursors
    float2 *list;         // infected positions sorted by cell
};

// Move every agent; count the agents infected at the start of the step by
// their new cell.
__global__ __launch_bounds__(256) void k_cont_sir_move(ContSir c, uint32_t t)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t a = 2 * q;
    if (a >= c.n) return;
    const uint4 r = philox(q, t, P_STEP, c.k0, c.k1);
    const uint32_t dw[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (uint32_t j = 0; j < 2; ++j) {
        const uint32_t b = a + j;
        if (b >= c.n) break;
        const float nx = clamp_w(__fadd_rn(c.x[b], unit_delta(dw[2 * j])), c.W);
        const float ny = clamp_w(__fadd_rn(c.y[b], unit_delta(dw[2 * j + 1])), c.W);
        c.x[b] = nx;
        c.y[b] = ny;
        if (c.s[b] == ST_I)
            atomicAdd(&c.cnt[cell_axis(ny, c.r, c.nc) * c.nc + cell_axis(nx, c.r, c.nc)], 1u);
    }
}

// Exclusive scan of the cell counts (one workgroup), and the cursors.
__global__ __launch_bounds__(1024) void k_cont_scan(uint32_t *__restrict__ cnt,
                                                    uint32_t *__restrict__ cursor, uint32_t cells)
{
    __shared__ uint32_t part[1024];
    const uint32_t per = (cells + blockDim.x - 1) / blockDim.x;
    const uint32_t lo = threadIdx.x * per;
    const uint32_t hi = lo + per < cells ? lo + per : cells;
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; ++i) s += cnt[i];
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
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t v = cnt[i];
        cnt[i] = run;
        cursor[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(256) void k_cont_place(ContSir c)
{
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= c.n || c.s[a] != ST_I) return;
    const float px = c.x[a], py = c.y[a];
    const uint32_t cell = cell_axis(py, c.r, c.nc) * c.nc + cell_axis(px, c.r, c.nc);
    c.list[atomicAdd(&c.cursor[cell], 1u)] = make_float2(px, py);
}

// Contacts and transitions of step t; four agents per thread share one EPI
// block.  Offsets: the scan left cnt[cell] = start of the cell's run, and
// the placement moved each cursor to the run's end.
__global__ __launch_bounds__(256) void k_cont_sir_transition(ContSir c, uint32_t t)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t a0 = 4 * q;
    if (a0 >= c.n) return;
    const float r2 = __fmul_rn(c.r, c.r);
    uint32_t st[4], k[4] = {0, 0, 0, 0};
    bool need = false;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t a = a0 + j;
        st[j] = a < c.n ? c.s[a] : (uint32_t)ST_R;
        if (st[j] == ST_I) need = true;
        if (st[j] != ST_S) continue;
        const float px = c.x[a], py = c.y[a];
        const uint32_t cx = cell_axis(px, c.r, c.nc), cy = cell_axis(py, c.r, c.nc);
        for (uint32_t yy = cy ? cy - 1 : 0; yy <= cy + 1 && yy < c.nc; ++yy) {
            for (uint32_t xx = cx ? cx - 1 : 0; xx <= cx + 1 && xx < c.nc; ++xx) {
                const uint32_t cell = yy * c.nc + xx;
                const uint32_t e1 = c.cursor[cell];
                for (uint32_t e = c.cnt[cell]; e < e1; ++e) {
                    const float2 b = c.list[e];
                    const float dx = __fsub_rn(px, b.x), dy = __fsub_rn(py, b.y);
                    k[j] += __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)) <= r2;
                }
            }
        }
        need |= k[j] >= 1;
    }
    if (!need) return;
    const uint4 r = philox(q, t, P_EPI, c.k0, c.k1);
    const uint32_t u[4] = {r.x, r.y, r.z, r.w};
    const uint32_t last = c.table_len - 1;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t a = a0 + j;
        if (a >= c.n) break;
        if (st[j] == ST_S && k[j] >= 1) {
            if (u[j] < c.t_inf[k[j] < last ? k[j] : last]) {
                c.s[a] = ST_I;
                c.days[a] = 0;
            }
        } else if (st[j] == ST_I) {
            const uint32_t d = c.days[a] + 1u;
            c.days[a] = (uint8_t)d;
            if (d >= c.recover) c.s[a] = ST_R;
        }
    }
}

// Up to 240 words per launch travel in the kernel arguments (no host buffer
// has to outlive the call).
struct Words240 {
    uint32_t w[240];
};
__global__ void k_put_words(uint32_t *__restrict__ dst, Words240 src, uint32_t count)
{
    const uint32_t i = threadIdx.x;
    if (i < count) dst[i] = src.w[i];
}

__global__ __launch_bounds__(256) void k_cont_clear(uint32_t *__restrict__ p, uint32_t count)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

uint64_t a16(uint64_t v) { return (v + 15) & ~15ull; }

}  // namespace

uint64_t cont_sir_workspace(uint32_t n, uint32_t nc, uint32_t table_len)
{
    const uint64_t cells = (uint64_t)nc * nc;
    return a16(4 * (cells + 1)) + a16(4 * cells) + a16(8ull * n) + a16(4ull * table_len);
}

hipError_t launch_cont_init(float *x, float *y, uint32_t n, float W, uint32_t k0, uint32_t k1,
                            hipStream_t st)
{
    const uint32_t pairs = (n + 1) / 2;
    hipLaunchKernelGGL(k_cont_init, dim3((pairs + 255) / 256), dim3(256), 0, st, x, y, n, W, k0, k1);
    return hipGetLastError();
}

hipError_t launch_cont_states(uint8_t *s, uint8_t *days, uint32_t n, uint32_t i0, hipStream_t st)
{
    hipLaunchKernelGGL(k_cont_states, dim3((n + 255) / 256), dim3(256), 0, st, s, days, n, i0);
    return hipGetLastError();
}

hipError_t launch_cont_walk(float *x, float *y, uint32_t n, float W, uint32_t k0, uint32_t k1,
                            uint32_t t0, uint32_t n_steps, hipStream_t st)
{
    const uint32_t pairs = (n + 1) / 2;
    hipLaunchKernelGGL(k_cont_walk, dim3((pairs + 255) / 256), dim3(256), 0, st, x, y, n, W, k0,
                       k1, t0, n_steps);
    return hipGetLastError();
}

hipError_t launch_cont_sir(float *x, float *y, uint8_t *s, uint8_t *days, uint32_t n, float W,
                           float r, uint32_t nc, uint32_t k0, uint32_t k1, const uint32_t *table,
                           uint32_t table_len, uint32_t recover, uint32_t t0, uint32_t n_steps,
                           void *ws, hipStream_t st)
{
    const uint64_t cells = (uint64_t)nc * nc;
    uint8_t *b = (uint8_t *)ws;
    ContSir c;
    c.x = x;
    c.y = y;
    c.s = s;
    c.days = days;
    c.n = n;
    c.nc = nc;
    c.k0 = k0;
    c.k1 = k1;
    c.table_len = table_len;
    c.recover = recover;
    c.W = W;
    c.r = r;
    c.cnt = (uint32_t *)b;
    c.cursor = (uint32_t *)(b + a16(4 * (cells + 1)));
    c.list = (float2 *)(b + a16(4 * (cells + 1)) + a16(4 * cells));
    uint32_t *tab = (uint32_t *)(b + a16(4 * (cells + 1)) + a16(4 * cells) + a16(8ull * n));
    c.t_inf = tab;
    for (uint32_t i = 0; i < table_len; i += 240) {
        Words240 w;
        const uint32_t cnt = table_len - i < 240 ? table_len - i : 240;
        for (uint32_t j = 0; j < cnt; ++j) w.w[j] = table[i + j];
        hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, st, tab + i, w, cnt);
    }
    const uint32_t pairs = (n + 1) / 2, quads = (n + 3) / 4;
    for (uint32_t i = 0; i < n_steps; ++i) {
        const uint32_t t = t0 + i;
        hipLaunchKernelGGL(k_cont_clear, dim3((uint32_t)((cells + 256) / 256)), dim3(256), 0, st,
                           c.cnt, (uint32_t)(cells + 1));
        hipLaunchKernelGGL(k_cont_sir_move, dim3((pairs + 255) / 256), dim3(256), 0, st, c, t);
        hipLaunchKernelGGL(k_cont_scan, dim3(1), dim3(1024), 0, st, c.cnt, c.cursor,
                           (uint32_t)cells);
        hipLaunchKernelGGL(k_cont_place, dim3((n + 255) / 256), dim3(256), 0, st, c);
        hipLaunchKernelGGL(k_cont_sir_transition, dim3((quads + 255) / 256), dim3(256), 0, st, c, t);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace amber
