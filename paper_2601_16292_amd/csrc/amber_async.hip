// amber_async.hip -- wealth transfer under asynchronous (sequential) update
// semantics (Sec. 3.4): within step t the agents act one at a time, in the
// order of their ORDER words (ties by id), and each sees the wealth the
// agents before it left.
//
// The order only decides who gives.  An agent gives iff its wealth is
// positive at its turn; an agent loses wealth only at its own turn, so its
// wealth then is its start-of-step wealth plus the units it received from
// donors acting before it.  The donor set D is therefore the least set with
//     D = {a : w_a > 0}  U  {a : some b in D acts before a and draws a},
// and every donor gives one unit to its (synchronous-model) recipient.  D is
// built by a fixed point on the GPU: generation 1 is the agents with
// positive wealth, and generation g + 1 the agents first reached by a donor
// of generation g that acts before them.  Once D is known the step is the
// synchronous scatter of the wealth model with D as the donors:
//     w'_a = w_a - [a in D] + #{b in D : recipient(b) = a},
// integer sums that any order of atomic adds gives exactly.  The result
// equals the one-agent-at-a-time loop of the definition.
//
// Per step: ORDER words and recipients for every agent (one Philox block
// per four agents for ORDER, one per two agents for RECIPIENT), a stable
// radix sort of the ORDER words into the acting order and each agent's
// rank in it, the generations (each a pass over the agents that returns at
// once when the previous generation added no one), then the scatter.
#include "amber_device_common.h"

namespace amber {
namespace {

constexpr uint32_t ASYNC_MAX_GEN = 64;   // generations launched per step
constexpr uint32_t ADDED_WORDS = 68;     // ASYNC_MAX_GEN + 2 flags, a multiple of 4 words

struct AsyncWs {
    uint32_t *key;      // ORDER word of each agent (the sort's input)
    uint32_t *recip;    // recipient of each agent
    uint32_t *rank;     // position in the acting order
    uint32_t *gen;      // donor generation (0 = not a donor)
    uint32_t *added;    // added[g] != 0: generation g has members (g <= ASYNC_MAX_GEN + 1);
                        // cleared before each step
    void *sort;         // radix-sort workspace
};

__global__ __launch_bounds__(256) void k_async_prep(const int32_t *__restrict__ w, uint32_t n,
                                                    uint32_t t, uint32_t k0, uint32_t k1,
                                                    AsyncWs ws)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;     // agents 4q .. 4q + 3
    const uint32_t a0 = 4 * q;
    if (a0 >= n) return;
    const uint4 o = philox(q, t, P_ORDER, k0, k1);
    const uint4 r0 = philox(2 * q, t, P_RECIPIENT, k0, k1);
    const uint4 r1 = philox(2 * q + 1, t, P_RECIPIENT, k0, k1);
    const uint32_t ow[4] = {o.x, o.y, o.z, o.w};
    const uint32_t rc[4] = {recipient(r0.x, r0.y, n), recipient(r0.z, r0.w, n),
                            recipient(r1.x, r1.y, n), recipient(r1.z, r1.w, n)};
    bool any = false;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t a = a0 + j;
        if (a >= n) break;
        ws.key[a] = ow[j];
        ws.recip[a] = rc[j];
        const bool d = w[a] > 0;
        ws.gen[a] = d ? 1u : 0u;
        any |= d;
    }
    if (any) ws.added[1] = 1;      // a plain store of the same value from many threads
}

__global__ __launch_bounds__(256) void k_async_rank(const uint32_t *__restrict__ order, uint32_t n,
                                                    uint32_t *__restrict__ rank)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rank[order[i]] = i;
}

// Generation g: every donor of generation g reaches its recipient if it acts
// before it; a recipient not yet a donor joins generation g + 1.
__global__ __launch_bounds__(256) void k_async_generation(uint32_t n, uint32_t g, AsyncWs ws)
{
    if (ws.added[g] == 0) return;                 // the previous generation added no one
    const uint32_t stride = gridDim.x * blockDim.x;
    bool grew = false;
    for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += stride) {
        if (ws.gen[a] != g) continue;
        const uint32_t r = ws.recip[a];
        if (ws.rank[a] < ws.rank[r] && ws.gen[r] == 0)
            grew |= atomicCAS(&ws.gen[r], 0u, g + 1) == 0u;
    }
    if (grew) ws.added[g + 1] = 1;
}

// Every donor gives one unit to its recipient.  A fixed point not reached in
// ASYNC_MAX_GEN generations raises the sticky error word instead.
__global__ __launch_bounds__(256) void k_async_apply(int32_t *__restrict__ w, uint32_t n,
                                                     AsyncWs ws, uint32_t *err)
{
    if (ws.added[ASYNC_MAX_GEN + 1]) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            __hip_atomic_fetch_or(err, ERR_ASYNC_GENERATIONS, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += stride) {
        if (ws.gen[a] == 0) continue;
        atomicAdd(&w[a], -1);
        atomicAdd(&w[ws.recip[a]], 1);
    }
}

uint64_t align16(uint64_t v) { return (v + 15) & ~15ull; }

}  // namespace

uint64_t async_wealth_workspace(uint32_t n)
{
    return 4 * align16(4ull * n) + 4ull * ADDED_WORDS + view_scatter_f32_workspace(n);
}

hipError_t launch_wealth_async(int32_t *w, uint32_t n, uint32_t k0, uint32_t k1, uint32_t t0,
                               uint32_t n_steps, void *ws_base, uint32_t *err, hipStream_t st)
{
    uint8_t *b = (uint8_t *)ws_base;
    AsyncWs ws;
    const uint64_t col = align16(4ull * n);
    ws.key = (uint32_t *)b;
    ws.recip = (uint32_t *)(b + col);
    ws.rank = (uint32_t *)(b + 2 * col);
    ws.gen = (uint32_t *)(b + 3 * col);
    ws.added = (uint32_t *)(b + 4 * col);
    ws.sort = b + 4 * col + 4ull * ADDED_WORDS;
    const uint32_t quads = (n + 3) / 4;
    const uint32_t pass_blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    for (uint32_t i = 0; i < n_steps; ++i) {
        const uint32_t t = t0 + i;
        hipError_t e = launch_zero_words(ws.added, ADDED_WORDS, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_async_prep, dim3((quads + 255) / 256), dim3(256), 0, st, w, n, t, k0,
                           k1, ws);
        const uint32_t *keys = nullptr, *order = nullptr;
        e = radix_sort_ids(ws.key, 0xffffffffull, n, ws.sort, st, &keys, &order);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_async_rank, dim3((n + 255) / 256), dim3(256), 0, st, order, n,
                           ws.rank);
        for (uint32_t g = 1; g <= ASYNC_MAX_GEN; ++g)
            hipLaunchKernelGGL(k_async_generation, dim3(pass_blocks), dim3(256), 0, st, n, g, ws);
        hipLaunchKernelGGL(k_async_apply, dim3(pass_blocks), dim3(256), 0, st, w, n, ws, err);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace amber
