// amber_batch.hip -- batched forms: many runs (replicates, sweep points,
// served requests) of one model advance together, one launch per phase for a
// whole chunk of runs instead of one launch per run.
//
// A chunk's run table travels in the kernel arguments (no device allocation):
// run r owns workgroups [block_end[r-1], block_end[r]), and each workgroup
// finds its run with a wavefront-uniform scan of block_end.  Every run keeps
// its own descriptor, key and step index, and each of its agent groups runs
// exactly the per-group body the single-run kernels use, so a run's result is
// bit-identical alone or in any batch.
#include "amber_device_common.h"

namespace amber {

// Run index of this workgroup and its block index within that run.
__device__ __forceinline__ uint32_t batch_run(const uint32_t *block_end, uint32_t nruns,
                                              uint32_t &local_block, uint32_t &run_blocks)
{
    uint32_t r = 0;
    while (r + 1 < nruns && blockIdx.x >= block_end[r]) ++r;
    const uint32_t first = r ? block_end[r - 1] : 0;
    local_block = blockIdx.x - first;
    run_blocks = block_end[r] - first;
    return r;
}

// ------------------------------------------------------------------ random walk

__global__ void k_walk_batch(WalkBatch b, uint32_t n_steps)
{
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.block_end, b.nruns, lb, nb);
    const uint32_t q = lb * blockDim.x + threadIdx.x;
    if (q < groups_of(b.n[r]))
        walk_group((int4 *)b.x[r], (int4 *)b.y[r], q, b.L[r], b.k0[r], b.k1[r], b.t0[r], n_steps);
}

// ------------------------------------------------------------------ wealth

// One workgroup per small run (state in LDS for every step).
__global__ __launch_bounds__(WEALTH_SMALL_THREADS) void k_wealth_small_batch(WealthSmallBatch b,
                                                                             uint32_t n_steps)
{
    __shared__ int32_t sw[WEALTH_SMALL_MAX];
    __shared__ int32_t sinc[WEALTH_SMALL_MAX];
    const uint32_t r = blockIdx.x;
    wealth_small_run(b.w[r], sw, sinc, b.n[r], b.k0[r], b.k1[r], b.t0[r], n_steps);
}

// Step i of the call for every large run of the chunk.
__global__ void k_wealth_step_batch(WealthBatch b, uint32_t i)
{
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.block_end, b.nruns, lb, nb);
    const uint32_t q = lb * blockDim.x + threadIdx.x;
    if (q < groups_of(b.n[r]))
        wealth_step_group((int4 *)b.base[r], (int4 *)b.inc[i & 1][r], b.inc[(i + 1) & 1][r], q,
                          b.n[r], b.k0[r], b.k1[r], b.t0[r] + i);
}

__global__ void k_wealth_fold_batch(WealthBatch b, uint32_t parity)
{
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.block_end, b.nruns, lb, nb);
    const uint32_t q = lb * blockDim.x + threadIdx.x;
    if (q < groups_of(b.n[r])) wealth_fold_group((int4 *)b.base[r], (int4 *)b.inc[parity][r], q);
}

template <int XB, int PMAX, int NT>
__global__ __launch_bounds__(NT) void k_wealth_x_batch(WealthXBatch b, uint32_t i,
                                                       uint32_t parity_in, uint32_t mode)
{
    __shared__ __align__(16) int32_t hist[1u << XB];
    __shared__ uint32_t pcount[PMAX];
    __shared__ uint32_t poff[PMAX];
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.block_end, b.nruns, lb, nb);
    // blocks lb and lb + 8 of a run sit on one XCD whatever the run's first
    // block: the run's partitions are dealt as in the single-run kernel
    wealth_exchange_partition<XB, PMAX, NT>(b.run[r], xcd_partition(lb, nb), b.t0[r] + i,
                                            parity_in, (mode & 1u) != 0, (mode & 2u) != 0, hist,
                                            pcount, poff);
}

// ------------------------------------------------------------------ SIR (pipelined)

// In gather mode each run's last workgroup holds no agents and does the
// demand-binning bookkeeping (as in the single-run kernels).
template <bool BOX>
__global__ void k_sir_head_batch(SirBatch b)
{
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.block_end, b.nruns, lb, nb);
    const SirParams &p = b.run[r];
    const uint32_t q = lb * blockDim.x + threadIdx.x;
    if (BOX) {
        if (q < p.groups) sir_head_group<BOX>(p, q, b.t0[r]);
        return;
    }
    if (lb == nb - 1) {
        sir_demand_book(p, 0);
        return;
    }
    __shared__ uint32_t s_wc[2 * 16];
    sir_head_demand(p, q, (nb - 1) * blockDim.x, b.t0[r], lb, s_wc);
}

template <bool BOX>
__global__ void k_sir_body_batch(SirBatch b, uint32_t i)
{
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.block_end, b.nruns, lb, nb);
    const SirParams &p = b.run[r];
    const uint32_t t = b.t0[r] + i;
    const uint32_t q = lb * blockDim.x + threadIdx.x;
    if (BOX) {
        if (q < p.groups) sir_body_group<BOX>(p, q, t);
        return;
    }
    if (lb == nb - 1) {
        sir_demand_book(p, i);
        return;
    }
    __shared__ uint32_t s_wc[2 * 16];
    sir_body_demand(p, q, (nb - 1) * blockDim.x, t, i, lb, s_wc);
}

// gather mode: the dirty check reads the flag of the run's last body launch
template <bool BOX>
__global__ void k_sir_tail_batch(SirBatch b, uint32_t i)
{
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.block_end, b.nruns, lb, nb);
    const SirParams &p = b.run[r];
    const uint32_t t = b.t0[r] + i;
    const uint32_t q = lb * blockDim.x + threadIdx.x;
    if (!BOX) {
        zero_quads(grid_of(p, t + 2), p.quads, q, nb * blockDim.x);
        if (sir_demand_dirty(p, b.i_last[r])) {     // a body launch ran transition(t)
            zero_quads(grid_of(p, t), p.quads, q, nb * blockDim.x);
            zero_quads(grid_of(p, t + 1), p.quads, q, nb * blockDim.x);
            return;
        }
    }
    if (q < p.groups) sir_tail_group<BOX>(p, q, t);
}

// Box and clear kernels map workgroups to each run's grid cells.
__global__ void k_sir_box_batch(SirBatch b, uint32_t i)
{
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.cell_block_end, b.nruns, lb, nb);
    const SirParams &p = b.run[r];
    const uint32_t t = b.t0[r] + i;
    const uint32_t c = lb * blockDim.x + threadIdx.x;
    zero_quads(cgrid_box(p, t + 1), p.quads, c, nb * blockDim.x);
    if (c < p.quads) sir_box_quad(p, cgrid_box(p, t), kgrid_box(p), c);
}

__global__ void k_sir_clear_batch(SirBatch b, uint32_t mask)
{
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.cell_block_end, b.nruns, lb, nb);
    const SirParams &p = b.run[r];
    const uint32_t c = lb * blockDim.x + threadIdx.x;
    for (int g = 0; g < 3; ++g)
        if (mask & (1u << g)) zero_quads(p.count[g], p.quads, c, nb * blockDim.x);
    if (lb == 0) sir_demand_reset(p, threadIdx.x, blockDim.x);
}

// Exchange count mode, batched: producer workgroups and band workgroups of
// every run of the chunk in one launch each.
constexpr uint32_t BX_PMAX = 2048;
constexpr uint32_t BX_HIST = 16384;

template <bool TRANSITION>
__global__ __launch_bounds__(256) void k_sir_xbody_batch(SirBatch b, uint32_t i)
{
    __shared__ uint32_t pcount[BX_PMAX];
    __shared__ uint32_t poff[BX_PMAX];
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.xblock_end, b.nruns, lb, nb);
    sir_exchange_produce<TRANSITION>(b.run[r], lb, b.t0[r] + i, pcount, poff);
}

__global__ __launch_bounds__(256) void k_sir_xcount_batch(SirBatch b)
{
    __shared__ uint32_t hist[BX_HIST];
    __shared__ uint32_t scnt[XCHUNK];
    __shared__ uint32_t soff[XCHUNK];
    __shared__ uint32_t sraw[XCHUNK];
    uint32_t lb, nb;
    const uint32_t r = batch_run(b.band_end, b.nruns, lb, nb);
    sir_exchange_count(b.run[r], lb, hist, scnt, soff, sraw);
}

// ------------------------------------------------------------------ launchers

hipError_t launch_walk_batch(const WalkBatch &b, uint32_t n_steps, uint32_t block, hipStream_t st)
{
    const uint32_t blocks = b.block_end[b.nruns - 1];
    hipLaunchKernelGGL(k_walk_batch, dim3(blocks), dim3(block), 0, st, b, n_steps);
    return hipGetLastError();
}

hipError_t launch_wealth_small_batch(const WealthSmallBatch &b, uint32_t n_steps, hipStream_t st)
{
    hipLaunchKernelGGL(k_wealth_small_batch, dim3(b.nruns), dim3(WEALTH_SMALL_THREADS), 0, st, b,
                       n_steps);
    return hipGetLastError();
}

hipError_t launch_wealth_batch(const WealthBatch &b, uint32_t n_steps, uint32_t block,
                               hipStream_t st)
{
    const uint32_t blocks = b.block_end[b.nruns - 1];
    for (uint32_t i = 0; i < n_steps; ++i) {
        hipLaunchKernelGGL(k_wealth_step_batch, dim3(blocks), dim3(block), 0, st, b, i);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_wealth_fold_batch, dim3(blocks), dim3(block), 0, st, b, n_steps & 1);
    return hipGetLastError();
}

template <int XB, int PMAX, int NT>
static hipError_t wealth_x_batch_steps(const WealthXBatch &b, uint32_t n_steps, hipStream_t st)
{
    const uint32_t blocks = b.block_end[b.nruns - 1];
    for (uint32_t i = 0; i <= n_steps; ++i) {
        // i < n_steps: step i (mode 2 first, then 3); i == n_steps: final fold
        const uint32_t mode = i == n_steps ? 1u : (i ? 3u : 2u);
        const uint32_t parity_in = i == n_steps ? ((n_steps - 1) & 1u) : ((i + 1) & 1u);
        hipLaunchKernelGGL((k_wealth_x_batch<XB, PMAX, NT>), dim3(blocks), dim3(NT), 0, st, b, i,
                           parity_in, mode);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_wealth_exchange_batch(const WealthXBatch &b, uint32_t n_steps, uint32_t bits,
                                        hipStream_t st)
{
    for (uint32_t r = 0; r < b.nruns; ++r)
        if (b.run[r].P > (bits == 14 ? 1024u : 512u)) return hipErrorInvalidValue;
    if (bits == 11) return wealth_x_batch_steps<11, 512, 512>(b, n_steps, st);
    if (bits == 12) return wealth_x_batch_steps<12, 512, 1024>(b, n_steps, st);
    if (bits == 14) return wealth_x_batch_steps<14, 1024, 1024>(b, n_steps, st);
    return hipErrorInvalidValue;
}

hipError_t launch_sir_batch(const SirBatch &b, uint32_t n_steps, uint32_t mode, uint32_t block,
                            hipStream_t st)
{
    const uint32_t blocks = b.block_end[b.nruns - 1];
    const uint32_t cblocks = b.cell_block_end[b.nruns - 1];
    hipError_t e;
#define AMBER_LAUNCH(...)                                              \
    do {                                                               \
        hipLaunchKernelGGL(__VA_ARGS__);                               \
        if ((e = hipGetLastError()) != hipSuccess) return e;           \
    } while (0)
    if (mode == 3) {
        const uint32_t xblocks = b.xblock_end[b.nruns - 1];
        const uint32_t bands = b.band_end[b.nruns - 1];
        AMBER_LAUNCH(k_sir_xbody_batch<false>, dim3(xblocks), dim3(256), 0, st, b, 0u);
        AMBER_LAUNCH(k_sir_xcount_batch, dim3(bands), dim3(256), 0, st, b);
        for (uint32_t i = 1; i < n_steps; ++i) {
            AMBER_LAUNCH(k_sir_xbody_batch<true>, dim3(xblocks), dim3(256), 0, st, b, i);
            AMBER_LAUNCH(k_sir_xcount_batch, dim3(bands), dim3(256), 0, st, b);
        }
        AMBER_LAUNCH(k_sir_tail_batch<true>, dim3(blocks), dim3(block), 0, st, b, n_steps - 1);
        AMBER_LAUNCH(k_sir_clear_batch, dim3(cblocks), dim3(256), 0, st, b, 4u);
    } else if (mode == 2) {
        AMBER_LAUNCH(k_sir_head_batch<true>, dim3(blocks), dim3(block), 0, st, b);
        AMBER_LAUNCH(k_sir_box_batch, dim3(cblocks), dim3(256), 0, st, b, 0u);
        for (uint32_t i = 1; i < n_steps; ++i) {
            AMBER_LAUNCH(k_sir_body_batch<true>, dim3(blocks), dim3(block), 0, st, b, i);
            AMBER_LAUNCH(k_sir_box_batch, dim3(cblocks), dim3(256), 0, st, b, i);
        }
        AMBER_LAUNCH(k_sir_tail_batch<true>, dim3(blocks), dim3(block), 0, st, b, n_steps - 1);
        AMBER_LAUNCH(k_sir_clear_batch, dim3(cblocks), dim3(256), 0, st, b,
                     (1u << ((n_steps - 1) & 1)) | 4u);
    } else {
        return hipErrorInvalidValue;           // gather mode: launch_sir_gather_batch
    }
#undef AMBER_LAUNCH
    return hipSuccess;
}

hipError_t launch_sir_gather_batch(const SirBatch &b, uint32_t phase, uint32_t i, uint32_t n_steps,
                                   uint32_t block, hipStream_t st)
{
    const uint32_t blocks = b.block_end[b.nruns - 1];
    const uint32_t cblocks = b.cell_block_end[b.nruns - 1];
    if (phase == 0)
        hipLaunchKernelGGL(k_sir_head_batch<false>, dim3(blocks), dim3(block), 0, st, b);
    else if (phase == 1)
        hipLaunchKernelGGL(k_sir_body_batch<false>, dim3(blocks), dim3(block), 0, st, b, i);
    else if (phase == 2)
        hipLaunchKernelGGL(k_sir_tail_batch<false>, dim3(blocks), dim3(block), 0, st, b,
                           n_steps - 1);
    else
        hipLaunchKernelGGL(k_sir_clear_batch, dim3(cblocks), dim3(256), 0, st, b,
                           1u << ((n_steps - 1) % 3));
    return hipGetLastError();
}

}  // namespace amber
