// amber_env.hip -- spatial environments of the method (Sec. 4.1) as device
// primitives: grid lattices of 1 to 4 dimensions with Moore or von Neumann
// neighbourhoods, torus-wrapped or bounded, and networks as CSR adjacency
// lists; plus the SIR transition on its own, given each agent's count.
//
// Grid cells are numbered with the first axis fastest (in 2-D, y * L + x,
// the layout of the SIR model's count grid).  A neighbour query is three
// streaming passes: bin the agents that count into a cell grid (one integer
// atomic per agent that counts), sum each cell's neighbourhood (the distinct
// cells of its Moore or von Neumann block; a torus side below 3 reaches a
// cell twice and counts it once), and gather each agent's cell.  All sums
// are integer, so every result is exact.
#include "amber_device_common.h"

namespace amber {
namespace {

__device__ __forceinline__ bool grid_cell(const GridDesc &g, uint64_t a, uint32_t *cell)
{
    uint32_t c = 0;
#pragma unroll
    for (uint32_t i = 0; i < MAX_DIMS; ++i) {
        if (i >= g.ndim) break;
        const int32_t v = g.pos[i][a];
        if (v < 0 || (uint32_t)v >= g.dims[i]) return false;
        c += (uint32_t)v * g.stride[i];
    }
    *cell = c;
    return true;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, uint64_t count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = 0;
}

__global__ __launch_bounds__(256) void k_grid_count(GridDesc g, uint64_t n,
                                                    const uint8_t *__restrict__ state,
                                                    uint32_t match, uint32_t *__restrict__ counts)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += stride) {
        if (state && state[a] != match) continue;
        uint32_t c;
        if (grid_cell(g, a, &c)) atomicAdd(counts + c, 1u);
    }
}

// One thread per cell: the offsets of {-1, 0, 1}^d (von Neumann: those with
// at most one non-zero component), wrapped or dropped at the edges; with
// `dedup` (a torus side below 3) a cell met twice is summed once.
__global__ __launch_bounds__(256) void k_grid_neighbour_sum(GridDesc g, uint64_t cells,
                                                            uint32_t von_neumann, uint32_t torus,
                                                            uint32_t dedup,
                                                            const uint32_t *__restrict__ counts,
                                                            uint32_t *__restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t noff = 1;
    for (uint32_t i = 0; i < g.ndim; ++i) noff *= 3;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += stride) {
        int32_t co[MAX_DIMS];
        uint32_t rest = (uint32_t)c;
#pragma unroll
        for (uint32_t i = 0; i < MAX_DIMS; ++i) {
            co[i] = 0;
            if (i < g.ndim) {
                co[i] = (int32_t)(rest % g.dims[i]);
                rest /= g.dims[i];
            }
        }
        uint32_t seen[81];
        uint32_t nseen = 0, sum = 0;
        for (uint32_t o = 0; o < noff; ++o) {
            uint32_t code = o, nonzero = 0, nb = 0;
            bool inside = true;
#pragma unroll
            for (uint32_t i = 0; i < MAX_DIMS; ++i) {
                if (i >= g.ndim) break;
                const int32_t d = (int32_t)(code % 3) - 1;
                code /= 3;
                nonzero += d != 0;
                int32_t v = co[i] + d;
                const int32_t L = (int32_t)g.dims[i];
                if (v < 0 || v >= L) {
                    if (torus) v = v < 0 ? v + L : v - L;
                    else inside = false;
                }
                nb += (uint32_t)v * g.stride[i];
            }
            if (!inside || (von_neumann && nonzero > 1)) continue;
            if (dedup) {
                bool dup = false;
                for (uint32_t k = 0; k < nseen; ++k) dup |= seen[k] == nb;
                if (dup) continue;
                seen[nseen++] = nb;
            }
            sum += counts[nb];
        }
        out[c] = sum;
    }
}

__global__ __launch_bounds__(256) void k_grid_gather(GridDesc g, uint64_t n,
                                                     const uint32_t *__restrict__ table,
                                                     uint32_t *__restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += stride) {
        uint32_t c;
        out[a] = grid_cell(g, a, &c) ? table[c] : 0u;
    }
}

// One thread per node; adjacency entries past nnz or naming no node are not
// counted.
__global__ __launch_bounds__(256) void k_graph_count(const uint32_t *__restrict__ row,
                                                     const uint32_t *__restrict__ col, uint64_t n,
                                                     uint64_t nnz, const uint8_t *__restrict__ state,
                                                     uint32_t match, uint32_t *__restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t e1 = row[i + 1] < nnz ? row[i + 1] : nnz;
        uint32_t k = 0;
        for (uint64_t e = row[i]; e < e1; ++e) {
            const uint32_t j = col[e];
            k += j < n && state[j] == match;
        }
        out[i] = k;
    }
}

// Four agents per thread (one EPI block per four agents, as in the model):
// S with k >= 1 to I iff u < T_inf[min(k, len - 1)], I to R iff u < T_rec.
__global__ __launch_bounds__(256) void k_sir_transition_only(uint8_t *__restrict__ s,
                                                             const uint32_t *__restrict__ k,
                                                             uint64_t n, uint32_t k0, uint32_t k1,
                                                             uint32_t t,
                                                             const uint32_t *__restrict__ t_inf,
                                                             uint32_t table_len, uint32_t t_rec)
{
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t a0 = 4 * q;
    if (a0 >= n) return;
    uint32_t st[4], kk[4];
    bool need = false;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        st[j] = a0 + j < n ? s[a0 + j] : (uint32_t)ST_R;
        kk[j] = a0 + j < n ? k[a0 + j] : 0u;
        need |= (st[j] == ST_S && kk[j] >= 1) || st[j] == ST_I;
    }
    if (!need) return;
    const uint4 r = philox((uint32_t)q, t, P_EPI, k0, k1);
    const uint32_t u[4] = {r.x, r.y, r.z, r.w};
    const uint32_t last = table_len - 1;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        if (a0 + j >= n) break;
        if (st[j] == ST_S && kk[j] >= 1) {
            if (u[j] < t_inf[kk[j] < last ? kk[j] : last]) s[a0 + j] = ST_I;
        } else if (st[j] == ST_I) {
            if (u[j] < t_rec) s[a0 + j] = ST_R;
        }
    }
}

uint32_t env_grid(uint64_t items)
{
    const uint64_t g = (items + 255) / 256;
    return (uint32_t)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

}  // namespace

hipError_t launch_grid_count(const GridDesc &g, uint64_t n, const uint8_t *state, uint32_t match,
                             uint32_t *counts, uint64_t cells, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(env_grid(cells)), dim3(256), 0, st, counts, cells);
    if (n) hipLaunchKernelGGL(k_grid_count, dim3(env_grid(n)), dim3(256), 0, st, g, n, state,
                              match, counts);
    return hipGetLastError();
}

hipError_t launch_grid_neighbour_sum(const GridDesc &g, uint64_t cells, uint32_t von_neumann,
                                     uint32_t torus, uint32_t dedup, const uint32_t *counts,
                                     uint32_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_grid_neighbour_sum, dim3(env_grid(cells)), dim3(256), 0, st, g, cells,
                       von_neumann, torus, dedup, counts, out);
    return hipGetLastError();
}

hipError_t launch_grid_gather(const GridDesc &g, uint64_t n, const uint32_t *table, uint32_t *out,
                              hipStream_t st)
{
    if (n) hipLaunchKernelGGL(k_grid_gather, dim3(env_grid(n)), dim3(256), 0, st, g, n, table, out);
    return hipGetLastError();
}

hipError_t launch_graph_count(const uint32_t *row, const uint32_t *col, uint64_t n, uint64_t nnz,
                              const uint8_t *state, uint32_t match, uint32_t *out, hipStream_t st)
{
    if (n) hipLaunchKernelGGL(k_graph_count, dim3(env_grid(n)), dim3(256), 0, st, row, col, n, nnz,
                              state, match, out);
    return hipGetLastError();
}

hipError_t launch_sir_transition_only(uint8_t *s, const uint32_t *k, uint64_t n, uint32_t k0,
                                      uint32_t k1, uint32_t t, const uint32_t *t_inf,
                                      uint32_t table_len, uint32_t t_rec, hipStream_t st)
{
    const uint64_t quads = (n + 3) / 4;
    if (n) hipLaunchKernelGGL(k_sir_transition_only, dim3((unsigned)((quads + 255) / 256)),
                              dim3(256), 0, st, s, k, n, k0, k1, t, t_inf, table_len, t_rec);
    return hipGetLastError();
}

}  // namespace amber
