// amber_internal.h -- launchers shared by the host runtime (amber_host.cpp)
// and the gfx950 kernels (amber_device.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace amber {

// Purposes of the counter-based random stream (counter word 2).
enum : uint32_t { P_INIT_POS = 0, P_MOVE = 1, P_EPI = 2, P_RECIPIENT = 3 };

// State codes of the SIR column.
enum : uint8_t { ST_S = 0, ST_I = 1, ST_R = 2 };

// Every column is padded to whole groups of this many agents.
constexpr uint32_t AGENT_PAD = 64;

// Device-side accumulators of amber_invariants (lives at workspace offset 0).
struct DevInvariants {
    unsigned long long wealth_sum;   // two's-complement int64 sum
    unsigned long long n_s, n_i, n_r;
    unsigned long long out_of_bounds;
    unsigned long long digest;
    int wealth_min;
    int pad[3];
};
static_assert(sizeof(DevInvariants) <= 256, "invariants block must fit 256 B");

// Per-run parameters of a SIR step, passed by value.
struct SirParams {
    int32_t *x;
    int32_t *y;
    uint8_t *s;
    uint32_t *count[2];        // per-cell infected counts, double buffered by step parity
    const uint32_t *t_inf;     // infection thresholds, table_len entries
    uint32_t table_len;        // k_sat + 1
    uint32_t t_rec;
    uint32_t n;
    int32_t L;
    uint32_t k0, k1;           // Philox key (seed, stream)
};

// Launch configuration knobs (results never depend on them).
struct Tuning {
    uint32_t block = 256;      // threads per workgroup (multiple of 64, <= 1024)
};

hipError_t launch_init_wealth(int32_t *w, int32_t *inc0, int32_t *inc1, uint32_t n,
                              int32_t w_init, hipStream_t st);
hipError_t launch_init_positions(int32_t *x, int32_t *y, uint32_t n, int32_t L,
                                 uint32_t k0, uint32_t k1, hipStream_t st);
hipError_t launch_init_states(uint8_t *s, uint32_t n, uint32_t i0, hipStream_t st);
hipError_t launch_zero_words(uint32_t *p, uint64_t words, hipStream_t st);

// Random walk: steps t0 .. t0+n_steps-1 with positions held in registers.
hipError_t launch_walk(int32_t *x, int32_t *y, uint32_t n, int32_t L, uint32_t k0,
                       uint32_t k1, uint32_t t0, uint32_t n_steps, const Tuning &tu,
                       hipStream_t st);

// Wealth: one step t.  The state is base + inc_cur; the step leaves base' in
// base, zeroes inc_cur and scatters the recipients' units into inc_nxt
// (which must be zero on entry).
hipError_t launch_wealth_step(int32_t *base, int32_t *inc_cur, int32_t *inc_nxt, uint32_t n,
                              uint32_t k0, uint32_t k1, uint32_t t, const Tuning &tu,
                              hipStream_t st);
// base += inc; inc = 0.
hipError_t launch_wealth_fold(int32_t *base, int32_t *inc, uint32_t n, hipStream_t st);
// Whole run segment for small N in one workgroup (state in LDS).
hipError_t launch_wealth_small(int32_t *w, uint32_t n, uint32_t k0, uint32_t k1,
                               uint32_t t0, uint32_t n_steps, hipStream_t st);
uint32_t wealth_small_max_agents();

// SIR: one step t (move + bin into count[t&1]; then transition, which also
// clears count[(t+1)&1] for the next step).
hipError_t launch_sir_step(const SirParams &p, uint32_t t, const Tuning &tu, hipStream_t st);

hipError_t launch_invariants(uint32_t model, uint32_t n, int32_t L, const int32_t *w,
                             const int32_t *x, const int32_t *y, const uint8_t *s,
                             DevInvariants *acc, hipStream_t st);

}  // namespace amber
