// amber_host.cpp -- host runtime and C ABI of libamber (see include/amber.h).
//
// Validates run descriptors, derives the run's parameters (grid side, initial
// infected count, exact uint32 Bernoulli thresholds), lays out the caller's
// workspace, and enqueues the gfx950 kernels on the caller's HIP stream.  The
// library never allocates device memory.
#include "amber.h"
#include "amber_internal.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

using namespace amber;

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

static amber_status_t fail(amber_status_t st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

static amber_status_t hip_fail(hipError_t e, const char *what)
{
    return fail(AMBER_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ------------------------------------------------------------------ bignum
// Exact infection thresholds T[k] = floor(2^32 (d^k - m^k) / d^k), m = d - n,
// for beta = n/d.  Numbers are little-endian vectors of 32-bit limbs.

namespace {

using Limbs = std::vector<uint32_t>;

void trim(Limbs &a)
{
    while (a.size() > 1 && a.back() == 0) a.pop_back();
}

void mul_small(Limbs &a, uint32_t m)
{
    uint64_t carry = 0;
    for (auto &l : a) {
        const uint64_t v = (uint64_t)l * m + carry;
        l = (uint32_t)v;
        carry = v >> 32;
    }
    if (carry) a.push_back((uint32_t)carry);
    trim(a);
}

int cmp(const Limbs &a, const Limbs &b)
{
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

// a -= b, requires a >= b
void sub_in_place(Limbs &a, const Limbs &b)
{
    int64_t borrow = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        int64_t v = (int64_t)a[i] - borrow - (i < b.size() ? (int64_t)b[i] : 0);
        borrow = v < 0;
        a[i] = (uint32_t)(v + (borrow << 32));
    }
    trim(a);
}

void add_in_place(Limbs &a, const Limbs &b)
{
    if (a.size() < b.size()) a.resize(b.size(), 0);
    uint64_t carry = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        const uint64_t v = (uint64_t)a[i] + (i < b.size() ? b[i] : 0) + carry;
        a[i] = (uint32_t)v;
        carry = v >> 32;
    }
    if (carry) a.push_back((uint32_t)carry);
}

uint32_t bit_length(const Limbs &a)
{
    const uint32_t top = a.back();
    uint32_t bits = 32 * (uint32_t)(a.size() - 1);
    return top ? bits + 32 - __builtin_clz(top) : bits;
}

// floor(a / 2^sh) truncated to 64 bits (callers ensure it fits)
uint64_t shifted_top(const Limbs &a, uint32_t sh)
{
    uint64_t out = 0;
    for (uint32_t b = 0; b < 64; ++b) {
        const uint32_t bit = sh + b;
        const size_t li = bit / 32;
        if (li < a.size() && ((a[li] >> (bit % 32)) & 1u)) out |= 1ull << b;
    }
    return out;
}

// floor(2^32 * num / den) for 0 <= num < den (result < 2^32).
uint32_t scaled_quotient(const Limbs &num, const Limbs &den)
{
    const uint32_t bl = bit_length(den);
    const uint32_t sh = bl > 64 ? bl - 64 : 0;
    const uint64_t nt = shifted_top(num, sh);
    const uint64_t dt = shifted_top(den, sh);
    unsigned __int128 est = ((unsigned __int128)nt << 32) / dt;
    if (est > 0xffffffffull) est = 0xffffffffull;
    uint32_t q = (uint32_t)est;
    // exact correction: want q*den <= num*2^32 < (q+1)*den
    Limbs target(num.size() + 1, 0);
    std::copy(num.begin(), num.end(), target.begin() + 1);
    trim(target);
    Limbs prod = den;
    mul_small(prod, q);
    while (cmp(prod, target) > 0) {
        sub_in_place(prod, den);
        --q;
    }
    for (;;) {
        Limbs next = prod;
        add_in_place(next, den);
        if (cmp(next, target) > 0) break;
        prod.swap(next);
        ++q;
    }
    return q;
}

// Builds the table; returns AMBER_OK, AMBER_E_INVALID or AMBER_E_UNSUPPORTED.
amber_status_t build_infection_table_exact(uint32_t num, uint32_t den, std::vector<uint32_t> &out)
{
    out.clear();
    if (den == 0 || num >= den)
        return fail(AMBER_E_INVALID, "beta must satisfy 0 <= num < den (got %u/%u)", num, den);
    out.push_back(0);
    if (num == 0) return AMBER_OK;
    const uint32_t m = den - num;
    Limbs miss{1}, whole{1};                  // m^k, d^k
    for (;;) {
        mul_small(miss, m);
        mul_small(whole, den);
        Limbs hit = whole;
        sub_in_place(hit, miss);              // d^k - m^k
        const uint32_t t = scaled_quotient(hit, whole);
        out.push_back(t);
        if (t == 0xffffffffu) return AMBER_OK;
        if (out.size() >= AMBER_MAX_TABLE)
            return fail(AMBER_E_UNSUPPORTED,
                        "beta %u/%u needs more than %u threshold entries", num, den,
                        AMBER_MAX_TABLE);
    }
}

// The exact tables of the betas seen so far (a pure function of beta; long
// tables take milliseconds of big-integer arithmetic, and sweeps repeat a
// few betas over many runs).  At most 256 are kept.
amber_status_t build_infection_table(uint32_t num, uint32_t den, std::vector<uint32_t> &out)
{
    static std::mutex mu;
    static std::map<std::pair<uint32_t, uint32_t>, std::vector<uint32_t>> *cache =
        new std::map<std::pair<uint32_t, uint32_t>, std::vector<uint32_t>>;   // never destroyed
    const std::pair<uint32_t, uint32_t> key(num, den);
    {
        std::lock_guard<std::mutex> lk(mu);
        const auto it = cache->find(key);
        if (it != cache->end()) {
            out = it->second;
            return AMBER_OK;
        }
    }
    const amber_status_t st = build_infection_table_exact(num, den, out);
    if (st == AMBER_OK) {
        std::lock_guard<std::mutex> lk(mu);
        if (cache->size() >= 256) cache->clear();
        (*cache)[key] = out;
    }
    return st;
}

uint32_t bernoulli_threshold(uint32_t num, uint32_t den)
{
    return (uint32_t)(((uint64_t)num << 32) / den);
}

// round(sqrt(n)), halves up: s = isqrt(n); s + 1 iff n > s^2 + s.
uint32_t round_sqrt(uint32_t n)
{
    uint64_t s = 0;
    for (int b = 31; b >= 0; --b) {
        const uint64_t c = s | (1ull << b);
        if (c * c <= n) s = c;
    }
    return (uint32_t)(((uint64_t)n > s * s + s) ? s + 1 : s);
}

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

uint32_t groups_of_host(uint32_t n) { return (n + 3) / 4; }

// Resolved, validated parameters of a run.
struct Resolved {
    uint32_t model = 0, n = 0, L = 0, i0 = 0, seed = 0, stream = 0;
    int32_t w_init = 0;
    uint32_t t_rec = 0;
    std::vector<uint32_t> t_inf;
    // workspace layout (byte offsets)
    uint64_t off_inc0 = 0, off_inc1 = 0, off_table = 0, off_count[3] = {0, 0, 0}, off_sync = 0;
    uint64_t off_nsi = 0, off_dmap[3] = {0, 0, 0};
    uint32_t cside = 0;                             // coarse demand maps (0 = none)
    uint32_t xbits = 0, xparts = 0;                 // wealth partition exchange (0 = unavailable)
    uint32_t sx_h = 0, sx_P = 0, sx_W = 0;          // SIR exchange count mode (0 = unavailable)
    uint64_t off_sxrec = 0, off_sxtab = 0;
    uint64_t off_xrec[2] = {0, 0}, off_xtab[2] = {0, 0};
    // SIR tiled count mode (tile_tiles = 0: unavailable)
    uint32_t tile_tiles = 0;                        // tiles of the smallest side the buffers fit
    uint64_t tile_rec = 0;                          // record slots per generation
    uint64_t off_trec[2] = {0, 0}, off_thdr[2] = {0, 0}, off_tring[2] = {0, 0};
    uint64_t off_tcur = 0, off_tctr = 0, off_tscnt = 0;
    uint64_t ws_bytes = 0;
};

uint64_t padded_agents(uint32_t n) { return align_up(n, AGENT_PAD); }

amber_status_t resolve(const amber_run_desc_t *d, Resolved &r, bool want_table)
{
    if (!d) return fail(AMBER_E_INVALID, "descriptor is NULL");
    if (d->abi_version != AMBER_ABI_VERSION)
        return fail(AMBER_E_INVALID, "abi_version %u != %u", d->abi_version, AMBER_ABI_VERSION);
    if (d->model > AMBER_SIR) return fail(AMBER_E_INVALID, "unknown model %u", d->model);
    if (d->n_agents == 0 || d->n_agents > 0x7fffffffu)
        return fail(AMBER_E_INVALID, "n_agents must be in [1, 2^31-1] (got %u)", d->n_agents);
    r.model = d->model;
    r.n = d->n_agents;
    r.seed = d->seed;
    r.stream = d->stream;
    uint64_t ws = INV_REGION;   // invariants result + per-block partials
    if (d->model == AMBER_WEALTH) {
        if (d->wealth_init < 0) return fail(AMBER_E_INVALID, "wealth_init must be >= 0");
        if ((uint64_t)d->n_agents * (uint64_t)d->wealth_init > 0x7fffffffull)
            return fail(AMBER_E_INVALID, "N * wealth_init must stay below 2^31");
        r.w_init = d->wealth_init;
        const uint64_t col = align_up(padded_agents(r.n) * 4, 256);
        r.off_inc0 = ws;
        r.off_inc1 = ws + col;
        ws += 2 * col;
        if (r.n > wealth_small_max_agents() && (r.xbits = wealth_exchange_bits(r.n)) != 0) {
            r.xparts = (uint32_t)((r.n + (1ull << r.xbits) - 1) >> r.xbits);
            const uint64_t rec = align_up((uint64_t)r.xparts << (r.xbits + 2), 256);
            const uint64_t tab = align_up((uint64_t)r.xparts * r.xparts * 4, 256);
            for (int b = 0; b < 2; ++b) {
                r.off_xrec[b] = ws;
                ws += rec;
                r.off_xtab[b] = ws;
                ws += tab;
            }
        }
    } else {
        const uint32_t L = d->grid_side ? d->grid_side : round_sqrt(d->n_agents);
        if (L == 0 || (uint64_t)L * L > 0x7fffffffull)
            return fail(AMBER_E_INVALID, "grid side must satisfy 1 <= L and L*L < 2^31 (got %u)", L);
        r.L = L;
        if (d->model == AMBER_SIR) {
            if (d->gamma_den == 0 || d->gamma_num >= d->gamma_den)
                return fail(AMBER_E_INVALID, "gamma must satisfy 0 <= num < den (got %u/%u)",
                            d->gamma_num, d->gamma_den);
            if (d->beta_den == 0 || d->beta_num >= d->beta_den)
                return fail(AMBER_E_INVALID, "beta must satisfy 0 <= num < den (got %u/%u)",
                            d->beta_num, d->beta_den);
            r.i0 = d->initial_infected ? d->initial_infected
                                       : std::max<uint32_t>(1, (d->n_agents + 500u) / 1000u);
            if (r.i0 > r.n) return fail(AMBER_E_INVALID, "initial_infected %u > N", r.i0);
            r.t_rec = bernoulli_threshold(d->gamma_num, d->gamma_den);
            if (want_table) {
                amber_status_t st = build_infection_table(d->beta_num, d->beta_den, r.t_inf);
                if (st != AMBER_OK) return st;
            }
            const uint64_t cells = align_up((uint64_t)L * L, AGENT_PAD) * 4;
            r.off_table = ws;
            ws += align_up((uint64_t)AMBER_MAX_TABLE * 4, 256);
            for (int b = 0; b < 3; ++b) {
                r.off_count[b] = ws;
                ws += align_up(cells, 256);
            }
            r.off_nsi = ws;
            ws += align_up((uint64_t)NSI_WORDS * 4, 256);
            // demand maps, each followed by its coarse map (one byte per 8 x 8
            // cells) on grids larger than an XCD's L2
            r.cside = (uint64_t)L * L > (4ull << 20) ? (L + 7) / 8 : 0u;
            for (int b = 0; b < 3; ++b) {
                r.off_dmap[b] = ws;
                ws += align_up((uint64_t)L * L, 256) + align_up((uint64_t)r.cside * r.cside, 256);
            }
            r.off_sync = ws;
            ws += align_up((uint64_t)SYNC_WORDS * 4, 256);
            if (sir_exchange_shape(r.n, L, &r.sx_h, &r.sx_P, &r.sx_W)) {
                r.off_sxrec = ws;
                ws += align_up((uint64_t)r.sx_W * XSEG_WORDS * 4, 256);
                r.off_sxtab = ws;
                ws += align_up((uint64_t)r.sx_W * r.sx_P * 4, 256);
            }
            const uint32_t nt = sir_tile_count(L, TILE_MIN);
            if (nt && r.n <= TILE_MAX_AGENTS) {
                // records (slots of every tile side plus the overflow area),
                // headers and ring arrays of both generations; headers and
                // rings are sized for the smallest tile side
                r.tile_tiles = nt * nt;
                uint64_t slots = 0;
                for (uint32_t T = TILE_MIN; T <= 64; T *= 2) {
                    const uint64_t k = sir_tile_count(L, T);
                    if (k) slots = std::max<uint64_t>(slots, k * k * sir_tile_cap(r.n, (uint32_t)(k * k)));
                }
                r.tile_rec = slots + r.n;
                for (int b = 0; b < 2; ++b) {
                    r.off_trec[b] = ws;
                    ws += align_up(r.tile_rec * 8, 256);
                    r.off_thdr[b] = ws;
                    ws += align_up((uint64_t)r.tile_tiles * TILE_HDR * 4, 256);
                    r.off_tring[b] = ws;
                    ws += align_up(sir_tile_ring_words(L) * 4, 256);
                }
                r.off_tcur = ws;
                ws += align_up((uint64_t)r.tile_tiles * 4, 256);
                r.off_tctr = ws;
                ws += 512;
                r.off_tscnt = ws;               // susceptible agents per tile
                ws += align_up((uint64_t)r.tile_tiles * 4, 256);
            }
        }
    }
    r.ws_bytes = ws;
    return AMBER_OK;
}

size_t column_bytes(const Resolved &r, amber_col_t c)
{
    const uint64_t pad = padded_agents(r.n);
    switch (c) {
    case AMBER_COL_WEALTH: return r.model == AMBER_WEALTH ? pad * 4 : 0;
    case AMBER_COL_X:
    case AMBER_COL_Y: return r.model != AMBER_WEALTH ? pad * 4 : 0;
    case AMBER_COL_STATE: return r.model == AMBER_SIR ? pad : 0;
    }
    return 0;
}

}  // namespace

// ------------------------------------------------------------------ handle

// Optional per-kernel timing: HIP events recorded on the handle's stream
// around every kernel the handle enqueues.
struct KernelTimer {
    bool on = false;
    struct Pending {
        uint32_t kernel;
        uint32_t count;          // launches between start and stop
        hipEvent_t start, stop;
    };
    std::vector<Pending> pending;
    bool chain = false;          // the last pending pair may be extended
    std::vector<hipEvent_t> pool;
    std::vector<std::string> names;
    std::vector<uint64_t> launches;
    std::vector<double> total_ms;

    uint32_t id(const char *name)
    {
        for (uint32_t i = 0; i < names.size(); ++i)
            if (names[i] == name) return i;
        names.emplace_back(name);
        launches.push_back(0);
        total_ms.push_back(0.0);
        return (uint32_t)names.size() - 1;
    }
    hipError_t event(hipEvent_t *e)
    {
        if (!pool.empty()) {
            *e = pool.back();
            pool.pop_back();
            return hipSuccess;
        }
        return hipEventCreate(e);
    }
    ~KernelTimer()
    {
        for (auto &p : pending) {
            (void)hipEventDestroy(p.start);
            (void)hipEventDestroy(p.stop);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

struct amber_pop {
    Resolved r;
    amber_buffers_t b{};
    hipStream_t stream = nullptr;
    int device = 0;
    uint64_t step = 0;
    amber::Tuning tuning;
    DevInvariants *acc = nullptr;      // inside the workspace
    KernelTimer timer;
    uint32_t persist_g = 0, persist_blocks = 0;   // SIR persistent form fit (0 = none)
    // SIR gather-mode early stop: pinned word written by the device (host and
    // device addresses, a slot of the process-wide pool), the number of the
    // last polled call, two poll events (created on first use)
    uint32_t *stop_host = nullptr, *stop_dev = nullptr;
    uint32_t call_seq = 0;
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    bool scratch = false;              // workspace is the device's no-allocation scratch
    ~amber_pop();
};

namespace {
// Pinned, device-mapped host words for the early stop, handed out from 4 KB
// pages of 64 slots (one 64-byte line each).  Pages are kept until the
// process ends; a released handle's slot is reused (its stream has drained).
struct StopWordPool {
    std::mutex mu;
    std::vector<std::pair<uint32_t *, uint32_t *>> free_slots;   // (host, device)
    hipError_t take(uint32_t **host, uint32_t **dev)
    {
        std::lock_guard<std::mutex> lk(mu);
        if (free_slots.empty()) {
            void *page = nullptr, *dpage = nullptr;
            hipError_t e = hipHostMalloc(&page, 4096, hipHostMallocMapped | hipHostMallocCoherent |
                                                          hipHostMallocPortable);
            if (e == hipSuccess) e = hipHostGetDevicePointer(&dpage, page, 0);
            if (e != hipSuccess) return e;
            for (uint32_t k = 0; k < 64; ++k)
                free_slots.emplace_back((uint32_t *)((char *)page + 64 * k),
                                        (uint32_t *)((char *)dpage + 64 * k));
        }
        *host = free_slots.back().first;
        *dev = free_slots.back().second;
        free_slots.pop_back();
        __atomic_store_n(*host, 0u, __ATOMIC_RELEASE);
        return hipSuccess;
    }
    void give(uint32_t *host, uint32_t *dev)
    {
        std::lock_guard<std::mutex> lk(mu);
        free_slots.emplace_back(host, dev);
    }
};
// never destroyed: handles may be released during process teardown
StopWordPool &stop_words()
{
    static StopWordPool *pool = new StopWordPool;
    return *pool;
}
}  // namespace

amber_pop::~amber_pop()
{
    for (hipEvent_t e : poll_ev)
        if (e) (void)hipEventDestroy(e);
    if (stop_host) stop_words().give(stop_host, stop_dev);
}

// The two poll events of a handle, created on its first polled call.
hipError_t poll_events(amber_pop *p)
{
    for (int k = 0; k < 2; ++k)
        if (!p->poll_ev[k]) {
            const hipError_t e = hipEventCreateWithFlags(&p->poll_ev[k], hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

constexpr uint32_t SIR_POLL = 16;      // body launches between early-stop polls
// The gather mode's polls come twice as often: the launches still queued
// when the early stop is seen each cost a launch that does nothing.
constexpr uint32_t SIR_POLL_GATHER = 8;

// sir_poll values: how a long SIR call learns what the device has reached.
// NOWAIT reads the pinned words only when the device has already written
// them (a plain host load of the early-stop word; hipEventQuery before the
// susceptible count of the tiled-then-gather mode) and never waits, so
// amber_step only enqueues.  PACED also waits, every SIR_POLL launches,
// until at most 2 x SIR_POLL launches are queued, so the early stop and the
// mode switch take effect at once; amber_step then blocks for most of the
// call.  OFF reads nothing: one launch per step.
constexpr uint32_t POLL_NOWAIT = 0, POLL_OFF = 1, POLL_PACED = 2;

// Whether work enqueued on st is being captured into a graph (then the host
// cannot wait for it, and nothing is polled).
bool stream_capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return true;
    }
    return cs != hipStreamCaptureStatusNone;
}


namespace {
// The set of live handles and its lock are never destroyed: a handle may be
// released (or a call validated) from another library's teardown at process
// exit, after this library's ordinary static objects would be gone.
std::mutex &g_live_mu = *new std::mutex;
std::unordered_set<const amber_pop *> &g_live = *new std::unordered_set<const amber_pop *>;

bool is_live(const amber_pop *p)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    return p && g_live.count(p);
}

amber_status_t check_device_ptr(const void *p, int device, const char *what, size_t need)
{
    if (!p) return fail(AMBER_E_INVALID, "%s is NULL", what);
    if (((uintptr_t)p & 15u) != 0) return fail(AMBER_E_INVALID, "%s is not 16-byte aligned", what);
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(AMBER_E_INVALID, "%s is not a HIP device pointer", what);
    }
    if (attr.type != hipMemoryTypeDevice)
        return fail(AMBER_E_INVALID, "%s is not device memory", what);
    if (attr.device != device)
        return fail(AMBER_E_INVALID, "%s lives on device %d, current device is %d", what,
                    attr.device, device);
    // The need bytes from p must lie inside the allocation that holds p (the
    // runtime may not know the extent of every kind of allocation: then only
    // the caller's declared sizes stand).
    hipDeviceptr_t base = nullptr;
    size_t extent = 0;
    if (hipMemGetAddressRange(&base, &extent, const_cast<void *>(p)) != hipSuccess) {
        (void)hipGetLastError();
        return AMBER_OK;
    }
    const uint64_t off = (uint64_t)((uintptr_t)p - (uintptr_t)base);
    if ((uintptr_t)p < (uintptr_t)base || off > extent || extent - off < need)
        return fail(AMBER_E_INVALID,
                    "%s has %llu bytes left in its allocation, the run needs %llu", what,
                    (unsigned long long)((uintptr_t)p < (uintptr_t)base || off > extent ? 0 : extent - off),
                    (unsigned long long)need);
    return AMBER_OK;
}

// A device buffer of `need` bytes at p for the view calls: element-aligned
// (`align` bytes), device memory of `device`, inside its allocation where the
// runtime reports the allocation's extent.
amber_status_t check_view_ptr(const void *p, int device, const char *what, uint64_t need,
                              uint32_t align)
{
    if (!p) return fail(AMBER_E_INVALID, "%s is NULL", what);
    if (((uintptr_t)p % align) != 0)
        return fail(AMBER_E_INVALID, "%s is not %u-byte aligned", what, align);
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(AMBER_E_INVALID, "%s is not a HIP device pointer", what);
    }
    if (attr.type != hipMemoryTypeDevice) return fail(AMBER_E_INVALID, "%s is not device memory", what);
    if (attr.device != device)
        return fail(AMBER_E_INVALID, "%s lives on device %d, current device is %d", what,
                    attr.device, device);
    hipDeviceptr_t base = nullptr;
    size_t extent = 0;
    if (hipMemGetAddressRange(&base, &extent, const_cast<void *>(p)) != hipSuccess) {
        (void)hipGetLastError();
        return AMBER_OK;
    }
    const uint64_t off = (uint64_t)((uintptr_t)p - (uintptr_t)base);
    if ((uintptr_t)p < (uintptr_t)base || off > extent || extent - off < need)
        return fail(AMBER_E_INVALID, "%s has fewer than the %llu bytes the call needs", what,
                    (unsigned long long)need);
    return AMBER_OK;
}

// After a synchronisation: report (and clear) the sticky device error word
// that a persistent launch sets when one of its barrier waits gave up.
amber_status_t check_device_flag(amber_pop *p, uint32_t flag)
{
    if (!flag) return AMBER_OK;
    const uint32_t zero = 0;
    HIP_TRY(hipMemcpy((uint8_t *)p->b.workspace + ERR_FLAG_OFFSET, &zero, 4, hipMemcpyHostToDevice),
            "error flag clear");
    if (flag & ERR_TILE_LISTS)
        return fail(AMBER_E_DEVICE, "the tiled SIR mode found its record lists out of range; "
                                    "the run's state is invalid");
    if (flag & ERR_ASYNC_GENERATIONS)
        return fail(AMBER_E_DEVICE, "an asynchronous wealth step did not close its donor set "
                                    "within its generations; the run's state is invalid");
    return fail(AMBER_E_DEVICE, "a device-wide barrier of the persistent SIR form timed out; "
                                "the run's state is invalid");
}

// Record the stop event of the open run of launches, if any.
hipError_t timer_close(amber_pop *p)
{
    KernelTimer &tm = p->timer;
    if (!tm.chain) return hipSuccess;
    tm.chain = false;
    return hipEventRecord(tm.pending.back().stop, p->stream);
}

// Launch one kernel through f(), timed with events when enabled.  A run of
// launches of one kernel shares one pair of events: the start goes before the
// first and the stop after the last, once the run ends.
template <class F>
hipError_t timed(amber_pop *p, const char *name, F &&f)
{
    KernelTimer &tm = p->timer;
    if (!tm.on) return f();
    const uint32_t k = tm.id(name);
    hipError_t e;
    if (tm.chain && !tm.pending.empty() && tm.pending.back().kernel == k) {
        // same kernel again, nothing enqueued in between: extend the open run
        if ((e = f()) != hipSuccess) return e;
        tm.pending.back().count += 1;
        return hipSuccess;
    }
    if ((e = timer_close(p)) != hipSuccess) return e;
    hipEvent_t a, b;
    if ((e = tm.event(&a)) != hipSuccess) return e;
    if ((e = tm.event(&b)) != hipSuccess) return e;
    if ((e = hipEventRecord(a, p->stream)) != hipSuccess) return e;
    tm.pending.push_back({k, 0u, a, b});
    tm.chain = true;
    if ((e = f()) != hipSuccess) return e;
    tm.pending.back().count = 1;
    return hipSuccess;
}

// Untimed work follows (or may follow) on the stream: close the open run, so
// the next timed launch opens a new pair of events.
hipError_t timer_cut(amber_pop *p)
{
    hipError_t e = timer_close(p);
    p->timer.chain = false;
    return e;
}

int32_t *col_i32(amber_pop *p, amber_col_t c) { return (int32_t *)p->b.col[c]; }
uint8_t *ws_ptr(amber_pop *p, uint64_t off) { return (uint8_t *)p->b.workspace + off; }

SirParams sir_params(amber_pop *p, uint32_t t_base)
{
    const Resolved &r = p->r;
    SirParams sp{};
    sp.x = col_i32(p, AMBER_COL_X);
    sp.y = col_i32(p, AMBER_COL_Y);
    sp.s = (uint8_t *)p->b.col[AMBER_COL_STATE];
    for (int b = 0; b < 3; ++b) {
        sp.count[b] = (uint32_t *)ws_ptr(p, r.off_count[b]);
        sp.dmap[b] = ws_ptr(p, r.off_dmap[b]);
    }
    sp.cside = r.cside;
    sp.nsi = (uint32_t *)ws_ptr(p, r.off_nsi);
    sp.t_inf = (const uint32_t *)ws_ptr(p, r.off_table);
    sp.table_len = (uint32_t)r.t_inf.size();
    sp.t_rec = r.t_rec;
    sp.n = r.n;
    sp.L = (int32_t)r.L;
    sp.k0 = r.seed;
    sp.k1 = r.stream;
    sp.t_base = t_base;
    if (r.sx_P) {
        sp.xrec = (uint32_t *)ws_ptr(p, r.off_sxrec);
        sp.xtab = (uint32_t *)ws_ptr(p, r.off_sxtab);
        sp.xh = r.sx_h;
        sp.xP = r.sx_P;
        sp.xW = r.sx_W;
    }
    return sp;
}

// SIR neighbour-count mode of the pipelined form: 1 gather, 2 box, 3 exchange,
// 4 tiled, 5 tiled until few susceptible agents remain, then gather.
// Automatic choice for grids that fit in the last-level cache: the 3x3
// gathers.  Beyond it every gathered cell and every binning atomic costs its
// own memory line: the box mode then (one read per agent instead of nine),
// and inside a plain call the tiled mode ahead of both (no random access).
// A call of SIR_AUTO_LONG_CALL steps or more on a grid of more than
// SIR_AUTO_SWITCH_CELLS cells starts tiled and moves to the gather mode once
// few susceptible agents are left: from then on the demand-driven binning
// and the launch that runs the steps left once none remains make the gather
// steps the cheaper ones.  500-step runs, all gather against tiled then
// gather: 2.89 / 3.27 ms at 1e6 agents (L = 1000), 5.70 / 5.56 ms at 2e6,
// 8.99 / 7.94 ms at 3e6, 53.9 / 38.8 ms at 1.6e7, 0.543 / 0.296 s at 2^27.
constexpr uint32_t SIR_AUTO_LONG_CALL = 128;
constexpr uint64_t SIR_AUTO_SWITCH_CELLS = 2ull << 20;
// A tiled call pays a sort of the columns into records and a scatter back
// (about 19 ms at 2^27 agents, against 1.8 ms saved per step over the box
// mode), so on big grids calls of fewer steps stay in the box mode.
constexpr uint32_t SIR_AUTO_TILED_CALL = 16;

uint32_t sir_auto_count_mode(const amber_pop *p, uint32_t n_steps)
{
    const uint64_t cells = (uint64_t)p->r.L * p->r.L;
    // the switch needs the host to see the susceptible count while the call
    // is still being enqueued, which only the paced poll guarantees: an
    // unpaced call is enqueued long before its first poll has run, and
    // would stay tiled
    if (n_steps >= SIR_AUTO_LONG_CALL)
        return cells > SIR_AUTO_SWITCH_CELLS && p->tuning.sir_poll == POLL_PACED ? 5u : 1u;
    return cells > (16ull << 20) ? 2u : 1u;
}

uint32_t sir_tile_side(const amber_pop *p);

// Tile side of the tiled mode for this run (0 when it does not fit).
uint32_t sir_tile_side(const amber_pop *p)
{
    const uint32_t want = p->tuning.sir_tile ? p->tuning.sir_tile : TILE_MIN;
    const uint32_t nt = sir_tile_count(p->r.L, want);
    if (!nt || !p->r.tile_tiles) return 0;
    const uint64_t rs = 4ull * want + 8;
    const uint64_t tiles = (uint64_t)nt * nt;
    if (tiles > p->r.tile_tiles || tiles * rs > sir_tile_ring_words(p->r.L) ||
        tiles * sir_tile_cap(p->r.n, (uint32_t)tiles) + p->r.n > p->r.tile_rec)
        return 0;
    return want;
}

uint32_t sir_count_mode(const amber_pop *p, uint32_t n_steps)
{
    const uint32_t want = p->tuning.sir_count;
    if (want == 3) return p->r.sx_P ? 3u : 0u;    // 0: unavailable, caller reports it
    if (want == 4 || want == 5) return sir_tile_side(p) ? want : 0u;
    if (want == 1 || want == 2) return want;
    const uint32_t m = sir_auto_count_mode(p, n_steps);
    if (m == 2) return sir_tile_side(p) && n_steps >= SIR_AUTO_TILED_CALL ? 4u : 2u;
    if (m == 5) return sir_tile_side(p) ? 5u : 1u;
    return m;
}

// Count mode of a run inside amber_step_batch (the batched kernels have the
// gather, box and exchange modes): the tiled modes become box for short
// calls on big grids and gather otherwise.
uint32_t sir_batch_count_mode(const amber_pop *p, uint32_t n_steps)
{
    const uint32_t m = sir_count_mode(p, n_steps);
    if (m == 4 || m == 5) return sir_auto_count_mode(p, n_steps) == 2 ? 2u : 1u;
    return m == 0 ? 1u : m;     // exchange requested but unavailable: gather
}

TileParams tile_params(amber_pop *p, uint32_t T)
{
    const Resolved &r = p->r;
    TileParams tp{};
    tp.x = col_i32(p, AMBER_COL_X);
    tp.y = col_i32(p, AMBER_COL_Y);
    tp.s = (uint8_t *)p->b.col[AMBER_COL_STATE];
    tp.t_inf = (const uint32_t *)ws_ptr(p, r.off_table);
    tp.table_len = (uint32_t)r.t_inf.size();
    tp.t_rec = r.t_rec;
    tp.n = r.n;
    tp.k0 = r.seed;
    tp.k1 = r.stream;
    tp.L = (int32_t)r.L;
    tp.T = T;
    tp.tshift = T == 64 ? 6u : 5u;
    tp.nT = sir_tile_count(r.L, T);
    tp.rs = 4 * T + 8;
    tp.cap = sir_tile_cap(r.n, tp.nT * tp.nT);
    tp.ovf0 = tp.nT * tp.nT * tp.cap;
    for (int b = 0; b < 2; ++b) {
        tp.rec[b] = (uint2 *)ws_ptr(p, r.off_trec[b]);
        tp.hdr[b] = (uint32_t *)ws_ptr(p, r.off_thdr[b]);
        tp.C[b] = (uint32_t *)ws_ptr(p, r.off_count[b]);
        tp.ring[b] = (uint32_t *)ws_ptr(p, r.off_tring[b]);
    }
    tp.cursor = (uint32_t *)ws_ptr(p, r.off_tcur);
    tp.ctr = (uint32_t *)ws_ptr(p, r.off_tctr);
    tp.err = (uint32_t *)ws_ptr(p, ERR_FLAG_OFFSET);
    return tp;
}

// Threads per tile workgroup: the tuned block, raised so that a tile of
// average occupancy plus a margin fits one round of 8 records per thread.
uint32_t tile_block(const amber_pop *p, const TileParams &tp)
{
    const uint64_t tiles = (uint64_t)tp.nT * tp.nT;
    const uint64_t want = (p->r.n * 5ull / 4 + tiles - 1) / tiles / 8 + 1;
    uint32_t b = 64;
    while (b < want && b < 1024) b *= 2;
    return std::max(b, p->tuning.block);
}

// SIR steps t0 .. t0 + n_steps - 1 of the pipelined form in the gather mode.
amber_status_t enqueue_sir_gather(amber_pop *p, uint32_t t0, uint32_t n_steps)
{
    const Tuning &tu = p->tuning;
    hipStream_t st = p->stream;
    SirParams sp = sir_params(p, t0);
    sp.t_last = t0 + n_steps - 1;
    // Early stop: once no susceptible agent is left, one body launch
    // runs the call's remaining steps and announces it in a pinned
    // word; the later launches would do nothing.  Every SIR_POLL_GATHER
    // launches the host reads the word (PACED: after waiting until at
    // most 2 x SIR_POLL_GATHER launches are queued) and stops enqueueing
    // once it holds this call's number.  Results do not depend on where it
    // stops.
    const bool watch = tu.sir_poll != POLL_OFF && p->stop_host &&
                       n_steps > 2 * SIR_POLL_GATHER && !stream_capturing(st);
    const bool paced = watch && tu.sir_poll == POLL_PACED;
    if (watch) {
        if (paced) HIP_TRY(poll_events(p), "poll events");
        if (++p->call_seq == 0) ++p->call_seq;
        sp.stop_word = p->stop_dev;
        sp.stop_seq = p->call_seq;
    }
    HIP_TRY(timed(p, "sir_head", [&] { return launch_sir_head(sp, t0, false, tu, st); }),
            "sir head kernel");
    uint32_t last = n_steps - 1;
    for (uint32_t i = 1; i < n_steps; ++i) {
        HIP_TRY(timed(p, "sir_body",
                      [&] { return launch_sir_body(sp, t0 + i, false, tu, st); }),
                "sir body kernel");
        if (!watch || i % SIR_POLL_GATHER != 0) continue;
        if (paced) {
            const uint32_t k = i / SIR_POLL_GATHER;
            HIP_TRY(hipEventRecord(p->poll_ev[k & 1], st), "poll event record");
            if (k < 2) continue;
            HIP_TRY(hipEventSynchronize(p->poll_ev[(k - 1) & 1]), "poll event synchronize");
        }
        if (__atomic_load_n(p->stop_host, __ATOMIC_ACQUIRE) == p->call_seq) {
            last = i;
            break;
        }
    }
    HIP_TRY(timed(p, "sir_tail",
                  [&] { return launch_sir_tail(sp, t0 + n_steps - 1, last, false, tu, st); }),
            "sir tail kernel");
    HIP_TRY(timed(p, "sir_clear",
                  [&] { return launch_sir_clear(sp, 1u << ((n_steps - 1) % 3), st); }),
            "sir clear kernel");
    return AMBER_OK;
}

// Fraction of susceptible agents at or below which a tiled-then-gather call
// moves to the gather mode: S * SIR_SWITCH_DIV <= N, read one poll (16
// steps) late.  At 2^27 agents the switch then lands where S is near N / 20,
// about where a gather-mode step (nine gathers per susceptible agent,
// demand-driven binning on coarse and fine maps) becomes cheaper than a
// tiled step (every agent sorted).
constexpr uint32_t SIR_SWITCH_DIV = 4;

// SIR steps t0 .. t0 + n_steps - 1 in the tiled mode: sort, head, bodies,
// tail, then the two count grids back to zero.  With may_switch the bodies
// also count the susceptible agents per tile; every SIR_POLL body launches
// a one-workgroup kernel sums them into the handle's pinned words, and the
// host reads the sum of the previous poll.  Once S * SIR_SWITCH_DIV <= N it
// ends the tiled segment there (the tail writes the columns back) and
// reports in *done how many steps the segment covered; the caller runs the
// rest in the gather mode.  Results do not depend on where it switches.
amber_status_t enqueue_sir_tiled(amber_pop *p, uint32_t t0, uint32_t n_steps, bool may_switch,
                                 uint32_t *done)
{
    const Resolved &r = p->r;
    hipStream_t st = p->stream;
    const bool poll = may_switch && p->tuning.sir_poll != POLL_OFF && p->stop_host &&
                      n_steps > 2 * SIR_POLL && !stream_capturing(st);
    const bool paced = p->tuning.sir_poll == POLL_PACED;
    TileParams tp = tile_params(p, sir_tile_side(p));
    if (poll) {
        HIP_TRY(poll_events(p), "poll events");
        tp.scnt = (uint32_t *)ws_ptr(p, r.off_tscnt);
    }
    const uint32_t blk = tile_block(p, tp);
    HIP_TRY(timed(p, "sir_tile_sort", [&] { return launch_sir_tile_sort(tp, st); }),
            "sir tile sort kernels");
    HIP_TRY(timed(p, "sir_tile_head", [&] { return launch_sir_tile_step(tp, t0, 0, n_steps, blk, st); }),
            "sir tile step kernel");
    uint32_t k = n_steps;                        // steps of the tiled segment
    for (uint32_t i = 1; i < n_steps; ++i) {
        HIP_TRY(timed(p, "sir_tile_body",
                      [&] { return launch_sir_tile_step(tp, t0, i, n_steps, blk, st); }),
                "sir tile step kernel");
        if (!poll || i % SIR_POLL != 0 || i + 1 >= n_steps) continue;
        const uint32_t q = i / SIR_POLL;
        uint32_t *sum_dev = p->stop_dev + 1 + (q & 1);       // words 1 and 2 of the slot
        HIP_TRY(timed(p, "sir_tile_count",
                      [&] { return launch_sum_words(tp.scnt, tp.nT * tp.nT, sum_dev, st); }),
                "sir tile count kernel");
        HIP_TRY(hipEventRecord(p->poll_ev[q & 1], st), "poll event record");
        if (q < 2) continue;
        if (paced) {
            HIP_TRY(hipEventSynchronize(p->poll_ev[(q - 1) & 1]), "poll event synchronize");
        } else {
            // the previous poll's sum only if the device has already written it
            const hipError_t e = hipEventQuery(p->poll_ev[(q - 1) & 1]);
            if (e == hipErrorNotReady) {
                (void)hipGetLastError();
                continue;
            }
            HIP_TRY(e, "poll event query");
        }
        const uint32_t sus = __atomic_load_n(p->stop_host + 1 + ((q - 1) & 1), __ATOMIC_ACQUIRE);
        if ((uint64_t)sus * SIR_SWITCH_DIV <= r.n) {
            k = i + 1;
            break;
        }
    }
    if (k < n_steps) {
        // the gather segment's head bins on marks the column write-back
        // makes (see k_tile_unpack and sir_demand_book)
        const SirParams sp = sir_params(p, t0 + k);
        tp.mark = sp.dmap[0];
        tp.mark_cside = sp.cside;
        const uint64_t cells = (uint64_t)r.L * r.L;
        tp.mark_coarse = sp.dmap[0] + ((cells + 255) & ~255ull);
        tp.mark_t = t0 + k;
        tp.mark_flags = sp.nsi + NSI_FLAGS;
    }
    HIP_TRY(timed(p, "sir_tile_tail", [&] { return launch_sir_tile_step(tp, t0, k, k, blk, st); }),
            "sir tile step kernel");
    // the two count grids it used go back to zero, as the other modes expect
    const uint64_t words = (r.off_count[2] - r.off_count[0]) / 4;
    HIP_TRY(timed(p, "sir_clear", [&] { return launch_zero_words(tp.C[0], words, st); }),
            "sir clear kernel");
    *done = k;
    return AMBER_OK;
}

// SIR steps t0 .. t0 + n_steps - 1 in the form and count mode the tuning
// (or the automatic choice) selects.
amber_status_t enqueue_sir(amber_pop *p, uint32_t t0, uint32_t n_steps)
{
    const Resolved &r = p->r;
    hipStream_t st = p->stream;
    const Tuning &tu = p->tuning;
    const uint32_t mode = sir_count_mode(p, n_steps);
    SirParams sp = sir_params(p, t0);
    sp.t_last = t0 + n_steps - 1;
    // Automatic choice: the pipelined form.  The persistent form keeps the
    // state in registers but pays a device-wide barrier per step, which on
    // gfx950 costs more than the launch it saves; it runs only on request.
    uint32_t g = 0, blocks = 0;
    if (tu.sir_form == 2) {
        if (tu.max_g >= 8) {
            g = p->persist_g;
            blocks = p->persist_blocks;
        } else {
            g = sir_persistent_groups_per_thread(r.n, tu.max_g, &blocks);
        }
        if (g == 0)
            return fail(AMBER_E_UNSUPPORTED,
                        "the persistent SIR form does not fit %u agents on this device", r.n);
    }
    if (g) {
        uint32_t *sync_words = (uint32_t *)ws_ptr(p, r.off_sync);
        uint32_t *err = (uint32_t *)ws_ptr(p, ERR_FLAG_OFFSET);
        HIP_TRY(timed(p, "sir_persistent",
                      [&] {
                          return launch_sir_persistent(sp, sync_words, err, t0, n_steps, g,
                                                       blocks, st);
                      }),
                "sir persistent kernel");
        HIP_TRY(timed(p, "sir_clear",
                      [&] { return launch_sir_clear(sp, 1u << ((n_steps - 1) % 3), st); }),
                "sir clear kernel");
    } else if (tu.sir_count == 3 && !r.sx_P) {
        return fail(AMBER_E_UNSUPPORTED, "the exchange count mode does not fit this run "
                                         "(grid side %u, %u agents)", r.L, r.n);
    } else if (tu.sir_count == 4 && !sir_tile_side(p)) {
        return fail(AMBER_E_UNSUPPORTED, "the tiled count mode needs a grid side of at least "
                                         "2 x tile + 2 (grid side %u, tile %u)",
                    r.L, tu.sir_tile ? tu.sir_tile : TILE_MIN);
    } else if (tu.sir_count == 5 && !sir_tile_side(p)) {
        return fail(AMBER_E_UNSUPPORTED, "the tiled-then-gather count mode needs a grid side of "
                                         "at least 2 x tile + 2 (grid side %u, tile %u)",
                    r.L, tu.sir_tile ? tu.sir_tile : TILE_MIN);
    } else if (mode == 4 || mode == 5) {
        uint32_t done = 0;
        const amber_status_t rc = enqueue_sir_tiled(p, t0, n_steps, mode == 5, &done);
        if (rc != AMBER_OK || done == n_steps) return rc;
        return enqueue_sir_gather(p, t0 + done, n_steps - done);
    } else if (mode == 3) {
        HIP_TRY(timed(p, "sir_xbody", [&] { return launch_sir_xbody(sp, t0, false, st); }),
                "sir exchange body kernel");
        HIP_TRY(timed(p, "sir_xcount", [&] { return launch_sir_xcount(sp, st); }),
                "sir exchange count kernel");
        for (uint32_t i = 1; i < n_steps; ++i) {
            HIP_TRY(timed(p, "sir_xbody",
                          [&] { return launch_sir_xbody(sp, t0 + i, true, st); }),
                    "sir exchange body kernel");
            HIP_TRY(timed(p, "sir_xcount", [&] { return launch_sir_xcount(sp, st); }),
                    "sir exchange count kernel");
        }
        HIP_TRY(timed(p, "sir_tail_box",
                      [&] { return launch_sir_tail(sp, t0 + n_steps - 1, n_steps - 1, true, tu, st); }),
                "sir tail kernel");
        HIP_TRY(timed(p, "sir_clear",
                      [&] { return launch_sir_clear(sp, 4u, st); }),
                "sir clear kernel");
    } else if (mode == 2) {
        HIP_TRY(timed(p, "sir_head", [&] { return launch_sir_head(sp, t0, true, tu, st); }),
                "sir head kernel");
        HIP_TRY(timed(p, "sir_box", [&] { return launch_sir_box(sp, t0, st); }),
                "sir box kernel");
        for (uint32_t i = 1; i < n_steps; ++i) {
            HIP_TRY(timed(p, "sir_body_box",
                          [&] { return launch_sir_body(sp, t0 + i, true, tu, st); }),
                    "sir body kernel");
            HIP_TRY(timed(p, "sir_box", [&] { return launch_sir_box(sp, t0 + i, st); }),
                    "sir box kernel");
        }
        HIP_TRY(timed(p, "sir_tail_box",
                      [&] { return launch_sir_tail(sp, t0 + n_steps - 1, n_steps - 1, true, tu, st); }),
                "sir tail kernel");
        HIP_TRY(timed(p, "sir_clear",
                      [&] { return launch_sir_clear(sp, (1u << ((n_steps - 1) & 1)) | 4u, st); }),
                "sir clear kernel");
    } else {
        return enqueue_sir_gather(p, t0, n_steps);
    }
    return AMBER_OK;
}

amber_status_t enqueue_steps(amber_pop *p, uint32_t n_steps)
{
    const Resolved &r = p->r;
    const uint32_t t0 = (uint32_t)p->step;
    hipStream_t st = p->stream;
    const Tuning &tu = p->tuning;
    if (r.model == AMBER_RANDOM_WALK) {
        int32_t *x = col_i32(p, AMBER_COL_X), *y = col_i32(p, AMBER_COL_Y);
        HIP_TRY(timed(p, "walk", [&] {
                    return launch_walk(x, y, r.n, (int32_t)r.L, r.seed, r.stream, t0, n_steps, tu,
                                       st);
                }),
                "walk kernel");
    } else if (r.model == AMBER_WEALTH) {
        int32_t *w = col_i32(p, AMBER_COL_WEALTH);
        const bool exchange = r.xbits != 0 && tu.wealth_form != 1;
        const uint32_t wide = tu.wealth_form == 3 ? 4u : 0u;    // the 32-bit fold throughout
        if (tu.wealth_form >= 2 && !exchange)
            return fail(AMBER_E_UNSUPPORTED, "the partition-exchange wealth path does not cover "
                                             "%u agents", r.n);
        if (r.n <= wealth_small_max_agents()) {
            HIP_TRY(timed(p, "wealth_small", [&] {
                        return launch_wealth_small(w, r.n, r.seed, r.stream, t0, n_steps, st);
                    }),
                    "wealth small kernel");
        } else if (exchange) {
            WealthXParams x;
            x.w = w;
            for (int b = 0; b < 2; ++b) {
                x.rec[b] = (uint32_t *)ws_ptr(p, r.off_xrec[b]);
                x.tab[b] = (uint32_t *)ws_ptr(p, r.off_xtab[b]);
            }
            x.n = r.n;
            x.P = r.xparts;
            x.k0 = r.seed;
            x.k1 = r.stream;
            for (uint32_t i = 0; i < n_steps; ++i)
                HIP_TRY(timed(p, "wealth_exchange", [&] {
                            return launch_wealth_exchange(x, t0 + i, (i + 1) & 1u,
                                                          (i ? 3u : 2u) | wide, r.xbits, st);
                        }),
                        "wealth exchange kernel");
            HIP_TRY(timed(p, "wealth_exchange_fold", [&] {
                        return launch_wealth_exchange(x, t0 + n_steps, (n_steps - 1) & 1u,
                                                      1u | wide, r.xbits, st);
                    }),
                    "wealth exchange fold kernel");
        } else {
            int32_t *inc[2] = {(int32_t *)ws_ptr(p, r.off_inc0), (int32_t *)ws_ptr(p, r.off_inc1)};
            for (uint32_t i = 0; i < n_steps; ++i)
                HIP_TRY(timed(p, "wealth_step", [&] {
                            return launch_wealth_step(w, inc[i & 1], inc[(i + 1) & 1], r.n, r.seed,
                                                      r.stream, t0 + i, tu, st);
                        }),
                        "wealth step kernel");
            HIP_TRY(timed(p, "wealth_fold",
                          [&] { return launch_wealth_fold(w, inc[n_steps & 1], r.n, st); }),
                    "wealth fold kernel");
        }
    } else {
        return enqueue_sir(p, t0, n_steps);
    }
    return AMBER_OK;
}

// Join the streams of the batch's handles onto the first handle's stream
// (before) or the first stream onto the others (after).
amber_status_t join_streams(amber_pop *const *pops, uint32_t n, bool before)
{
    hipStream_t main = pops[0]->stream;
    std::vector<hipStream_t> others;
    for (uint32_t i = 1; i < n; ++i)
        if (pops[i]->stream != main &&
            std::find(others.begin(), others.end(), pops[i]->stream) == others.end())
            others.push_back(pops[i]->stream);
    for (hipStream_t o : others) {
        hipEvent_t ev;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
        hipError_t e = hipEventRecord(ev, before ? o : main);
        if (e == hipSuccess) e = hipStreamWaitEvent(before ? main : o, ev, 0);
        (void)hipEventDestroy(ev);
        if (e != hipSuccess) return hip_fail(e, "stream join");
    }
    return AMBER_OK;
}

// SIR gather-mode runs of a batch, enqueued step by step: each step is one
// body launch per pack of at most BATCH_RUNS active runs.  With polling,
// every SIR_POLL steps the host waits until at most 2 x SIR_POLL steps are
// queued, and a run whose launch running its remaining steps has started
// (its pinned word holds its call number) leaves the later launches: the
// active runs are packed again.  Each run's tail checks the flag of the last
// body launch that held it.  Results do not depend on when a run leaves.
amber_status_t run_sir_gather_batch(amber_pop *lead, const std::vector<amber_pop *> &runs,
                                    uint32_t n_steps, uint32_t block, hipStream_t st)
{
    const uint32_t R = (uint32_t)runs.size();
    std::vector<SirParams> prm(R);
    std::vector<uint32_t> t0(R), seq(R, 0), i_last(R, n_steps - 1);
    bool poll = n_steps > 2 * SIR_POLL && !stream_capturing(st);
    bool paced = true;
    for (amber_pop *p : runs) {
        poll = poll && p->stop_host && p->tuning.sir_poll != POLL_OFF;
        paced = paced && p->tuning.sir_poll == POLL_PACED;
    }
    for (uint32_t r = 0; r < R; ++r) {
        amber_pop *p = runs[r];
        prm[r] = sir_params(p, (uint32_t)p->step);
        sir_fill(prm[r]);
        t0[r] = (uint32_t)p->step;
        prm[r].t_last = t0[r] + n_steps - 1;
        if (poll) {
            if (++p->call_seq == 0) ++p->call_seq;
            seq[r] = p->call_seq;
            prm[r].stop_word = p->stop_dev;
            prm[r].stop_seq = seq[r];
        }
    }
    // packs of at most BATCH_RUNS runs (one more workgroup per run for the
    // demand-binning bookkeeping)
    auto make_packs = [&](const std::vector<uint32_t> &idx) {
        std::vector<SirBatch> packs;
        for (size_t c = 0; c < idx.size(); c += BATCH_RUNS) {
            SirBatch b{};
            uint32_t blocks = 0, cblocks = 0;
            for (size_t k = c; k < idx.size() && k < c + BATCH_RUNS; ++k) {
                const uint32_t r = idx[k], j = b.nruns++;
                b.run[j] = prm[r];
                b.t0[j] = t0[r];
                b.i_last[j] = i_last[r];
                blocks += (groups_of_host(runs[r]->r.n) + block - 1) / block + 1;
                b.block_end[j] = blocks;
                cblocks += (prm[r].quads + 255) / 256;
                b.cell_block_end[j] = cblocks;
            }
            packs.push_back(b);
        }
        return packs;
    };
    std::vector<uint32_t> all(R), active;
    for (uint32_t r = 0; r < R; ++r) all[r] = r;
    active = all;
    auto launch_packs = [&](const std::vector<SirBatch> &packs, uint32_t phase, uint32_t i) {
        for (const SirBatch &b : packs) {
            hipError_t e = launch_sir_gather_batch(b, phase, i, n_steps, block, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    if (poll && paced) {
        const hipError_t e = poll_events(runs[0]);
        if (e != hipSuccess) return hip_fail(e, "poll events");
    }
    hipEvent_t *ev = runs[0]->poll_ev;
    auto steps = [&]() -> hipError_t {
        hipError_t e = launch_packs(make_packs(all), 0, 0);
        std::vector<SirBatch> packs = make_packs(active);
        for (uint32_t i = 1; i < n_steps && e == hipSuccess && !active.empty(); ++i) {
            e = launch_packs(packs, 1, i);
            if (e != hipSuccess || !poll || i % SIR_POLL != 0) continue;
            if (paced) {
                const uint32_t k = i / SIR_POLL;
                if ((e = hipEventRecord(ev[k & 1], st)) != hipSuccess || k < 2) continue;
                if ((e = hipEventSynchronize(ev[(k - 1) & 1])) != hipSuccess) break;
            }
            std::vector<uint32_t> still;
            for (uint32_t r : active) {
                if (__atomic_load_n(runs[r]->stop_host, __ATOMIC_ACQUIRE) == seq[r]) i_last[r] = i;
                else still.push_back(r);
            }
            if (still.size() != active.size()) {
                active.swap(still);
                packs = make_packs(active);
            }
        }
        if (e == hipSuccess) e = launch_packs(make_packs(all), 2, 0);   // with the runs' i_last
        if (e == hipSuccess) e = launch_packs(make_packs(all), 3, 0);
        return e;
    };
    HIP_TRY(timed(lead, "sir_batch", steps), "sir batch kernels");
    return AMBER_OK;
}

amber_status_t run_batch(amber_pop *const *pops, uint32_t n, uint32_t n_steps)
{
    amber_pop *lead = pops[0];
    hipStream_t st = lead->stream;
    const uint32_t block = lead->tuning.block;
    amber_status_t rc = join_streams(pops, n, true);
    if (rc != AMBER_OK) return rc;

    // partition-exchange runs grouped by partition size (2^15 partitions use
    // the atomic kernels inside a batch; results are the same)
    const uint32_t xsizes[3] = {11, 12, 14};
    std::vector<amber_pop *> walk, wealth_small, wealth_big, wealth_x[3], sir;
    for (uint32_t i = 0; i < n; ++i) {
        amber_pop *p = pops[i];
        if (p->r.model == AMBER_RANDOM_WALK) walk.push_back(p);
        else if (p->r.model == AMBER_SIR) sir.push_back(p);
        else if (p->r.n <= wealth_small_max_agents()) wealth_small.push_back(p);
        else {
            int k = 0;
            while (k < 3 && (p->tuning.wealth_form == 1 || p->r.xbits != xsizes[k])) ++k;
            if (k < 3) wealth_x[k].push_back(p);
            else wealth_big.push_back(p);
        }
    }
    for (int which = 0; which < 3; ++which) {
        const std::vector<amber_pop *> &runs = wealth_x[which];
        const uint32_t bits = xsizes[which];
        for (size_t c = 0; c < runs.size(); c += BATCH_RUNS) {
            WealthXBatch b{};
            uint32_t blocks = 0;
            for (size_t k = c; k < runs.size() && k < c + BATCH_RUNS; ++k) {
                amber_pop *p = runs[k];
                const uint32_t j = b.nruns++;
                WealthXParams &x = b.run[j];
                x.w = col_i32(p, AMBER_COL_WEALTH);
                for (int pb = 0; pb < 2; ++pb) {
                    x.rec[pb] = (uint32_t *)ws_ptr(p, p->r.off_xrec[pb]);
                    x.tab[pb] = (uint32_t *)ws_ptr(p, p->r.off_xtab[pb]);
                }
                x.n = p->r.n;
                x.P = p->r.xparts;
                x.k0 = p->r.seed;
                x.k1 = p->r.stream;
                b.t0[j] = (uint32_t)p->step;
                blocks += x.P;
                b.block_end[j] = blocks;
            }
            HIP_TRY(timed(lead, "wealth_exchange_batch",
                          [&] { return launch_wealth_exchange_batch(b, n_steps, bits, st); }),
                    "wealth exchange batch kernels");
        }
    }
    auto blocks_for = [&](uint32_t agents) { return (groups_of_host(agents) + block - 1) / block; };

    for (size_t c = 0; c < walk.size(); c += BATCH_RUNS) {
        WalkBatch b{};
        uint32_t blocks = 0;
        for (size_t k = c; k < walk.size() && k < c + BATCH_RUNS; ++k) {
            amber_pop *p = walk[k];
            const uint32_t j = b.nruns++;
            b.x[j] = col_i32(p, AMBER_COL_X);
            b.y[j] = col_i32(p, AMBER_COL_Y);
            b.n[j] = p->r.n;
            b.L[j] = (int32_t)p->r.L;
            b.k0[j] = p->r.seed;
            b.k1[j] = p->r.stream;
            b.t0[j] = (uint32_t)p->step;
            blocks += blocks_for(p->r.n);
            b.block_end[j] = blocks;
        }
        HIP_TRY(timed(lead, "walk_batch", [&] { return launch_walk_batch(b, n_steps, block, st); }),
                "walk batch kernel");
    }
    for (size_t c = 0; c < wealth_small.size(); c += BATCH_SMALL_RUNS) {
        WealthSmallBatch b{};
        for (size_t k = c; k < wealth_small.size() && k < c + BATCH_SMALL_RUNS; ++k) {
            amber_pop *p = wealth_small[k];
            const uint32_t j = b.nruns++;
            b.w[j] = col_i32(p, AMBER_COL_WEALTH);
            b.n[j] = p->r.n;
            b.k0[j] = p->r.seed;
            b.k1[j] = p->r.stream;
            b.t0[j] = (uint32_t)p->step;
        }
        HIP_TRY(timed(lead, "wealth_small_batch",
                      [&] { return launch_wealth_small_batch(b, n_steps, st); }),
                "wealth small batch kernel");
    }
    for (size_t c = 0; c < wealth_big.size(); c += BATCH_RUNS) {
        WealthBatch b{};
        uint32_t blocks = 0;
        for (size_t k = c; k < wealth_big.size() && k < c + BATCH_RUNS; ++k) {
            amber_pop *p = wealth_big[k];
            const uint32_t j = b.nruns++;
            b.base[j] = col_i32(p, AMBER_COL_WEALTH);
            b.inc[0][j] = (int32_t *)ws_ptr(p, p->r.off_inc0);
            b.inc[1][j] = (int32_t *)ws_ptr(p, p->r.off_inc1);
            b.n[j] = p->r.n;
            b.k0[j] = p->r.seed;
            b.k1[j] = p->r.stream;
            b.t0[j] = (uint32_t)p->step;
            blocks += blocks_for(p->r.n);
            b.block_end[j] = blocks;
        }
        HIP_TRY(timed(lead, "wealth_batch",
                      [&] { return launch_wealth_batch(b, n_steps, block, st); }),
                "wealth batch kernels");
    }
    // SIR runs of the gather mode go step by step; box and exchange runs in
    // chunks of one count mode each
    {
        std::vector<amber_pop *> runs;
        for (amber_pop *p : sir)
            if (sir_batch_count_mode(p, n_steps) == 1) runs.push_back(p);
        if (!runs.empty()) {
            rc = run_sir_gather_batch(lead, runs, n_steps, block, st);
            if (rc != AMBER_OK) return rc;
        }
    }
    for (uint32_t mode = 2; mode <= 3; ++mode) {
        std::vector<amber_pop *> runs;
        for (amber_pop *p : sir) {
            if (sir_batch_count_mode(p, n_steps) == mode) runs.push_back(p);
        }
        for (size_t c = 0; c < runs.size(); c += BATCH_RUNS) {
            SirBatch b{};
            uint32_t blocks = 0, cblocks = 0, xblocks = 0, bands = 0;
            for (size_t k = c; k < runs.size() && k < c + BATCH_RUNS; ++k) {
                amber_pop *p = runs[k];
                const uint32_t j = b.nruns++;
                b.run[j] = sir_params(p, (uint32_t)p->step);
                sir_fill(b.run[j]);
                b.t0[j] = (uint32_t)p->step;
                b.run[j].t_last = b.t0[j] + n_steps - 1;
                b.i_last[j] = n_steps - 1;
                blocks += blocks_for(p->r.n);
                b.block_end[j] = blocks;
                cblocks += (b.run[j].quads + 255) / 256;
                b.cell_block_end[j] = cblocks;
                xblocks += b.run[j].xW;
                b.xblock_end[j] = xblocks;
                bands += b.run[j].xP;
                b.band_end[j] = bands;
            }
            HIP_TRY(timed(lead, "sir_batch",
                          [&] { return launch_sir_batch(b, n_steps, mode, block, st); }),
                    "sir batch kernels");
        }
    }
    return join_streams(pops, n, false);
}

}  // namespace

// ------------------------------------------------------------------ ABI

static_assert(NOALLOC_SCRATCH_BYTES == AMBER_NOALLOC_SCRATCH_BYTES,
              "the scratch size in the header and in the library agree");

namespace {
// Devices whose no-allocation scratch is held by a live handle.
bool g_scratch_held[NOALLOC_MAX_DEVICES] = {};

// amber_init_population, and its no-allocation variant: with noalloc the
// workspace is the device's scratch array instead of bufs->workspace, the
// handle takes no pinned early-stop word (the SIR early stop and the
// tiled-then-gather switch are then off, results unchanged), and at most one
// such handle per device may be live.
// A resumed run's host columns must hold a state of the model's domain:
// wealth non-negative with a sum below 2^31 (so no agent can overflow),
// coordinates on the grid (the kernels address the count grid with them),
// state codes 0, 1 or 2.
amber_status_t check_host_columns(const Resolved &r, const void *const *host)
{
    static const char *names[AMBER_NUM_COLS] = {"wealth", "x", "y", "state"};
    for (int c = 0; c < AMBER_NUM_COLS; ++c)
        if (column_bytes(r, (amber_col_t)c) != 0 && !host[c])
            return fail(AMBER_E_INVALID, "host %s column is NULL", names[c]);
    if (r.model == AMBER_WEALTH) {
        const int32_t *w = (const int32_t *)host[AMBER_COL_WEALTH];
        int64_t sum = 0;
        for (uint32_t a = 0; a < r.n; ++a) {
            if (w[a] < 0) return fail(AMBER_E_INVALID, "host wealth of agent %u is negative", a);
            sum += w[a];
        }
        if (sum > INT32_MAX)
            return fail(AMBER_E_INVALID, "host wealth sums to %lld, above 2^31-1", (long long)sum);
        return AMBER_OK;
    }
    for (int c = AMBER_COL_X; c <= AMBER_COL_Y; ++c) {
        const int32_t *v = (const int32_t *)host[c];
        for (uint32_t a = 0; a < r.n; ++a)
            if (v[a] < 0 || (uint32_t)v[a] >= r.L)
                return fail(AMBER_E_INVALID, "host %s of agent %u is %d, off the %u-cell grid",
                            names[c], a, v[a], r.L);
    }
    if (r.model == AMBER_SIR) {
        const uint8_t *s = (const uint8_t *)host[AMBER_COL_STATE];
        for (uint32_t a = 0; a < r.n; ++a)
            if (s[a] > 2) return fail(AMBER_E_INVALID, "host state of agent %u is %u", a, s[a]);
    }
    return AMBER_OK;
}

amber_status_t init_population(const amber_run_desc_t *desc, const amber_buffers_t *bufs,
                               void *hip_stream, amber_pop_t **out, bool noalloc,
                               const void *const *host_cols = nullptr, uint64_t t0 = 0)
{
    if (!out) return fail(AMBER_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!bufs) return fail(AMBER_E_INVALID, "buffers are NULL");
    Resolved r;
    amber_status_t st = resolve(desc, r, true);
    if (st != AMBER_OK) return st;
    static const char *names[AMBER_NUM_COLS] = {"wealth column", "x column", "y column",
                                                "state column"};
    for (int c = 0; c < AMBER_NUM_COLS; ++c)
        if (column_bytes(r, (amber_col_t)c) != 0 && !bufs->col[c])
            return fail(AMBER_E_INVALID, "%s is NULL", names[c]);
    if (host_cols) {
        if (t0 > 0xffffffffull) return fail(AMBER_E_INVALID, "step index above 2^32-1");
        if ((st = check_host_columns(r, host_cols)) != AMBER_OK) return st;
    }
    amber_buffers_t b = *bufs;
    if (noalloc) {
        if (b.workspace || b.workspace_bytes)
            return fail(AMBER_E_INVALID, "the no-allocation call takes no workspace (it must be "
                                         "NULL with 0 bytes)");
        if (r.ws_bytes > NOALLOC_SCRATCH_BYTES)
            return fail(AMBER_E_UNSUPPORTED,
                        "the run needs %llu bytes of workspace, above the %llu-byte device "
                        "scratch of the no-allocation call",
                        (unsigned long long)r.ws_bytes,
                        (unsigned long long)NOALLOC_SCRATCH_BYTES);
    } else {
        if (!b.workspace) return fail(AMBER_E_INVALID, "workspace is NULL");
        if (b.workspace_bytes < r.ws_bytes)
            return fail(AMBER_E_NOMEM, "workspace has %zu bytes, the run needs %llu",
                        b.workspace_bytes, (unsigned long long)r.ws_bytes);
    }
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    for (int c = 0; c < AMBER_NUM_COLS; ++c) {
        if (column_bytes(r, (amber_col_t)c) == 0) continue;
        st = check_device_ptr(b.col[c], device, names[c], column_bytes(r, (amber_col_t)c));
        if (st != AMBER_OK) return st;
    }
    if (noalloc) {
        if (device < 0 || device >= (int)NOALLOC_MAX_DEVICES)
            return fail(AMBER_E_UNSUPPORTED, "device %d is beyond the no-allocation scratch's "
                                             "%u devices", device, NOALLOC_MAX_DEVICES);
        void *scr = nullptr;
        HIP_TRY(noalloc_scratch(device, &scr), "scratch symbol address");
        b.workspace = scr;
        b.workspace_bytes = NOALLOC_SCRATCH_BYTES;
    } else {
        st = check_device_ptr(b.workspace, device, "workspace", r.ws_bytes);
        if (st != AMBER_OK) return st;
    }
    if (((uintptr_t)b.workspace & 255u) != 0)
        return fail(AMBER_E_INVALID, "workspace is not 256-byte aligned");
    if (noalloc) {
        std::lock_guard<std::mutex> lk(g_live_mu);
        if (g_scratch_held[device])
            return fail(AMBER_E_STATE, "the no-allocation scratch of device %d is held by a live "
                                       "handle (release it first)", device);
        g_scratch_held[device] = true;
    }
    auto unhold = [&] {
        if (!noalloc) return;
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_scratch_held[device] = false;
    };

    amber_pop *p = new (std::nothrow) amber_pop;
    if (!p) {
        unhold();
        return fail(AMBER_E_NOMEM, "host allocation of the handle failed");
    }
    p->r = std::move(r);
    p->b = b;
    p->stream = (hipStream_t)hip_stream;
    p->device = device;
    p->scratch = noalloc;
    p->acc = (DevInvariants *)p->b.workspace;
    const Resolved &rr = p->r;

    auto bail = [&](amber_status_t s) {
        delete p;
        unhold();
        return s;
    };
    // header: invariants result and the sticky device error word
    hipError_t e = launch_zero_words((uint32_t *)p->b.workspace, 64, p->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "workspace clear"));
    if (rr.model == AMBER_WEALTH) {
        e = launch_init_wealth(col_i32(p, AMBER_COL_WEALTH), (int32_t *)ws_ptr(p, rr.off_inc0),
                               (int32_t *)ws_ptr(p, rr.off_inc1), rr.n, rr.w_init, p->stream);
    } else {
        e = launch_init_positions(col_i32(p, AMBER_COL_X), col_i32(p, AMBER_COL_Y), rr.n,
                                  (int32_t)rr.L, rr.seed, rr.stream, p->stream);
        if (e == hipSuccess && rr.model == AMBER_SIR) {
            e = launch_init_states((uint8_t *)p->b.col[AMBER_COL_STATE], rr.n, rr.i0, p->stream);
            const uint64_t cell_words = (rr.off_count[1] - rr.off_count[0]) / 4;
            if (e == hipSuccess)
                e = launch_zero_words((uint32_t *)ws_ptr(p, rr.off_count[0]), 3 * cell_words,
                                      p->stream);
            if (e == hipSuccess)     // the demand-binning counts start at zero
                e = launch_zero_words((uint32_t *)ws_ptr(p, rr.off_nsi),
                                      (rr.off_dmap[0] - rr.off_nsi) / 4, p->stream);
            if (e == hipSuccess)
                p->persist_g = sir_persistent_groups_per_thread(rr.n, 8, &p->persist_blocks);
            if (e == hipSuccess && !noalloc) e = stop_words().take(&p->stop_host, &p->stop_dev);
            if (e == hipSuccess)     // by kernel arguments: the host does not wait
                e = launch_write_words((uint32_t *)ws_ptr(p, rr.off_table), rr.t_inf.data(),
                                       rr.t_inf.size(), p->stream);
        }
    }
    if (e != hipSuccess) return bail(hip_fail(e, "init kernels"));
    if (host_cols) {
        // the state after t0 steps replaces the initial rows (the padding
        // rows past N keep their initial, in-domain values); the host
        // columns are read before the call returns
        for (int c = 0; c < AMBER_NUM_COLS && e == hipSuccess; ++c) {
            if (column_bytes(rr, (amber_col_t)c) == 0) continue;
            e = hipMemcpyAsync(p->b.col[c], host_cols[c],
                               (size_t)rr.n * (c == AMBER_COL_STATE ? 1 : 4),
                               hipMemcpyHostToDevice, p->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return bail(hip_fail(e, "column upload"));
        p->step = t0;
    }
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.insert(p);
    }
    *out = p;
    return AMBER_OK;
}
}  // namespace

extern "C" {

uint32_t amber_abi_version(void) { return AMBER_ABI_VERSION; }

const char *amber_last_error(void) { return g_last_error.c_str(); }

size_t amber_column_bytes(const amber_run_desc_t *desc, amber_col_t c)
{
    Resolved r;
    if (resolve(desc, r, false) != AMBER_OK) return 0;
    return column_bytes(r, c);
}

size_t amber_workspace_bytes(const amber_run_desc_t *desc)
{
    Resolved r;
    if (resolve(desc, r, false) != AMBER_OK) return 0;
    return (size_t)r.ws_bytes;
}

amber_status_t amber_infection_table(uint32_t beta_num, uint32_t beta_den, uint32_t *out,
                                     uint32_t cap, uint32_t *k_sat)
{
    std::vector<uint32_t> t;
    amber_status_t st = build_infection_table(beta_num, beta_den, t);
    if (st != AMBER_OK) return st;
    if (k_sat) *k_sat = (uint32_t)t.size() - 1;
    if (out) std::memcpy(out, t.data(), std::min<size_t>(cap, t.size()) * sizeof(uint32_t));
    return AMBER_OK;
}


amber_status_t amber_init_population(const amber_run_desc_t *desc, const amber_buffers_t *bufs,
                                     void *hip_stream, amber_pop_t **out)
{
    return init_population(desc, bufs, hip_stream, out, false);
}

amber_status_t amber_resume_population(const amber_run_desc_t *desc, const amber_buffers_t *bufs,
                                       const void *const *host_cols, uint64_t step,
                                       void *hip_stream, amber_pop_t **out)
{
    if (!host_cols) return fail(AMBER_E_INVALID, "host_cols is NULL");
    return init_population(desc, bufs, hip_stream, out, false, host_cols, step);
}

amber_status_t amber_init_population_noalloc(const amber_run_desc_t *desc,
                                             const amber_buffers_t *bufs, void *hip_stream,
                                             amber_pop_t **out)
{
    return init_population(desc, bufs, hip_stream, out, true);
}

amber_status_t amber_view_update(void *col, uint32_t dtype, uint64_t n, amber_value_t a,
                                 amber_value_t b, const void *pred, uint32_t pred_dtype,
                                 uint32_t cmp, amber_value_t thr, void *hip_stream)
{
    if (dtype != AMBER_DT_I32 && dtype != AMBER_DT_F32)
        return fail(AMBER_E_INVALID, "dtype must be AMBER_DT_I32 or AMBER_DT_F32");
    if (pred && pred_dtype != AMBER_DT_I32 && pred_dtype != AMBER_DT_F32)
        return fail(AMBER_E_INVALID, "pred_dtype must be AMBER_DT_I32 or AMBER_DT_F32");
    if (pred && cmp > AMBER_CMP_GT) return fail(AMBER_E_INVALID, "cmp must be an amber_cmp_t");
    if (n >= (1ull << 40)) return fail(AMBER_E_UNSUPPORTED, "columns of 2^40 rows or more");
    if (n == 0) return AMBER_OK;
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    amber_status_t st = check_view_ptr(col, device, "column", 4 * n, 4);
    if (st != AMBER_OK) return st;
    if (pred && (st = check_view_ptr(pred, device, "predicate column", 4 * n, 4)) != AMBER_OK)
        return st;
    ViewValue va, vb, vt;
    va.i = a.i;
    vb.i = b.i;
    vt.i = thr.i;
    HIP_TRY(launch_view_update(col, dtype, n, va, vb, pred, pred_dtype, cmp, vt,
                               (hipStream_t)hip_stream),
            "view update kernel");
    return AMBER_OK;
}

size_t amber_view_scatter_workspace_bytes(uint32_t dtype, uint64_t n, uint64_t m)
{
    (void)n;
    if (dtype == AMBER_DT_I32) return 0;
    if (dtype != AMBER_DT_F32 || m > (1ull << 31)) return 0;
    return (size_t)view_scatter_f32_workspace(m);
}

size_t amber_view_write_log_workspace_bytes(uint64_t m)
{
    return m > (1ull << 31) ? 0 : (size_t)view_scatter_f32_workspace(m);
}

amber_status_t amber_view_scatter_add(void *col, uint32_t dtype, uint64_t n, const uint32_t *ids,
                                      uint64_t m, const void *vals, amber_value_t scalar,
                                      void *workspace, size_t workspace_bytes, void *hip_stream)
{
    if (dtype != AMBER_DT_I32 && dtype != AMBER_DT_F32)
        return fail(AMBER_E_INVALID, "dtype must be AMBER_DT_I32 or AMBER_DT_F32");
    if (n > 0xffffffffull) return fail(AMBER_E_UNSUPPORTED, "columns of 2^32 rows or more");
    if (m > (1ull << 31)) return fail(AMBER_E_UNSUPPORTED, "more than 2^31 scatter entries");
    const uint64_t need = dtype == AMBER_DT_F32 ? view_scatter_f32_workspace(m) : 0;
    if (m && need && !workspace) return fail(AMBER_E_INVALID, "workspace is NULL");
    if (m && workspace_bytes < need)
        return fail(AMBER_E_NOMEM, "workspace has %zu bytes, the call needs %llu", workspace_bytes,
                    (unsigned long long)need);
    if (m == 0) return AMBER_OK;
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    amber_status_t st = AMBER_OK;
    if (n && (st = check_view_ptr(col, device, "column", 4 * n, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(ids, device, "ids", 4 * m, 4)) != AMBER_OK) return st;
    if (vals && (st = check_view_ptr(vals, device, "vals", 4 * m, 4)) != AMBER_OK) return st;
    if (need && (st = check_view_ptr(workspace, device, "workspace", need, 16)) != AMBER_OK)
        return st;
    if (n == 0) return AMBER_OK;                     // every id is out of range
    ViewValue sv;
    sv.i = scalar.i;
    HIP_TRY(launch_view_scatter_add(col, dtype, n, ids, m, vals, sv, workspace,
                                    (hipStream_t)hip_stream),
            "view scatter-add kernels");
    return AMBER_OK;
}

size_t amber_async_workspace_bytes(const amber_run_desc_t *desc)
{
    Resolved r;
    if (resolve(desc, r, false) != AMBER_OK) return 0;
    if (r.model == AMBER_WEALTH) return (size_t)async_wealth_workspace(r.n);
    return r.model == AMBER_RANDOM_WALK ? 16u : 0u;
}

amber_status_t amber_step_async(amber_pop_t *pop, uint32_t n_steps, void *workspace,
                                size_t workspace_bytes)
{
    if (!is_live(pop)) return fail(AMBER_E_STATE, "unknown or released handle");
    const Resolved &r = pop->r;
    if (r.model == AMBER_SIR)
        return fail(AMBER_E_UNSUPPORTED, "asynchronous semantics are built for the wealth and "
                                         "random-walk models only");
    if (pop->step + n_steps > 0xffffffffull)
        return fail(AMBER_E_INVALID, "step index would exceed 2^32-1");
    if (n_steps == 0) return AMBER_OK;
    if (r.model == AMBER_RANDOM_WALK) {
        // no agent reads another's state: the sequential step is the
        // synchronous one
        return amber_step(pop, n_steps);
    }
    const uint64_t need = async_wealth_workspace(r.n);
    if (!workspace) return fail(AMBER_E_INVALID, "workspace is NULL");
    if (workspace_bytes < need)
        return fail(AMBER_E_NOMEM, "workspace has %zu bytes, the asynchronous step needs %llu",
                    workspace_bytes, (unsigned long long)need);
    amber_status_t st = check_view_ptr(workspace, pop->device, "workspace", need, 16);
    if (st != AMBER_OK) return st;
    HIP_TRY(timed(pop, "wealth_async", [&] {
                return launch_wealth_async(col_i32(pop, AMBER_COL_WEALTH), r.n, r.seed, r.stream,
                                           (uint32_t)pop->step, n_steps, workspace,
                                           (uint32_t *)ws_ptr(pop, ERR_FLAG_OFFSET), pop->stream);
            }),
            "asynchronous wealth kernels");
    const hipError_t te = timer_cut(pop);
    if (te != hipSuccess) return hip_fail(te, "timing event");
    pop->step += n_steps;
    return AMBER_OK;
}

amber_status_t amber_view_write_log(void *col, uint32_t dtype, uint64_t n, const uint32_t *ids,
                                    uint64_t m, const void *vals, void *workspace,
                                    size_t workspace_bytes, void *hip_stream)
{
    if (dtype != AMBER_DT_I32 && dtype != AMBER_DT_F32)
        return fail(AMBER_E_INVALID, "dtype must be AMBER_DT_I32 or AMBER_DT_F32");
    if (n > 0xffffffffull) return fail(AMBER_E_UNSUPPORTED, "columns of 2^32 rows or more");
    if (m > (1ull << 31)) return fail(AMBER_E_UNSUPPORTED, "more than 2^31 log entries");
    if (m == 0) return AMBER_OK;
    const uint64_t need = view_scatter_f32_workspace(m);
    if (!workspace) return fail(AMBER_E_INVALID, "workspace is NULL");
    if (workspace_bytes < need)
        return fail(AMBER_E_NOMEM, "workspace has %zu bytes, the call needs %llu", workspace_bytes,
                    (unsigned long long)need);
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    amber_status_t st = AMBER_OK;
    if (n && (st = check_view_ptr(col, device, "column", 4 * n, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(ids, device, "ids", 4 * m, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(vals, device, "vals", 4 * m, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(workspace, device, "workspace", need, 16)) != AMBER_OK) return st;
    if (n == 0) return AMBER_OK;
    HIP_TRY(launch_view_write_log((uint32_t *)col, n, ids, m, (const uint32_t *)vals, workspace,
                                  (hipStream_t)hip_stream),
            "write-log kernels");
    return AMBER_OK;
}

namespace {
// Checks a lattice description and fills g (positions from pos when given).
amber_status_t grid_desc(const int32_t *const *pos, uint32_t ndim, const uint32_t *dims,
                         GridDesc &g, uint64_t &cells)
{
    if (ndim < 1 || ndim > MAX_DIMS)
        return fail(AMBER_E_INVALID, "ndim must be 1 .. %u", MAX_DIMS);
    if (!dims) return fail(AMBER_E_INVALID, "dims is NULL");
    std::memset(&g, 0, sizeof g);
    g.ndim = ndim;
    cells = 1;
    for (uint32_t i = 0; i < ndim; ++i) {
        if (dims[i] < 1) return fail(AMBER_E_INVALID, "dims[%u] is 0", i);
        g.dims[i] = dims[i];
        g.stride[i] = (uint32_t)cells;
        cells *= dims[i];
        if (cells > 0xffffffffull)
            return fail(AMBER_E_UNSUPPORTED, "lattices of 2^32 cells or more");
        if (pos) {
            if (!pos[i]) return fail(AMBER_E_INVALID, "pos[%u] is NULL", i);
            g.pos[i] = pos[i];
        }
    }
    return AMBER_OK;
}
}  // namespace

amber_status_t amber_grid_count(const int32_t *const *pos, uint32_t ndim, const uint32_t *dims,
                                uint64_t n, const uint8_t *state, uint32_t match,
                                uint32_t *counts, void *hip_stream)
{
    if (!pos) return fail(AMBER_E_INVALID, "pos is NULL");
    GridDesc g;
    uint64_t cells = 0;
    amber_status_t st = grid_desc(pos, ndim, dims, g, cells);
    if (st != AMBER_OK) return st;
    if (n > 0xffffffffull) return fail(AMBER_E_UNSUPPORTED, "more than 2^32-1 agents");
    if (match > 255) return fail(AMBER_E_INVALID, "match must be a state code (0 .. 255)");
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    if ((st = check_view_ptr(counts, device, "counts", 4 * cells, 4)) != AMBER_OK) return st;
    if (n) {
        for (uint32_t i = 0; i < ndim; ++i)
            if ((st = check_view_ptr(pos[i], device, "position column", 4 * n, 4)) != AMBER_OK)
                return st;
        if (state && (st = check_view_ptr(state, device, "state column", n, 1)) != AMBER_OK)
            return st;
    }
    HIP_TRY(launch_grid_count(g, n, state, match, counts, cells, (hipStream_t)hip_stream),
            "grid count kernels");
    return AMBER_OK;
}

amber_status_t amber_grid_neighbour_sum(const uint32_t *counts, uint32_t ndim,
                                        const uint32_t *dims, uint32_t neighbourhood,
                                        uint32_t torus, uint32_t *out, void *hip_stream)
{
    GridDesc g;
    uint64_t cells = 0;
    amber_status_t st = grid_desc(nullptr, ndim, dims, g, cells);
    if (st != AMBER_OK) return st;
    if (neighbourhood != AMBER_MOORE && neighbourhood != AMBER_VON_NEUMANN)
        return fail(AMBER_E_INVALID, "neighbourhood must be AMBER_MOORE or AMBER_VON_NEUMANN");
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    if ((st = check_view_ptr(counts, device, "counts", 4 * cells, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(out, device, "out", 4 * cells, 4)) != AMBER_OK) return st;
    if (counts == out) return fail(AMBER_E_INVALID, "out must not be counts");
    uint32_t dedup = 0;
    for (uint32_t i = 0; i < ndim; ++i) dedup |= torus && dims[i] < 3;
    HIP_TRY(launch_grid_neighbour_sum(g, cells, neighbourhood == AMBER_VON_NEUMANN, torus ? 1 : 0,
                                      dedup, counts, out, (hipStream_t)hip_stream),
            "grid neighbour kernel");
    return AMBER_OK;
}

amber_status_t amber_grid_gather(const uint32_t *table, const int32_t *const *pos, uint32_t ndim,
                                 const uint32_t *dims, uint64_t n, uint32_t *out,
                                 void *hip_stream)
{
    if (!pos) return fail(AMBER_E_INVALID, "pos is NULL");
    GridDesc g;
    uint64_t cells = 0;
    amber_status_t st = grid_desc(pos, ndim, dims, g, cells);
    if (st != AMBER_OK) return st;
    if (n > 0xffffffffull) return fail(AMBER_E_UNSUPPORTED, "more than 2^32-1 agents");
    if (n == 0) return AMBER_OK;
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    if ((st = check_view_ptr(table, device, "table", 4 * cells, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(out, device, "out", 4 * n, 4)) != AMBER_OK) return st;
    for (uint32_t i = 0; i < ndim; ++i)
        if ((st = check_view_ptr(pos[i], device, "position column", 4 * n, 4)) != AMBER_OK)
            return st;
    HIP_TRY(launch_grid_gather(g, n, table, out, (hipStream_t)hip_stream), "grid gather kernel");
    return AMBER_OK;
}

amber_status_t amber_graph_neighbour_count(const uint32_t *row, const uint32_t *col, uint64_t n,
                                           uint64_t nnz, const uint8_t *state, uint32_t match,
                                           uint32_t *out, void *hip_stream)
{
    if (n > 0xffffffffull || nnz > 0xffffffffull)
        return fail(AMBER_E_UNSUPPORTED, "graphs of 2^32 nodes or adjacency entries or more");
    if (match > 255) return fail(AMBER_E_INVALID, "match must be a state code (0 .. 255)");
    if (n == 0) return AMBER_OK;
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    amber_status_t st = AMBER_OK;
    if ((st = check_view_ptr(row, device, "row offsets", 4 * (n + 1), 4)) != AMBER_OK) return st;
    if (nnz && (st = check_view_ptr(col, device, "neighbour ids", 4 * nnz, 4)) != AMBER_OK)
        return st;
    if ((st = check_view_ptr(state, device, "state column", n, 1)) != AMBER_OK) return st;
    if ((st = check_view_ptr(out, device, "out", 4 * n, 4)) != AMBER_OK) return st;
    HIP_TRY(launch_graph_count(row, col, n, nnz, state, match, out, (hipStream_t)hip_stream),
            "graph count kernel");
    return AMBER_OK;
}

amber_status_t amber_recovery_threshold(uint32_t gamma_num, uint32_t gamma_den, uint32_t *out)
{
    if (!out) return fail(AMBER_E_INVALID, "out is NULL");
    if (gamma_den == 0 || gamma_num >= gamma_den)
        return fail(AMBER_E_INVALID, "need 0 <= gamma_num < gamma_den");
    *out = bernoulli_threshold(gamma_num, gamma_den);
    return AMBER_OK;
}

amber_status_t amber_sir_transition(uint8_t *state, const uint32_t *k, uint64_t n, uint32_t seed,
                                    uint32_t stream_id, uint32_t t, const uint32_t *t_inf,
                                    uint32_t table_len, uint32_t t_rec, void *hip_stream)
{
    if (table_len < 1 || table_len > AMBER_MAX_TABLE)
        return fail(AMBER_E_INVALID, "table_len must be 1 .. %u", AMBER_MAX_TABLE);
    if (n > 0xffffffffull) return fail(AMBER_E_UNSUPPORTED, "more than 2^32-1 agents");
    if (n == 0) return AMBER_OK;
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    amber_status_t st = AMBER_OK;
    if ((st = check_view_ptr(state, device, "state column", n, 1)) != AMBER_OK) return st;
    if ((st = check_view_ptr(k, device, "counts", 4 * n, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(t_inf, device, "infection table", 4ull * table_len, 4)) != AMBER_OK)
        return st;
    HIP_TRY(launch_sir_transition_only(state, k, n, seed, stream_id, t, t_inf, table_len, t_rec,
                                       (hipStream_t)hip_stream),
            "SIR transition kernel");
    return AMBER_OK;
}

namespace {
// Cells per axis of the continuous SIR's cell list, 0 when the world does
// not fit (W / r above CONT_MAX_CELLS).
constexpr uint32_t CONT_MAX_CELLS = 4096;
uint32_t cont_cells(float W, float r)
{
    if (!(r > 0.0f) || !(W >= 0.0f) || !std::isfinite(W) || !std::isfinite(r)) return 0;
    const double q = std::floor((double)W / (double)r);
    return q + 1 > CONT_MAX_CELLS ? 0u : (uint32_t)q + 1;
}
}  // namespace

amber_status_t amber_cont_init(float *x, float *y, uint8_t *state, uint8_t *days, uint64_t n,
                               float W, uint32_t seed, uint32_t stream_id,
                               uint32_t initial_infected, void *hip_stream)
{
    if (n == 0 || n > 0x7fffffffull) return fail(AMBER_E_INVALID, "n must be 1 .. 2^31-1");
    if (!(W >= 0.0f) || !std::isfinite(W)) return fail(AMBER_E_INVALID, "W must be finite and >= 0");
    if ((state == nullptr) != (days == nullptr))
        return fail(AMBER_E_INVALID, "state and days are both given (SIR) or both NULL (walk)");
    if (state && initial_infected > n)
        return fail(AMBER_E_INVALID, "initial_infected exceeds n");
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    amber_status_t st = AMBER_OK;
    if ((st = check_view_ptr(x, device, "x", 4 * n, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(y, device, "y", 4 * n, 4)) != AMBER_OK) return st;
    if (state) {
        if ((st = check_view_ptr(state, device, "state", n, 1)) != AMBER_OK) return st;
        if ((st = check_view_ptr(days, device, "days", n, 1)) != AMBER_OK) return st;
    }
    hipStream_t hs = (hipStream_t)hip_stream;
    HIP_TRY(launch_cont_init(x, y, (uint32_t)n, W, seed, stream_id, hs), "continuous init kernel");
    if (state)
        HIP_TRY(launch_cont_states(state, days, (uint32_t)n, initial_infected, hs),
                "continuous states kernel");
    return AMBER_OK;
}

amber_status_t amber_cont_walk(float *x, float *y, uint64_t n, float W, uint32_t seed,
                               uint32_t stream_id, uint32_t t0, uint32_t n_steps,
                               void *hip_stream)
{
    if (n == 0 || n > 0x7fffffffull) return fail(AMBER_E_INVALID, "n must be 1 .. 2^31-1");
    if (!(W >= 0.0f) || !std::isfinite(W)) return fail(AMBER_E_INVALID, "W must be finite and >= 0");
    if ((uint64_t)t0 + n_steps > 0xffffffffull)
        return fail(AMBER_E_INVALID, "step index would exceed 2^32-1");
    if (n_steps == 0) return AMBER_OK;
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    amber_status_t st = AMBER_OK;
    if ((st = check_view_ptr(x, device, "x", 4 * n, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(y, device, "y", 4 * n, 4)) != AMBER_OK) return st;
    HIP_TRY(launch_cont_walk(x, y, (uint32_t)n, W, seed, stream_id, t0, n_steps,
                             (hipStream_t)hip_stream),
            "continuous walk kernel");
    return AMBER_OK;
}

size_t amber_cont_sir_workspace_bytes(uint64_t n, float W, float r, uint32_t p_num,
                                      uint32_t p_den)
{
    const uint32_t nc = cont_cells(W, r);
    std::vector<uint32_t> t;
    if (!nc || n == 0 || n > 0x7fffffffull || build_infection_table(p_num, p_den, t) != AMBER_OK)
        return 0;
    return (size_t)cont_sir_workspace((uint32_t)n, nc, (uint32_t)t.size());
}

amber_status_t amber_cont_sir(float *x, float *y, uint8_t *state, uint8_t *days, uint64_t n,
                              float W, float r, uint32_t seed, uint32_t stream_id, uint32_t p_num,
                              uint32_t p_den, uint32_t recover, uint32_t t0, uint32_t n_steps,
                              void *workspace, size_t workspace_bytes, void *hip_stream)
{
    if (n == 0 || n > 0x7fffffffull) return fail(AMBER_E_INVALID, "n must be 1 .. 2^31-1");
    if (!(W >= 0.0f) || !std::isfinite(W)) return fail(AMBER_E_INVALID, "W must be finite and >= 0");
    const uint32_t nc = cont_cells(W, r);
    if (!nc)
        return fail(!(r > 0.0f) || !std::isfinite(r) ? AMBER_E_INVALID : AMBER_E_UNSUPPORTED,
                    "r must be finite and > 0, with W / r below %u", CONT_MAX_CELLS);
    if (recover < 1 || recover > 255) return fail(AMBER_E_INVALID, "recover must be 1 .. 255");
    if ((uint64_t)t0 + n_steps > 0xffffffffull)
        return fail(AMBER_E_INVALID, "step index would exceed 2^32-1");
    std::vector<uint32_t> table;
    amber_status_t st = build_infection_table(p_num, p_den, table);
    if (st != AMBER_OK) return st;
    const uint64_t need = cont_sir_workspace((uint32_t)n, nc, (uint32_t)table.size());
    if (!workspace) return fail(AMBER_E_INVALID, "workspace is NULL");
    if (workspace_bytes < need)
        return fail(AMBER_E_NOMEM, "workspace has %zu bytes, the call needs %llu", workspace_bytes,
                    (unsigned long long)need);
    if (n_steps == 0) return AMBER_OK;
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    if ((st = check_view_ptr(x, device, "x", 4 * n, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(y, device, "y", 4 * n, 4)) != AMBER_OK) return st;
    if ((st = check_view_ptr(state, device, "state", n, 1)) != AMBER_OK) return st;
    if ((st = check_view_ptr(days, device, "days", n, 1)) != AMBER_OK) return st;
    if ((st = check_view_ptr(workspace, device, "workspace", need, 16)) != AMBER_OK) return st;
    HIP_TRY(launch_cont_sir(x, y, state, days, (uint32_t)n, W, r, nc, seed, stream_id, table.data(),
                            (uint32_t)table.size(), recover, t0, n_steps, workspace,
                            (hipStream_t)hip_stream),
            "continuous SIR kernels");
    return AMBER_OK;
}

amber_status_t amber_step(amber_pop_t *pop, uint32_t n_steps)
{
    if (!is_live(pop)) return fail(AMBER_E_STATE, "unknown or released handle");
    if (n_steps == 0) return AMBER_OK;
    if (pop->step + n_steps > 0xffffffffull)
        return fail(AMBER_E_INVALID, "step index would exceed 2^32-1");
    amber_status_t st = enqueue_steps(pop, n_steps);
    const hipError_t te = timer_cut(pop);
    if (st != AMBER_OK) return st;
    if (te != hipSuccess) return hip_fail(te, "timing event");
    pop->step += n_steps;
    return AMBER_OK;
}

amber_status_t amber_step_batch(amber_pop_t *const *pops, uint32_t n, uint32_t n_steps)
{
    if (!pops && n) return fail(AMBER_E_INVALID, "pops is NULL");
    for (uint32_t i = 0; i < n; ++i) {
        if (!is_live(pops[i])) return fail(AMBER_E_STATE, "handle %u is unknown or released", i);
        for (uint32_t j = 0; j < i; ++j)
            if (pops[j] == pops[i]) return fail(AMBER_E_INVALID, "handle %u repeats", i);
        if (pops[i]->device != pops[0]->device)
            return fail(AMBER_E_STATE, "handles live on different devices");
        if (pops[i]->step + n_steps > 0xffffffffull)
            return fail(AMBER_E_INVALID, "step index would exceed 2^32-1");
    }
    if (n == 0 || n_steps == 0) return AMBER_OK;
    amber_status_t st = run_batch(pops, n, n_steps);
    hipError_t te = hipSuccess;
    for (uint32_t i = 0; i < n; ++i) {
        const hipError_t e = timer_cut(pops[i]);
        if (te == hipSuccess) te = e;
    }
    if (st != AMBER_OK) return st;
    if (te != hipSuccess) return hip_fail(te, "timing event");
    for (uint32_t i = 0; i < n; ++i) pops[i]->step += n_steps;
    return AMBER_OK;
}

amber_status_t amber_read_columns(amber_pop_t *pop, uint32_t col_mask, void *const *host_dst)
{
    if (!is_live(pop)) return fail(AMBER_E_STATE, "unknown or released handle");
    if (!host_dst) return fail(AMBER_E_INVALID, "host_dst is NULL");
    for (int c = 0; c < AMBER_NUM_COLS; ++c) {
        if (!(col_mask & (1u << c))) continue;
        if (column_bytes(pop->r, (amber_col_t)c) == 0)
            return fail(AMBER_E_INVALID, "column %d is not used by this model", c);
        if (!host_dst[c]) return fail(AMBER_E_INVALID, "host_dst[%d] is NULL", c);
    }
    if (col_mask >> AMBER_NUM_COLS) return fail(AMBER_E_INVALID, "unknown column bits in mask");
    for (int c = 0; c < AMBER_NUM_COLS; ++c) {
        if (!(col_mask & (1u << c))) continue;
        const size_t bytes = (size_t)pop->r.n * (c == AMBER_COL_STATE ? 1 : 4);
        HIP_TRY(hipMemcpyAsync(host_dst[c], pop->b.col[c], bytes, hipMemcpyDeviceToHost,
                               pop->stream),
                "column copy");
    }
    uint32_t flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, (uint8_t *)pop->b.workspace + ERR_FLAG_OFFSET, 4,
                           hipMemcpyDeviceToHost, pop->stream),
            "error flag copy");
    HIP_TRY(hipStreamSynchronize(pop->stream), "stream synchronize");
    amber_status_t fst = check_device_flag(pop, flag);
    if (fst != AMBER_OK) return fst;
    return AMBER_OK;
}

amber_status_t amber_invariants(amber_pop_t *pop, amber_invariants_t *out)
{
    if (!is_live(pop)) return fail(AMBER_E_STATE, "unknown or released handle");
    if (!out) return fail(AMBER_E_INVALID, "out is NULL");
    const Resolved &r = pop->r;
    HIP_TRY(launch_invariants(r.model, r.n, (int32_t)r.L, col_i32(pop, AMBER_COL_WEALTH),
                              col_i32(pop, AMBER_COL_X), col_i32(pop, AMBER_COL_Y),
                              (const uint8_t *)pop->b.col[AMBER_COL_STATE], pop->acc,
                              (DevInvariants *)ws_ptr(pop, INV_PARTIALS_OFFSET), pop->stream),
            "invariants kernel");
    uint8_t head[256];
    HIP_TRY(hipMemcpyAsync(head, pop->acc, sizeof head, hipMemcpyDeviceToHost, pop->stream),
            "invariants copy");
    HIP_TRY(hipStreamSynchronize(pop->stream), "stream synchronize");
    DevInvariants h;
    std::memcpy(&h, head, sizeof h);
    uint32_t flag;
    std::memcpy(&flag, head + ERR_FLAG_OFFSET, 4);
    amber_status_t fst = check_device_flag(pop, flag);
    if (fst != AMBER_OK) return fst;
    std::memset(out, 0, sizeof *out);
    out->step = pop->step;
    out->digest = h.digest;
    out->out_of_bounds = h.out_of_bounds;
    if (r.model == AMBER_WEALTH) {
        out->wealth_sum = (int64_t)h.wealth_sum;
        out->wealth_min = h.wealth_min;
    }
    if (r.model == AMBER_SIR) {
        out->n_s = h.n_s;
        out->n_i = h.n_i;
        out->n_r = h.n_r;
    }
    return AMBER_OK;
}

amber_status_t amber_pop_info(const amber_pop_t *pop, amber_pop_info_t *out)
{
    if (!is_live(pop)) return fail(AMBER_E_STATE, "unknown or released handle");
    if (!out) return fail(AMBER_E_INVALID, "out is NULL");
    const Resolved &r = pop->r;
    out->model = r.model;
    out->n_agents = r.n;
    out->grid_side = r.L;
    out->initial_infected = r.i0;
    out->seed = r.seed;
    out->stream = r.stream;
    out->table_len = (uint32_t)r.t_inf.size();
    out->t_rec = r.t_rec;
    out->step = pop->step;
    return AMBER_OK;
}

amber_status_t amber_set_tuning(amber_pop_t *pop, const amber_tuning_t *t)
{
    if (!is_live(pop)) return fail(AMBER_E_STATE, "unknown or released handle");
    if (!t) return fail(AMBER_E_INVALID, "tuning is NULL");
    if (t->block < 64 || t->block > 1024 || t->block % 64)
        return fail(AMBER_E_INVALID, "block must be a multiple of 64 in [64, 1024]");
    if (t->sir_form > 2) return fail(AMBER_E_INVALID, "sir_form must be 0, 1 or 2");
    if (t->max_groups_per_thread != 0 && t->max_groups_per_thread != 1 &&
        t->max_groups_per_thread != 2 && t->max_groups_per_thread != 4 &&
        t->max_groups_per_thread != 8)
        return fail(AMBER_E_INVALID, "max_groups_per_thread must be 0, 1, 2, 4 or 8");
    if (t->sir_count > 5) return fail(AMBER_E_INVALID, "sir_count must be in 0 .. 5");
    if (t->wealth_form > 3) return fail(AMBER_E_INVALID, "wealth_form must be 0, 1, 2 or 3");
    if (t->sir_tile != 0 && t->sir_tile != 32 && t->sir_tile != 64)
        return fail(AMBER_E_INVALID, "sir_tile must be 0, 32 or 64");
    if (t->sir_poll != POLL_NOWAIT && t->sir_poll != POLL_OFF && t->sir_poll != POLL_PACED)
        return fail(AMBER_E_INVALID, "sir_poll must be 0, 1 or 2");
    pop->tuning.sir_tile = t->sir_tile;
    pop->tuning.sir_poll = t->sir_poll;
    pop->tuning.wealth_form = t->wealth_form;
    pop->tuning.block = t->block;
    pop->tuning.sir_form = t->sir_form;
    pop->tuning.sir_count = t->sir_count;
    pop->tuning.max_g = t->max_groups_per_thread ? t->max_groups_per_thread : 8;
    return AMBER_OK;
}

amber_status_t amber_get_tuning(const amber_pop_t *pop, amber_tuning_t *t)
{
    if (!is_live(pop)) return fail(AMBER_E_STATE, "unknown or released handle");
    if (!t) return fail(AMBER_E_INVALID, "tuning is NULL");
    std::memset(t, 0, sizeof *t);
    t->block = pop->tuning.block;
    t->sir_form = pop->tuning.sir_form;
    t->max_groups_per_thread = pop->tuning.max_g;
    t->sir_count = pop->tuning.sir_count;
    t->wealth_form = pop->tuning.wealth_form;
    t->sir_tile = pop->tuning.sir_tile;
    t->sir_poll = pop->tuning.sir_poll;
    return AMBER_OK;
}

amber_status_t amber_profile_enable(amber_pop_t *pop, int enable)
{
    if (!is_live(pop)) return fail(AMBER_E_STATE, "unknown or released handle");
    KernelTimer &tm = pop->timer;
    if (enable) {
        HIP_TRY(hipStreamSynchronize(pop->stream), "stream synchronize");
        for (auto &p : tm.pending) {
            tm.pool.push_back(p.start);
            tm.pool.push_back(p.stop);
        }
        tm.pending.clear();
        std::fill(tm.launches.begin(), tm.launches.end(), 0);
        std::fill(tm.total_ms.begin(), tm.total_ms.end(), 0.0);
    }
    tm.on = enable != 0;
    return AMBER_OK;
}

amber_status_t amber_profile_read(amber_pop_t *pop, amber_kernel_time_t *out, uint32_t cap,
                                  uint32_t *count)
{
    if (!is_live(pop)) return fail(AMBER_E_STATE, "unknown or released handle");
    if (!count || (cap && !out)) return fail(AMBER_E_INVALID, "out/count is NULL");
    KernelTimer &tm = pop->timer;
    HIP_TRY(hipStreamSynchronize(pop->stream), "stream synchronize");
    for (auto &p : tm.pending) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.start, p.stop), "hipEventElapsedTime");
        tm.launches[p.kernel] += p.count;
        tm.total_ms[p.kernel] += ms;
        tm.pool.push_back(p.start);
        tm.pool.push_back(p.stop);
    }
    tm.pending.clear();
    *count = (uint32_t)tm.names.size();
    for (uint32_t i = 0; i < tm.names.size() && i < cap; ++i) {
        std::memset(&out[i], 0, sizeof out[i]);
        std::snprintf(out[i].name, sizeof out[i].name, "%s", tm.names[i].c_str());
        out[i].launches = tm.launches[i];
        out[i].total_ms = tm.total_ms[i];
    }
    return AMBER_OK;
}

amber_status_t amber_release(amber_pop_t *pop)
{
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        if (!pop || !g_live.count(pop)) return fail(AMBER_E_STATE, "unknown or released handle");
        g_live.erase(pop);
    }
    hipError_t e = hipStreamSynchronize(pop->stream);
    if (pop->scratch) {
        // the scratch is free for the next handle once this one's work is done
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_scratch_held[pop->device] = false;
    }
    delete pop;
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    return AMBER_OK;
}

}  // extern "C"
