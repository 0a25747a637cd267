// rp_wg.h -- the rounds of one shuffle on one group of lanes (a workgroup or
// a single wave) with all of its round state in LDS: the Knuth shuffle of
// Section 4.1 with the round structure of Algorithm 2 (relaxed-PIP rounds over
// the first k unfinished swaps) and the RP-Final reservation of Appendix A.2
// (one hashed priority slot per target, a dense window for the round's
// consecutive keys).  Used by the batched form (rp_batch.hip) and by the
// resident serving kernel (rp.hip).  Internal to the library; not part of the
// ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "rp.h"
#include "rp_device.h"

namespace rpwg {

using namespace rpdev;

// Workgroups of 256 or 1024 lanes (a schedule choice of the batched form) or
// 512 (the resident form); LDS for round state: 64 KB per 1024-lane
// workgroup, 32 KB otherwise, split in equal parts between the waves in wave
// mode.
template <int WGL> struct Shape {
    static constexpr int WAVES = WGL / 64;
    static constexpr uint32_t LDS_WORDS = WGL == 1024 ? 16384u : 8192u;
    static constexpr uint32_t WAVE_WORDS = LDS_WORDS / WAVES;
};
constexpr int BM = 8;                    // swap slots per lane (maximum)
// Priorities are tag:4 | rank:28 with rank = s - cnew.  A swap that enters
// the window stays active at most k rounds (every round the highest active
// swap commits, and no swap above it ever enters again), and the window moves
// down by at most k per round, so ranks stay below k*k + k: within 28 bits for
// any n since k <= 1024 * BM, with no rank throttle.  The 4-bit tag makes the
// values of a round exceed all older ones; the LDS slot array is cleared every
// 16 rounds, which costs little in LDS.
constexpr uint32_t BRANKB = 28;
constexpr uint32_t BTAG_CYCLE = 16;
constexpr uint32_t K_MAX_WG = 1024 * BM;  // largest k of any request
static_assert((uint64_t)K_MAX_WG * K_MAX_WG + K_MAX_WG < (1ull << BRANKB), "ranks overflow");
constexpr uint64_t BATCH_MAX_N = 1ull << 32;  // indices are 32-bit

struct BatchReq {
    unsigned char *A;
    const uint64_t *H;     // nullptr: seed mode
    uint64_t seed;
    uint32_t n, eb;
    uint32_t k;            // active-swap capacity
    uint32_t T;            // reservation slots (LDS words)
    uint32_t bmw;          // dense-window words per parity
    uint32_t wg_mode;      // 1: workgroup, 0: wave
    uint32_t orig;         // index in the caller's array
    uint32_t invalid;      // set on the device when some H[i] > i
};


// ------------------------------------------------------------ lane groups

// Workgroup: WGL lanes, LDS scratch shared, barrier = __syncthreads.
template <int WGL> struct WGGroup {
    static constexpr int BWAVES = WGL / 64;
    uint32_t *lds;
    uint32_t *sh_scan;  // BWAVES words
    __device__ uint32_t nlanes() const { return WGL; }
    __device__ uint32_t lane() const { return threadIdx.x; }
    __device__ void sync() const { __syncthreads(); }
    // Exclusive prefix of x over the group; *total = sum.  Contains a
    // barrier, which also separates one round from the next.
    __device__ uint32_t excl_scan(uint32_t x, uint32_t *total) const
    {
        const uint32_t wave = threadIdx.x >> 6, l = threadIdx.x & 63;
        const uint32_t xi = wave_incl_scan(x);
        if (l == 63)
            sh_scan[wave] = xi;
        __syncthreads();
        uint32_t below = 0, tot = 0;
#pragma unroll
        for (int i = 0; i < BWAVES; i++) {
            const uint32_t v = sh_scan[i];
            below += ((uint32_t)i < wave) ? v : 0u;
            tot += v;
        }
        *total = __builtin_amdgcn_readfirstlane(tot);
        return below + xi - x;
    }
};

// One wave, 64 lanes, executing in order: LDS and global accesses of its
// lanes are ordered by program order, so "sync" is only a compiler fence.
struct WaveGroup {
    uint32_t *lds;
    __device__ uint32_t nlanes() const { return 64; }
    __device__ uint32_t lane() const { return threadIdx.x & 63; }
    __device__ void sync() const { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup"); }
    __device__ uint32_t excl_scan(uint32_t x, uint32_t *total) const
    {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        const uint32_t xi = wave_incl_scan(x);
        *total = __builtin_amdgcn_readlane(xi, 63);
        return xi - x;
    }
};

// A request's arrays are device global memory.  Its pointers come from the
// descriptor array, so the compiler cannot see that by itself and would use
// flat instructions, which also count against the LDS counter: then every
// LDS wait before a group barrier would also wait for the records in flight.
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ gptr<T> as_global(T *p)
{
    return (gptr<T>)p;
}

__device__ __forceinline__ uint32_t breq_target(const BatchReq &r, uint32_t s)
{
    return r.H ? (uint32_t)as_global(r.H)[s] : seed_target(r.seed, s);
}

__device__ __forceinline__ uint32_t lds_ld(const uint32_t *p)
{
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_st(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Records moved with plain loads and stores: every access to A comes from the
// lanes of one group, which see each other's writes after the group's sync.
template <int EB> struct PRec;
template <> struct PRec<4> {
    uint32_t w;
    __device__ void load(const unsigned char *A, uint32_t i)
    { w = as_global(reinterpret_cast<const uint32_t *>(A))[i]; }
    __device__ void store(unsigned char *A, uint32_t i) const
    { as_global(reinterpret_cast<uint32_t *>(A))[i] = w; }
};
template <> struct PRec<8> {
    uint64_t w;
    __device__ void load(const unsigned char *A, uint32_t i)
    { w = as_global(reinterpret_cast<const uint64_t *>(A))[i]; }
    __device__ void store(unsigned char *A, uint32_t i) const
    { as_global(reinterpret_cast<uint64_t *>(A))[i] = w; }
};

__device__ __forceinline__ void pswap_generic(unsigned char *A, uint32_t eb,
                                              uint32_t a, uint32_t b)
{
    gptr<uint32_t> pa = as_global(reinterpret_cast<uint32_t *>(A + (uint64_t)a * eb));
    gptr<uint32_t> pb = as_global(reinterpret_cast<uint32_t *>(A + (uint64_t)b * eb));
    for (uint32_t j = 0; j < eb / 4; j++) {
        const uint32_t x = pa[j], y = pb[j];
        pa[j] = y;
        pb[j] = x;
    }
}

// Run one request on group g.  Returns (rounds, attempts) through pointers
// valid on every lane.
template <int EB, typename Group>
__device__ void run_request(const Group &g, const BatchReq &r, uint64_t max_rounds, bool late,
                            uint64_t *rounds_out, uint64_t *attempts_out,
                            uint32_t *status_out)
{
    const uint32_t L = g.nlanes(), lane = g.lane();
    const uint32_t T = r.T, bmw = r.bmw, W = r.bmw * 32u;
    if (T == 0) {
        // The bound holds no reservation state: k = 1, and a single active
        // swap always commits, so the rounds are the sequential loop.
        uint64_t rounds = 0;
        if (lane == 0) {
            for (uint32_t i = r.n; i-- > 0;) {
                const uint32_t h = breq_target(r, i);
                if (h == i)
                    continue;
                pswap_generic(r.A, r.eb, i, h);
                rounds++;
            }
        }
        g.sync();
        *rounds_out = rounds;
        *attempts_out = rounds;
        *status_out = 0;
        return;
    }
    uint32_t *slots = g.lds;
    uint32_t *bm = g.lds + T;
    g.sync();
    for (uint32_t i = lane; i < T + 2 * bmw; i += L)
        lds_st(&g.lds[i], 0u);
    g.sync();

    uint32_t src[BM], tgt[BM];
    bool usable[BM];
#pragma unroll
    for (int m = 0; m < BM; m++) {
        usable[m] = ((uint64_t)m * L + lane) < r.k;
        src[m] = EMPTY;
        tgt[m] = 0;
    }
    uint32_t cursor = r.n;
    uint64_t rounds = 0, attempts = 0;
    uint32_t status = 0;
    for (;;) {
        uint32_t f = 0, a = 0;
#pragma unroll
        for (int m = 0; m < BM; m++) {
            f += (usable[m] && src[m] == EMPTY) ? 1u : 0u;
            a += (src[m] != EMPTY) ? 1u : 0u;
        }
        uint32_t tot;
        const uint32_t x = (a << 16) | f;
        const uint32_t lane_off = g.excl_scan(x, &tot) & 0xFFFFu;
        const uint32_t totF = tot & 0xFFFFu, totA = tot >> 16;
        if (cursor == 0 && totA == 0)
            break;
        if (rounds >= max_rounds) {
            status = (uint32_t)(-RP_ETIMEOUT);
            break;
        }
        const uint32_t take = min(totF, cursor);
        const uint32_t cnew = cursor - take;
        const uint32_t par = (uint32_t)(rounds & 1);
        const uint32_t tag = (uint32_t)(rounds & (BTAG_CYCLE - 1));
        if (tag == 0 && rounds > 0) {
            // Tags restart: empty the slot array (every check of the last
            // round finished before the scan's barrier).
            for (uint32_t i = lane; i < T; i += L)
                lds_st(&slots[i], 0u);
            g.sync();
        }
        // refill
        uint32_t j = lane_off;
#pragma unroll
        for (int m = 0; m < BM; m++) {
            if (usable[m] && src[m] == EMPTY) {
                const uint32_t ord = j++;
                if (ord < take) {
                    const uint32_t s = cursor - 1u - ord;
                    const uint32_t h = breq_target(r, s);
                    if (h != s) {
                        src[m] = s;
                        tgt[m] = h;
                    }
                }
            }
        }
        // Records are read here, before the decision, unless `late`: then
        // only the round's winners read them, after the decision (fewer
        // random reads when a retry would read its records again).
        PRec<EB == 0 ? 4 : EB> r_s[BM], r_h[BM];
        if (EB != 0 && !late) {
#pragma unroll
            for (int m = 0; m < BM; m++)
                if (src[m] != EMPTY) {
                    r_s[m].load(r.A, src[m]);
                    r_h[m].load(r.A, tgt[m]);
                }
        }
        // reserve
#pragma unroll
        for (int m = 0; m < BM; m++) {
            if (src[m] != EMPTY) {
                attempts++;
                const uint32_t v = (tag << BRANKB) | (src[m] - cnew);
                __hip_atomic_fetch_max(&slots[slot1(tgt[m], T)], v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                const uint32_t d = tgt[m] - cnew;
                if (tgt[m] >= cnew && d < W)
                    __hip_atomic_fetch_or(&bm[par * bmw + (d >> 5)], 1u << (d & 31u),
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        for (uint32_t i = lane; i < bmw; i += L)
            lds_st(&bm[(par ^ 1u) * bmw + i], 0u);
        g.sync();
        // commit: decide every slot, then (late) read the winners' records,
        // then write them swapped
        bool win[BM];
#pragma unroll
        for (int m = 0; m < BM; m++) {
            win[m] = false;
            if (src[m] == EMPTY)
                continue;
            const uint32_t s = src[m], h = tgt[m];
            const uint32_t ds = s - cnew;
            const uint32_t v = (tag << BRANKB) | ds;
            bool w = lds_ld(&slots[slot1(h, T)]) == v;
            if (ds < W)
                w = w && !((lds_ld(&bm[par * bmw + (ds >> 5)]) >> (ds & 31u)) & 1u);
            else
                w = w && lds_ld(&slots[slot1(s, T)]) <= v;
            win[m] = w;
        }
        if (EB != 0 && late) {
#pragma unroll
            for (int m = 0; m < BM; m++)
                if (win[m]) {
                    r_s[m].load(r.A, src[m]);
                    r_h[m].load(r.A, tgt[m]);
                }
        }
#pragma unroll
        for (int m = 0; m < BM; m++) {
            if (!win[m])
                continue;
            const uint32_t s = src[m], h = tgt[m];
            if (EB != 0) {
                r_h[m].store(r.A, s);
                r_s[m].store(r.A, h);
            } else {
                pswap_generic(r.A, r.eb, s, h);
            }
            src[m] = EMPTY;
        }
        cursor = cnew;
        rounds++;
    }
    *rounds_out = rounds;
    *attempts_out = attempts;
    *status_out = status;
}

template <int BWAVES>
__device__ __forceinline__ uint64_t sum_over_group_wg(uint64_t v, uint64_t *sh)
{
    v = wave_sum64(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < BWAVES; i++)
        t += sh[i];
    __syncthreads();
    return t;
}


// ---------------------------------------------------------------- planning

// Round-state words for a request at the given table ratio and lane count,
// within the LDS words available; k = 0 means the request needs no rounds.
inline void plan_request(uint64_t n, double eps, double ratio, uint32_t lanes,
                  uint32_t lds_words, uint32_t *k, uint32_t *T, uint32_t *bmw)
{
    *k = *T = *bmw = 0;
    if (n <= 1)
        return;
    const uint64_t bound_bytes = rp_aux_bound_words(n, eps) * 8;
    const uint64_t cap_words = std::min<uint64_t>(bound_bytes / 4, lds_words);
    uint64_t best = 1;
    uint64_t lo = 1, hi = std::min<uint64_t>((uint64_t)lanes * BM, n);
    auto words = [&](uint64_t kk) {
        const uint64_t t = std::max<uint64_t>(1, (uint64_t)std::ceil(ratio * (double)kk));
        const uint64_t b = std::max<uint64_t>(1, (2 * kk + 31) / 32);
        return t + 2 * b;
    };
    while (lo <= hi) {
        const uint64_t mid = (lo + hi) / 2;
        if (words(mid) <= cap_words) {
            best = mid;
            lo = mid + 1;
        } else {
            hi = mid - 1;
        }
    }
    *k = (uint32_t)best;
    *T = (uint32_t)std::max<uint64_t>(1, (uint64_t)std::ceil(ratio * (double)best));
    *bmw = (uint32_t)std::max<uint64_t>(1, (2 * best + 31) / 32);
    if (words(best) > cap_words) {
        // Not even k = 1 with a table fits: run the request with k = 1 and no
        // round state at all (one active swap always commits).
        *k = 1;
        *T = 0;
        *bmw = 0;
    }
}

}  // namespace rpwg
