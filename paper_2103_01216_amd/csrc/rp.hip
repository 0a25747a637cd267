// librp: parallel in-place random permutation for MI355X (gfx950).
//
// Computes exactly the sequential Knuth shuffle (Gu, Obeya, Shun, "Parallel
// In-Place Algorithms: Theory and Practice", Section 4.1) with the relaxed-PIP
// round structure of Section 4.1 (work on the first k unfinished swaps, k on
// the order of n^(1-eps)), realised as the RP-Final scheme of Section 7.4 and
// Appendix A.2: one reservation per swap on R[H[s]], a dense array for the
// keys of the swaps added in the current round, a hash table for all other
// keys.  See include/rp.h for the ABI.
//
// Execution model on the GPU
// --------------------------
// One persistent cooperative kernel runs every round.  Each lane owns up to M
// swap slots held in registers (the active list); a slot is either empty or
// holds an unfinished swap (s, H[s]).  A round is
//   1. gather   all workgroups exchange (free slots, active swaps, oldest
//               active source) through a flag all-gather; from it every
//               workgroup derives the same new cursor and its own contiguous
//               share of the fresh indices, so the active set is always the
//               top unfinished swaps in the sequential order (decreasing
//               index), as the paper requires;
//   2. refill   free slots take fresh indices (decreasing), H[s] is computed
//               (seed mode) or read; self-loops retire at once (Section 4.1
//               removes them; a swap with H[s] = s is a no-op);
//   3. reserve  the priority write of Algorithm 1 on R[H[s]], into a hashed
//               reservation array: R[x] is replaced by the slot R'[h1(x)] of
//               an O(k)-word array (or two slots h1, h2 when two choices are
//               asked for), updated with an atomic max of the swap's
//               priority; bit H[s] of the dense window is set when H[s] lies
//               in it; then both records of every active swap are read;
//   4. barrier  (it waits for the reservations only: the record reads stay
//               in flight across it)
//   5. commit   swap s wins iff it is still the maximum in a slot of key
//               H[s] (so no active swap with a larger source, i.e. earlier
//               in the sequential order, targets H[s]) and no active swap
//               targets s (dense window bit; the slot of key s for the rare
//               source outside the window) -- the single-reservation test of
//               Appendix A.2.  Winners swap A[s] and A[H[s]]; losers stay in
//               their slots for the next round (the paper's pack step becomes
//               the per-workgroup prefix sum over free slots in step 1).
//
// Why the hashed array is exact: a slot holds the maximum priority over all
// keys that hash to it, so "s is the maximum in a slot of key x" implies that
// no active swap with higher priority reserved x (it would have raised every
// slot of x).  Collisions between different keys can only make a swap lose a
// round it could have won (it retries next round; the top unfinished swap is
// the maximum everywhere and always commits), never win wrongly.  The array
// has about one slot per active swap when the bound limits k, and up to four
// when the grid does and the bound leaves words to spare.
//
// Priorities are (tag:8 | rank:24) with rank = s - cursor_new and tag = round
// number mod 256, so values written in later rounds are larger and the array
// needs no cleaning between rounds; every 256 rounds all slots are reset
// behind an extra barrier.  The refill is throttled so that ranks stay below
// 2^24.  The dense window is double-buffered by round parity and the stale
// parity is cleared during step 3: the cleaning phase of Appendix A.1.
//
// Auxiliary layout (device memory, or LDS for the slot array and window of a
// one-workgroup launch; every byte counted against the bound):
//   slots[T]            hashed reservation array, 32-bit priorities
//   bm[par * bmw + i]   dense window: bit x set iff an active swap targets
//                       cursor_new + x, for x < 32 * bmw (at least 2k)
//   flags[par * G + w]  gather flags: epoch:16 | payload:48
//   err                 watchdog / error word
// RP-Final keeps R for the round's consecutive keys in a prefix-sized array;
// here that array holds one bit per key, because the commit test only asks
// whether any other active swap targets the source.
//
// Cross-workgroup data is accessed only with device-coherent relaxed
// agent-scope atomics.  A workgroup waits for all of its memory operations to
// complete before it publishes its barrier flag, and every access after a
// barrier is issued after the flags were observed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "rp.h"
#include "rp_device.h"
#include "rp_resident.h"
#include "rp_wg.h"

namespace {

using namespace rpdev;

constexpr int WG = 256;                 // threads per workgroup
constexpr int WAVES = WG / 64;
constexpr uint32_t TAG_CYCLE = 256;     // rounds between full resets
constexpr int MAXG = 2048;              // largest grid the gather supports
constexpr int POLL = 4;                 // barrier flags a lane loads at once
constexpr uint32_t LDS_TAB_BYTES = 65536;  // largest LDS table of such a launch
constexpr uint64_t WATCHDOG_TICKS = 500000000ull;  // 5 s at 100 MHz
constexpr double TABLE_RATIO = 1.0;     // reservation slots per active swap
constexpr double SPARE_RATIO_MAX = 4.0; // the most when spare words allow more

struct Params {
    unsigned char *A;
    const uint64_t *H;   // nullptr: seed mode
    uint64_t seed;
    uint32_t n;
    uint32_t eb;
    uint32_t k;
    uint32_t T;          // reservation slots
    uint32_t bmw;        // dense-window words per parity
    uint32_t choices;    // reservation slots per key: 1 or 2
    uint32_t *slots;
    uint32_t *bm;
    uint64_t *flags;
    uint32_t *err;
    uint64_t *dstats;    // rp_stats laid out as S_WORDS 64-bit words
    uint64_t max_rounds;
    uint32_t rank_cap;   // refill throttle: active ranks stay below this
    uint32_t variant;    // RP_VARIANT_*: how reservations are held and checked
    uint32_t lds_tab;    // 1: the launch uses the LDS variant of the kernel
    uint64_t *R64;       // RP_VARIANT_LINEAR: one priority word per position
    uint32_t *hflat;     // RP_VARIANT_FLAT: H of each active swap, by swap slot
    uint64_t *htab;      // RP_VARIANT_NAIVE: hashed (source + 1, H) pairs, two parities
    uint32_t hcap;       // RP_VARIANT_NAIVE: entries per parity (a power of two)
    uint32_t wg_first;   // this shuffle's workgroups: [wg_first, wg_first + wg_count)
    uint32_t wg_count;   // of the launch (all of it, except in a group launch)
    uint32_t chunk_log2; // one-barrier kernel: fresh indices are dealt in chunks of 2^this
};

// rp_stats word indices
enum { S_K, S_AUX, S_BOUND, S_ROUNDS, S_ATTEMPTS, S_RETRIES, S_MAXACT,
       S_SELF, S_GRID, S_SLOTS, S_TABLE, S_STATUS, S_INFLIGHT, S_THROTTLED,
       S_WORDS };
static_assert(S_WORDS * 8 == sizeof(rp_stats), "rp_stats layout");

__device__ __forceinline__ uint32_t target_of(const Params &p, uint32_t s)
{
    return p.H ? (uint32_t)p.H[s] : seed_target(p.seed, s);
}

// --------------------------------------------------------------- the gather

// Wave 0 of every workgroup (w: its index among the p.wg_count workgroups of
// the shuffle): publish the 48-bit `payload` under `epoch`,
// wait for every workgroup's flag of the same epoch and hand each payload to
// `visit` (lane-strided).  Flags hold epoch:16 | payload:48 and are
// double-buffered by epoch parity: a workgroup cannot publish epoch e+2
// before every workgroup has read epoch e, so 16 epoch bits never alias.
// Returns false when the watchdog fired.  The caller has made this
// workgroup's memory operations complete (wait_mem in every wave, then a
// workgroup barrier) before calling.
template <typename Visit>
__device__ __forceinline__ bool gather_wave0(const Params &p, uint32_t w, uint32_t epoch,
                                             uint64_t payload, Visit visit)
{
    const uint32_t G = p.wg_count, lane = threadIdx.x & 63;
    const uint32_t e16 = epoch & 0xFFFFu;
    uint64_t *fl = p.flags + (uint64_t)(epoch & 1u) * G;
    if (lane == 0)
        st(&fl[w], ((uint64_t)e16 << 48) | payload);
    // Poll every flag this lane covers at once; look at the clock and the
    // error word only every 64 sweeps so that a sweep costs one load latency.
    const int nj = (int)((G + 63u) / 64u);
    uint32_t pending = 0;
#pragma unroll 1
    for (int j = 0; j < nj; j++)
        pending |= (lane + 64u * j < G) ? (1u << j) : 0u;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    bool ok = true;
    for (uint32_t sweep = 1; pending; sweep++) {
        // Issue the loads of up to POLL flags before looking at any of them,
        // so that a sweep costs about one load latency, not one per flag.
#pragma unroll 1
        for (int j0 = 0; j0 < nj; j0 += POLL) {
            uint64_t f[POLL];
#pragma unroll
            for (int u = 0; u < POLL; u++) {
                const int j = j0 + u;
                f[u] = (j < nj && (pending & (1u << j))) ? ld(&fl[lane + 64u * j]) : 0ull;
            }
#pragma unroll
            for (int u = 0; u < POLL; u++) {
                const int j = j0 + u;
                if (j < nj && (pending & (1u << j)) && (uint32_t)(f[u] >> 48) == e16) {
                    pending &= ~(1u << j);
                    visit(lane + 64u * j, f[u] & ((1ull << 48) - 1));
                }
            }
        }
        if (pending && (sweep & 63u) == 0) {
            if (__builtin_amdgcn_s_memrealtime() - t0 > WATCHDOG_TICKS ||
                ld(p.err) != 0u) {
                st(p.err, 1u);
                ok = false;
                break;
            }
        }
        if (pending)
            __builtin_amdgcn_s_sleep(1);
    }
    asm volatile("" ::: "memory");
    return __all(ok);
}

// -------------------------------------------------------------- the kernel

// Barrier with no payload (the periodic reset of the reservation array).
__device__ __forceinline__ bool plain_barrier(const Params &p, uint32_t w, uint32_t epoch,
                                              uint64_t *sh_res)
{
    wait_mem();
    __syncthreads();
    if ((threadIdx.x >> 6) == 0) {
        bool ok = true;
        if (p.wg_count > 1)
            ok = gather_wave0(p, w, epoch, 0, [](uint32_t, uint64_t) {});
        if ((threadIdx.x & 63) == 0)
            sh_res[3] = ok ? 0u : 1u;
    }
    __syncthreads();
    return sh_res[3] == 0;
}

// The naive variant's table of H: open addressing with linear probing over
// `cap` 64-bit entries (source + 1) << 32 | H, 0 = empty; at most half full.
__device__ __forceinline__ uint32_t htab_home(uint32_t key, uint32_t cap)
{
    return (uint32_t)(((uint64_t)key * 0xD6E8FEB86659FD93ull) >> 32) & (cap - 1u);
}

__device__ __forceinline__ void htab_insert(uint64_t *tab, uint32_t cap, uint32_t key,
                                            uint32_t val)
{
    const uint64_t e = ((uint64_t)(key + 1u) << 32) | val;
    uint32_t i = htab_home(key, cap);
    for (uint32_t probe = 0; probe < cap; probe++) {
        uint64_t expect = 0;
        if (__hip_atomic_compare_exchange_strong(&tab[i], &expect, e, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        i = (i + 1u) & (cap - 1u);
    }
}

// H of `key`, or sets *missing when the key is absent (never, in a correct
// round: every active swap inserted its pair in this round's parity).
__device__ __forceinline__ uint32_t htab_find(const uint64_t *tab, uint32_t cap, uint32_t key,
                                              bool *missing)
{
    uint32_t i = htab_home(key, cap);
    for (uint32_t probe = 0; probe < cap; probe++) {
        const uint64_t e = ld(&tab[i]);
        if ((uint32_t)(e >> 32) == key + 1u)
            return (uint32_t)e;
        if (e == 0)
            break;
        i = (i + 1u) & (cap - 1u);
    }
    *missing = true;
    return 0;
}

// The rounds of one shuffle on its workgroups.  HX: the flat and naive
// variants (H of the active swaps outside the registers) are compiled in.
// M: swap slots per lane.  EB:
// record size held in registers (4, 8, 16), or 0 for any multiple of 4 up to
// 256 bytes, moved after the decision.  LDS: a one-workgroup launch whose
// slot array and window live in dynamic LDS.
template <int M, int EB, bool LDS, bool HX = false>
__device__ __forceinline__ void rounds_body(const Params &p)
{
    __shared__ uint32_t sh_wave[WAVES];
    __shared__ uint32_t sh_age[WAVES];
    __shared__ uint64_t sh_res[5];

    const uint32_t G = p.wg_count, w = blockIdx.x - p.wg_first, t = threadIdx.x;
    const uint32_t wave = t >> 6, lane = t & 63;
    // Dense window only in the final variant: the one-reservation variant
    // checks sources through the hashed slots, the two-reservation one
    // reserves sources there, the linear one has exact per-position words.
    const uint32_t W = p.variant == RP_VARIANT_FINAL ? p.bmw * 32u : 0u;
    const bool linear = p.variant == RP_VARIANT_LINEAR;
    // Algorithm 1's two reservations: the two-reservation variant holds H of
    // every active swap in registers, the flat one in a prefix-sized array
    // indexed by the swap's slot, the naive one in a hashed table keyed by
    // the source.
    const bool flat = HX && p.variant == RP_VARIANT_FLAT;
    const bool naive = HX && p.variant == RP_VARIANT_NAIVE;
    const bool twores = p.variant == RP_VARIANT_TWORES || flat || naive;

    // A one-workgroup launch keeps its slot array and window in LDS (the
    // same words, on chip): its rounds are then workgroup barriers and LDS
    // atomics.
    uint32_t *slots = p.slots, *bm = p.bm;
    if constexpr (LDS) {
        extern __shared__ uint32_t dyn_lds[];
        slots = dyn_lds;
        bm = dyn_lds + p.T;
        for (uint32_t i = t; i < p.T + 2 * p.bmw; i += WG)
            dyn_lds[i] = 0u;
        __syncthreads();
    }

    uint32_t src[M], tgt[M];
    bool usable[M];
#pragma unroll
    for (int m = 0; m < M; m++) {
        usable[m] = ((uint64_t)m * G * WG + (uint64_t)w * WG + t) < p.k;
        src[m] = EMPTY;
        tgt[m] = 0;
    }
    uint32_t cursor = p.n;  // fresh swaps are the indices below the cursor
    uint32_t epoch = 0;
    uint64_t rounds = 0, attempts = 0, retries = 0, selfl = 0, maxact = 0,
             throttled = 0;
    bool failed = false;

    for (;;) {
        // ---- 1. gather: free slots, active swaps, oldest active source
        uint32_t f = 0, a = 0, age = 0;
#pragma unroll
        for (int m = 0; m < M; m++) {
            f += (usable[m] && src[m] == EMPTY) ? 1u : 0u;
            if (src[m] != EMPTY) {
                a++;
                age = max(age, min(src[m] - cursor, RANKMAX));  // losers: src >= cursor
            }
        }
        const uint32_t x = (a << 16) | f;  // both sums stay below 2^12
        const uint32_t xi = wave_incl_scan(x);
        const uint32_t agew = wave_max(age);
        if (lane == 63)
            sh_wave[wave] = xi;
        if (lane == 0)
            sh_age[wave] = agew;
        wait_mem();
        __syncthreads();
        uint32_t below = 0, wgtot = 0, wgage = 0;
#pragma unroll
        for (int i = 0; i < WAVES; i++) {
            const uint32_t v = sh_wave[i];
            below += ((uint32_t)i < wave) ? v : 0u;
            wgtot += v;
            wgage = max(wgage, sh_age[i]);
        }
        const uint32_t lane_off = (below + xi - x) & 0xFFFFu;
        ++epoch;
        if (wave == 0) {
            uint64_t pre = 0, totF = 0, totA = 0;
            uint32_t agemax = 0;
            bool ok = true;
            if (G == 1) {
                totF = wgtot & 0xFFFFu;
                totA = wgtot >> 16;
                agemax = wgage;
            } else {
                const uint64_t pay = ((uint64_t)(wgtot >> 16) << 36) |
                                     ((uint64_t)(wgtot & 0xFFFFu) << 24) | wgage;
                ok = gather_wave0(p, w, epoch, pay, [&](uint32_t v, uint64_t y) {
                    const uint32_t fv = (uint32_t)(y >> 24) & 0xFFFu;
                    pre += (v < w) ? fv : 0u;
                    totF += fv;
                    totA += (uint32_t)(y >> 36) & 0xFFFu;
                    agemax = max(agemax, (uint32_t)y & RANKMAX);
                });
                pre = wave_sum64(pre);
                totF = wave_sum64(totF);
                totA = wave_sum64(totA);
                agemax = wave_max(agemax);
            }
            if (lane == 0) {
                sh_res[0] = pre;
                sh_res[1] = totF;
                sh_res[2] = totA;
                sh_res[3] = ok ? 0u : 1u;
                sh_res[4] = agemax;
            }
        }
        __syncthreads();
        const uint64_t pre = sh_res[0], totF = sh_res[1], totA = sh_res[2];
        const uint32_t agemax = (uint32_t)sh_res[4];
        if (sh_res[3]) {
            failed = true;
            break;
        }
        if (cursor == 0 && totA == 0)
            break;
        if (rounds >= p.max_rounds) {
            if (t == 0)
                st(p.err, 2u);
            failed = true;
            break;
        }
        // Fresh swaps, throttled so that every active rank fits in 24 bits
        // (below rank_cap, which is 2^24 - 1 unless a test lowers it).
        const uint64_t want = min<uint64_t>(totF, cursor);
        const uint64_t room = agemax < p.rank_cap ? (uint64_t)(p.rank_cap - agemax) : 0ull;
        const uint32_t take = (uint32_t)min<uint64_t>(want, room);
        throttled += take < want ? 1u : 0u;
        const uint32_t cnew = cursor - take;
        const uint32_t par = (uint32_t)(rounds & 1);
        const uint32_t tag = (uint32_t)(rounds % TAG_CYCLE);

        // Every TAG_CYCLE rounds: reset the reservation array behind an
        // extra barrier, so that tags restart from 0 over an empty array.
        if (tag == 0 && rounds > 0 && !linear) {
            for (uint32_t i = w + G * t; i < p.T; i += G * WG)
                clear_rmw(&slots[i]);
            if (!plain_barrier(p, w, ++epoch, sh_res)) {
                failed = true;
                break;
            }
        }

        // ---- 2. refill free slots with fresh indices, decreasing
        uint32_t j = (uint32_t)pre + lane_off;
#pragma unroll
        for (int m = 0; m < M; m++) {
            if (usable[m] && src[m] == EMPTY) {
                const uint32_t ord = j++;
                if (ord < take) {
                    const uint32_t s = cursor - 1u - ord;
                    const uint32_t h = target_of(p, s);
                    if (h == s) {
                        selfl++;
                    } else {
                        src[m] = s;
                        tgt[m] = h;
                        if (flat)
                            st(&p.hflat[(uint64_t)m * G * WG + (uint64_t)w * WG + t], h);
                    }
                }
            }
        }
        // ---- 3. reserve: clean the stale window parity (and the naive
        // table's stale parity, whose last lookups were before the gather);
        // priority write on the slot(s) of H[s]; dense window bit
        {
            const uint32_t op = par ^ 1u;
            for (uint32_t i = w + G * t; i < p.bmw; i += G * WG)
                clear_rmw(&bm[(uint64_t)op * p.bmw + i]);
            if (naive)
                for (uint32_t i = w + G * t; i < p.hcap; i += G * WG)
                    (void)__hip_atomic_exchange(&p.htab[(uint64_t)op * p.hcap + i], (uint64_t)0,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // H of every active swap for this round's reservations: read back
        // from the flat array, or (naive) set in this round's table.
        if (flat || naive) {
#pragma unroll
            for (int m = 0; m < M; m++) {
                if (src[m] == EMPTY)
                    continue;
                if (flat)
                    tgt[m] = ld(&p.hflat[(uint64_t)m * G * WG + (uint64_t)w * WG + t]);
                else
                    htab_insert(p.htab + (uint64_t)par * p.hcap, p.hcap, src[m], tgt[m]);
            }
        }
        uint32_t act = 0;
#pragma unroll
        for (int m = 0; m < M; m++) {
            if (src[m] != EMPTY) {
                act++;
                if (linear) {
                    // round + 1 in the high word: later rounds beat every
                    // older value, so the array is never cleaned.
                    const uint64_t v64 = ((rounds + 1) << 32) | (src[m] - cnew);
                    __hip_atomic_fetch_max(&p.R64[tgt[m]], v64, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    continue;
                }
                const uint32_t v = (tag << RANKB) | (src[m] - cnew);
                __hip_atomic_fetch_max(&slots[slot1(tgt[m], p.T)], v,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (p.choices > 1)
                    __hip_atomic_fetch_max(&slots[slot2(tgt[m], p.T)], v,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (twores)
                    __hip_atomic_fetch_max(&slots[slot1(src[m], p.T)], v,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t d = tgt[m] - cnew;
                if (tgt[m] >= cnew && d < W)
                    __hip_atomic_fetch_or(&bm[(uint64_t)par * p.bmw + (d >> 5)],
                                          1u << (d & 31u), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        attempts += act;

        // Read both records of every active swap now, after the
        // reservations.  If the swap wins this round, no other winner touches
        // either location, and every earlier round's writes completed before
        // the gather above, so these values are exactly the ones the swap
        // exchanges.  Exactly two loads per slot are issued (an empty slot
        // reads record 0 and ignores it), so that the wait below can let
        // them stay in flight across the barrier: vector memory operations
        // of a wave complete in issue order, and the barrier needs only the
        // reservations and the window clears, issued before them.
        Rec<EB == 0 ? 4 : EB> r_s[M], r_h[M];
        constexpr bool hoisted = EB != 0;
        if constexpr (hoisted) {
#pragma unroll
            for (int m = 0; m < M; m++) {
                const bool on = src[m] != EMPTY;
                r_s[m].load(p.A, on ? src[m] : 0u);
                r_h[m].load(p.A, on ? tgt[m] : 0u);
            }
        }

        // ---- 4. barrier (wave 0 of workgroup 0 also totals the attempts)
        {
            const uint32_t ai = wave_incl_scan(act);
            if (lane == 63)
                sh_wave[wave] = ai;
        }
        if constexpr (hoisted)
            wait_mem_but<2 * M * Rec<EB == 0 ? 4 : EB>::LOADS>();
        else
            wait_mem();
        __syncthreads();
        ++epoch;
        if (wave == 0) {
            uint32_t actw = 0;
#pragma unroll
            for (int i = 0; i < WAVES; i++)
                actw += sh_wave[i];
            bool ok = true;
            uint64_t tot = 0;
            if (G == 1)
                tot = actw;
            else
                ok = gather_wave0(p, w, epoch, actw,
                                  [&](uint32_t, uint64_t y) { tot += y; });
            tot = wave_sum64(tot);
            if (lane == 0) {
                sh_res[3] = ok ? 0u : 1u;
                maxact = max(maxact, tot);
            }
        }
        __syncthreads();
        if (sh_res[3]) {
            failed = true;
            break;
        }

        // ---- 5. commit test and swap: issue every load, then decide.  The
        // flat and naive variants read H back first (array, or table).
        if (flat || naive) {
#pragma unroll
            for (int m = 0; m < M; m++) {
                if (src[m] == EMPTY)
                    continue;
                bool missing = false;
                tgt[m] = flat ? ld(&p.hflat[(uint64_t)m * G * WG + (uint64_t)w * WG + t])
                              : htab_find(p.htab + (uint64_t)par * p.hcap, p.hcap, src[m],
                                          &missing);
                if (missing) {
                    // Cannot happen in a correct round; keep the result
                    // right and report it in the status.
                    tgt[m] = target_of(p, src[m]);
                    st(&p.dstats[S_STATUS], (uint64_t)(int64_t)RP_EDEVICE);
                }
            }
        }
        uint32_t t1[M], t2[M], q1[M], q2[M];
#pragma unroll
        for (int m = 0; m < M; m++) {
            if (src[m] == EMPTY)
                continue;
            const uint32_t s = src[m], h = tgt[m];
            const uint32_t ds = s - cnew;  // s >= cnew for every active swap
            if (linear) {
                // (t2:t1) = R[H[s]], (q2:q1) = R[s]
                const uint64_t a = ld(&p.R64[h]), b = ld(&p.R64[s]);
                t1[m] = (uint32_t)a;
                t2[m] = (uint32_t)(a >> 32);
                q1[m] = (uint32_t)b;
                q2[m] = (uint32_t)(b >> 32);
                continue;
            }
            t1[m] = ld(&slots[slot1(h, p.T)]);
            t2[m] = (p.choices > 1) ? ld(&slots[slot2(h, p.T)]) : 0u;
            if (ds < W) {
                q1[m] = ld(&bm[(uint64_t)par * p.bmw + (ds >> 5)]);
            } else {
                q1[m] = ld(&slots[slot1(s, p.T)]);
                q2[m] = (p.choices > 1) ? ld(&slots[slot2(s, p.T)]) : 0u;
            }
        }
#pragma unroll
        for (int m = 0; m < M; m++) {
            if (src[m] == EMPTY)
                continue;
            const uint32_t s = src[m], h = tgt[m];
            const uint32_t ds = s - cnew;
            const uint32_t v = (tag << RANKB) | ds;
            // Target: still the maximum in a slot of H[s].
            const bool two = p.choices > 1;
            bool win = (t1[m] == v) || (two && t2[m] == v);
            // Source: no active swap targets s.  Such a swap has a larger
            // source, so it would have raised both slots of key s above v.
            if (ds < W)
                win = win && !((q1[m] >> (ds & 31u)) & 1u);
            else
                win = win && (q1[m] <= v || (two && q2[m] <= v));
            if (twores)  // Algorithm 1: both reservations must hold
                win = (t1[m] == v) && (q1[m] == v);
            if (linear) {
                // exact: the maximum on H[s] is this swap, and no swap of
                // this round reserved s
                const uint32_t rid = (uint32_t)(rounds + 1);
                win = t2[m] == rid && t1[m] == ds && q2[m] != rid;
            }
            if (win) {
                if (EB != 0) {
                    r_h[m].store(p.A, s);
                    r_s[m].store(p.A, h);
                } else {
                    swap_generic(p.A, p.eb, s, h);
                }
                src[m] = EMPTY;
            } else {
                retries++;
            }
        }
        cursor = cnew;
        rounds++;
    }

    // ---- statistics
    uint64_t s_att = wave_sum64(attempts), s_ret = wave_sum64(retries),
             s_self = wave_sum64(selfl);
    if (lane == 0) {
        __hip_atomic_fetch_add(&p.dstats[S_ATTEMPTS], s_att, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&p.dstats[S_RETRIES], s_ret, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&p.dstats[S_SELF], s_self, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    if (t == 0) {
        if (w == 0) {
            st(&p.dstats[S_ROUNDS], rounds);
            st(&p.dstats[S_MAXACT], maxact);
            st(&p.dstats[S_THROTTLED], throttled);
        }
        if (failed)
            st(&p.dstats[S_STATUS], (uint64_t)(int64_t)RP_ETIMEOUT);
    }
}

template <int M, int EB, bool LDS, bool HX = false>
__global__ __launch_bounds__(WG) void rp_rounds_kernel(Params p)
{
    rounds_body<M, EB, LDS, HX>(p);
}

// ------------------------------------------------- one barrier per round
//
// When the auxiliary bound, not the grid, limits k (the swaps fit one per
// lane with a few hundred per workgroup), the rounds run with one grid
// barrier each instead of two.  Between two barriers a workgroup checks and
// commits round r and refills and reserves round r+1.  What the second
// barrier of rounds_body provides is obtained otherwise:
//   * Fresh indices are handed out by quota.  At each barrier every
//     workgroup learns the active swaps and the swaps just committed of all
//     workgroups, and all of them derive the same quota q for the next
//     refill: enough fresh swaps to bring the active total back to about k,
//     never more than the fullest workgroup has free slots, never so many
//     that a rank leaves its field.  Workgroup w then takes the fresh indices
//     cursor-1-(w*q+j), j < q: the union over workgroups is the next
//     contiguous range below the cursor, so the active swaps stay the top
//     unfinished ones in sequential order, without a second exchange after
//     the commits.  A workgroup has WG1 lanes for about PER_WG1 active swaps,
//     so the quota always finds free slots.
//   * Records are read after the barrier, together with the check loads:
//     the barrier follows every commit of the previous round.  The targets
//     of the next fresh indices are computed (into LDS) while those loads are
//     in flight.
//   * A fast workgroup's reservations of round r+1 may land while a slow one
//     still checks round r.  They carry a larger round tag, so they can only
//     make such a check lose, never win wrongly.  The top active swap (whose
//     rank every workgroup learns at the barrier) commits regardless: nothing
//     active precedes it, so it always may, and every round makes progress.
//   * The dense window has three parities.  Round r+1 sets parity (r+1) mod 3
//     and clears parity (r+2) mod 3, whose last readers (the checks of round
//     r-1) finished before the barrier that opened round r.
constexpr int WG1 = 512;                // lanes of a one-barrier workgroup
constexpr int WAVES1 = WG1 / 64;
constexpr uint32_t PER_WG1 = 256;       // most active swaps per workgroup the grid is sized for
constexpr uint32_t MIN_PER_WG1 = 64;    // fewest, when the grid is widened
constexpr uint32_t WIDE_NUM = 11, WIDE_DEN = 16;  // widened grid: 11/16 of the compute units
constexpr uint32_t WPAR1 = 3;           // window parities
constexpr double WFRAC1 = 1.5;          // window keys per active swap

// The fresh indices of a round, cursor-1-o for o in [0, take), are dealt to
// the workgroups in chunks of C = 2^chunk_log2 consecutive indices, round
// robin: the j-th fresh index of workgroup w is o = fresh_ord(w, j, G, c).
// Dealing whole blocks (workgroup 0 the top block) made the workgroups
// holding the highest-priority fresh swaps win, and so move records, more
// than the others; chunks keep a chunk's records in one or a few cache lines.
// Quotas are whole chunks, so the planner keeps G * C within k / 16 (the
// active total then stays within a few percent of k).
constexpr uint32_t MAX_CHUNK_LOG2 = 3;

// Arrays up to this size read every active swap's records with its check
// loads; larger ones only the winners', after the decision.  Measured on the
// one-barrier kernel (ms, early / after): 2^20 int64 3.6 / 4.6, 2^28 int64
// 90.8 / 95.1; but 2^26 x 64 B 66.4 / 64.7 and 2^30 int64 256.2 / 248.2 -- over
// a few GiB of random reads the losers' extra loads miss the address
// translation caches and cost more than the overlap saves.
constexpr uint64_t EARLY_RECS_MAX_BYTES = 2ull << 30;

uint32_t early_recs_for(uint64_t n, uint32_t eb)
{
    const char *v = getenv("RP_EARLY_RECS");   // tuning override: 0 or 1
    if (v && *v)
        return atoi(v) != 0 ? 1u : 0u;
    return n * eb <= EARLY_RECS_MAX_BYTES ? 1u : 0u;
}

__device__ __forceinline__ uint32_t fresh_ord(uint32_t w, uint32_t j, uint32_t G, uint32_t cl)
{
    return ((w + G * (j >> cl)) << cl) + (j & ((1u << cl) - 1u));
}

// The rounds of one shuffle on workgroup w of its p.wg_count, with flag
// epochs counted from `epoch0` (the last epoch used before, on the same
// flags); returns the last epoch it used.  EARLY: every active swap reads
// its records with its check loads (else only the winners, after the
// decision).
template <int EB, bool EARLY>
__device__ __forceinline__ uint32_t rounds1_body(const Params &p, uint32_t w, uint32_t epoch0)
{
    __shared__ uint32_t sh_scan[WAVES1];
    __shared__ uint32_t sh_pay[WAVES1];
    __shared__ uint32_t sh_age[WAVES1];
    __shared__ uint32_t sh_h[WG1];
    __shared__ uint64_t sh_res[6];

    const uint32_t G = p.wg_count, t = threadIdx.x;
    const uint32_t wave = t >> 6, lane = t & 63;
    const uint32_t W = p.bmw * 32u;
    uint32_t *const slots = p.slots;
    uint32_t *const bm = p.bm;
    using R = Rec<EB == 0 ? 4 : EB>;

    uint32_t epoch = epoch0;
    uint32_t src = EMPTY, tgt = 0;
    uint32_t cursor = p.n;        // rank base of the round last reserved
    uint64_t rr = 0;              // rounds reserved so far
    uint64_t attempts = 0, retries = 0, selfl = 0, maxact = 0, throttled = 0;
    bool failed = false;
    uint32_t q = (uint32_t)min<uint64_t>(((uint64_t)p.k + G - 1) / G, (uint64_t)WG1);
    q = max(q >> p.chunk_log2, 1u) << p.chunk_log2;
    uint32_t take = (uint32_t)min<uint64_t>((uint64_t)G * q, p.n);
    uint32_t top = EMPTY;         // rank of the top active swap of the round to check
    uint64_t prevA = 0;           // active swaps of the round checked last
    const double rG = 1.0 / (double)G;

    // what the last barrier gathered: active swaps, swaps just committed,
    // the fullest workgroup's active swaps, the oldest active rank
    uint64_t g_act = 0, g_won = 0;
    uint32_t g_maxa = 0, g_age = 0;
    for (;;) {
        // ---- check round rr-1: issue the loads the decision needs
        const bool act = src != EMPTY;
        const uint32_t ds = src - cursor;
        uint32_t t1 = 0, q1 = 0;
        if (act) {
            const uint32_t par = (uint32_t)((rr - 1) % WPAR1);
            t1 = ld(&slots[slot1(tgt, p.T)]);
            q1 = ds < W ? ld(&bm[(uint64_t)par * p.bmw + (ds >> 5)])
                        : ld(&slots[slot1(src, p.T)]);
        }
        // Records read early (small arrays): issued with the check loads,
        // their latency overlaps the check's; a loser's are dropped.
        R r_s, r_h;
        if constexpr (EB != 0 && EARLY) {
            if (act) {
                r_s.load(p.A, src);
                r_h.load(p.A, tgt);
            }
        }
        if (rr > 0) {
            // ---- quota of this refill (the same in every workgroup): the
            // active swaps that will remain after the check are estimated
            // from the last check's win rate, and the quota refills them to
            // k.  (All counts are below 2^32; the quotients are taken in
            // double precision, which every workgroup evaluates identically
            // and which is exact for these magnitudes.)
            top = g_act ? g_age : EMPTY;
            const uint32_t a32 = (uint32_t)g_act;
            const uint32_t expect_w =
                prevA ? (uint32_t)((double)g_act * (double)g_won / (double)prevA) : a32 / 2u;
            prevA = g_act;
            const uint32_t want = p.k + expect_w > a32 ? p.k + expect_w - a32 : 0u;
            // Whole chunks (see fresh_ord): the target rounded to the nearest
            // chunk, the limits rounded down.
            const uint32_t C = 1u << p.chunk_log2;
            uint32_t qq = ((uint32_t)std::ceil((double)want * rG) + C / 2) / C * C;
            qq = min(qq, ((uint32_t)WG1 - g_maxa) / C * C);
            const uint32_t room =
                g_age < p.rank_cap ? (uint32_t)((double)(p.rank_cap - g_age) * rG) / C * C : 0u;
            if (qq > room) {
                qq = room;
                throttled++;
            }
            if (qq == 0 && g_act == 0 && cursor > 0)
                qq = C;
            q = qq;
            take = (uint32_t)min<uint64_t>((uint64_t)G * q, cursor);
        }
        // ---- meanwhile: targets of this workgroup's fresh indices
        if (t < q) {
            const uint32_t o = fresh_ord(w, t, G, p.chunk_log2);
            if (o < take)
                sh_h[t] = target_of(p, cursor - 1u - o);
        }
        // ---- decide (the records are not needed for it; winners move them
        // while the refill and the reservations proceed)
        uint32_t won = 0;
        const uint32_t ws = src, wt = tgt;
        if (act) {
            const uint32_t tag = (uint32_t)((rr - 1) % TAG_CYCLE);
            const uint32_t v = (tag << RANKB) | ds;
            // Target: still the maximum in the slot of H[s].  Source: no
            // active swap targets s (window bit, or the slot of key s).
            bool win = t1 == v;
            if (ds < W)
                win = win && !((q1 >> (ds & 31u)) & 1u);
            else
                win = win && q1 <= v;
            win = win || ds == top;
            attempts++;
            if (win) {
                src = EMPTY;
                won = 1;
            } else {
                retries++;
            }
        }
        // Otherwise winners read both records now (the barrier followed every
        // commit of the previous round, and no other winner of this round
        // touches them).  Either way they are written back swapped after the
        // reservations.
        if constexpr (EB != 0 && !EARLY) {
            if (won) {
                r_s.load(p.A, ws);
                r_h.load(p.A, wt);
            }
        }
        // ---- refill: the free slots take the fresh indices in order
        const bool f = src == EMPTY;
        const uint64_t fb = __ballot(f);
        if (lane == 0)
            sh_scan[wave] = (uint32_t)__popcll(fb);
        __syncthreads();
        uint32_t below = 0;
#pragma unroll
        for (int i = 0; i < WAVES1; i++)
            below += ((uint32_t)i < wave) ? sh_scan[i] : 0u;
        const uint32_t j = below + lane_rank(fb);
        const uint32_t oj = fresh_ord(w, j, G, p.chunk_log2);
        if (f && j < q && oj < take) {
            const uint32_t s = cursor - 1u - oj;
            const uint32_t h = sh_h[j];
            if (h == s) {
                selfl++;
            } else {
                src = s;
                tgt = h;
            }
        }
        cursor -= take;
        const uint32_t tag = (uint32_t)(rr % TAG_CYCLE);

        // Every TAG_CYCLE rounds the reservation array is reset between two
        // extra barriers: the first lets every workgroup finish its checks
        // of the old tags, the second every clear before a reservation with
        // the new ones.
        if (tag == 0 && rr > 0) {
            if (!plain_barrier(p, w, ++epoch, sh_res)) {
                failed = true;
                break;
            }
            for (uint32_t i = w + G * t; i < p.T; i += G * WG1)
                clear_rmw(&slots[i]);
            if (!plain_barrier(p, w, ++epoch, sh_res)) {
                failed = true;
                break;
            }
        }
        // ---- reserve round rr
        {
            const uint32_t cp = (uint32_t)((rr + 1) % WPAR1);
            for (uint32_t i = w + G * t; i < p.bmw; i += G * WG1)
                clear_rmw(&bm[(uint64_t)cp * p.bmw + i]);
        }
        if (src != EMPTY) {
            const uint32_t v = (tag << RANKB) | (src - cursor);
            __hip_atomic_fetch_max(&slots[slot1(tgt, p.T)], v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t d = tgt - cursor;
            if (tgt >= cursor && d < W)
                __hip_atomic_fetch_or(&bm[(uint64_t)(rr % WPAR1) * p.bmw + (d >> 5)],
                                      1u << (d & 31u), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
        }
        rr++;
        // ---- winners of the round just checked exchange their records
        if (won) {
            if constexpr (EB != 0) {
                r_h.store(p.A, ws);
                r_s.store(p.A, wt);
            } else {
                swap_generic(p.A, p.eb, ws, wt);
            }
        }

        // ---- barrier: active swaps, swaps just committed, oldest rank
        const bool a = src != EMPTY;
        const uint32_t xw = ((uint32_t)__popcll(__ballot(a)) << 16) |
                            (uint32_t)__popcll(__ballot(won != 0));
        const uint32_t agew = wave_max_dpp(a ? src - cursor : 0u);
        if (lane == 0)
            sh_pay[wave] = xw;
        if (lane == 0)
            sh_age[wave] = agew;
        wait_mem();
        __syncthreads();
        ++epoch;
        if (wave == 0) {
            uint32_t wgx = 0, wgage = 0;
#pragma unroll
            for (int i = 0; i < WAVES1; i++) {
                wgx += sh_pay[i];
                wgage = max(wgage, sh_age[i]);
            }
            uint64_t totA = 0, totW = 0;
            uint32_t maxA = 0, agemax = 0;
            bool ok = true;
            const uint64_t pay = ((uint64_t)(wgx >> 16) << 34) |
                                 ((uint64_t)(wgx & 0xFFFFu) << 24) | wgage;
            if (G == 1) {
                totA = maxA = wgx >> 16;
                totW = wgx & 0xFFFFu;
                agemax = wgage;
            } else {
                uint32_t sa = 0, sw = 0;
                ok = gather_wave0(p, w, epoch, pay, [&](uint32_t, uint64_t y) {
                    const uint32_t av = (uint32_t)(y >> 34) & 0x3FFFu;
                    sa += av;
                    sw += (uint32_t)(y >> 24) & 0x3FFu;
                    maxA = max(maxA, av);
                    agemax = max(agemax, (uint32_t)y & RANKMAX);
                });
                // (sums of at most 2048 workgroups of 512 lanes fit 32 bits)
                totA = wave_sum_dpp(sa);
                totW = wave_sum_dpp(sw);
                maxA = wave_max_dpp(maxA);
                agemax = wave_max_dpp(agemax);
            }
            if (lane == 0) {
                sh_res[0] = totA;
                sh_res[1] = totW;
                sh_res[2] = maxA;
                sh_res[3] = ok ? 0u : 1u;
                sh_res[4] = agemax;
            }
        }
        __syncthreads();
        if (sh_res[3]) {
            failed = true;
            break;
        }
        g_act = sh_res[0];
        g_won = sh_res[1];
        g_maxa = (uint32_t)sh_res[2];
        g_age = (uint32_t)sh_res[4];
        maxact = max(maxact, g_act);
        if (cursor == 0 && g_act == 0)
            break;
        if (rr > p.max_rounds) {
            if (t == 0)
                st(p.err, 2u);
            failed = true;
            break;
        }
    }

    // ---- statistics
    const uint64_t s_att = wave_sum64(attempts), s_ret = wave_sum64(retries),
                   s_self = wave_sum64(selfl);
    if (lane == 0) {
        __hip_atomic_fetch_add(&p.dstats[S_ATTEMPTS], s_att, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&p.dstats[S_RETRIES], s_ret, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&p.dstats[S_SELF], s_self, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    if (t == 0) {
        if (w == 0) {
            st(&p.dstats[S_ROUNDS], rr > 0 ? rr - 1 : 0);
            st(&p.dstats[S_MAXACT], maxact);
            st(&p.dstats[S_THROTTLED], throttled);
            // The quota aims at k active swaps; a round may hold a few more
            // (the winners of the round being refilled are not known yet),
            // so the register-held state is counted from the largest round.
            constexpr uint64_t per_swap = 8 + (EB == 0 ? 0 : 2 * EB);
            st(&p.dstats[S_INFLIGHT], (std::max<uint64_t>(maxact, p.k) * per_swap + 7) / 8);
        }
        if (failed)
            st(&p.dstats[S_STATUS], (uint64_t)(int64_t)RP_ETIMEOUT);
    }
    return epoch;
}

template <int EB, bool EARLY>
__global__ __launch_bounds__(WG1) void rp_rounds1_kernel(Params p)
{
    (void)rounds1_body<EB, EARLY>(p, blockIdx.x - p.wg_first, 0u);
}

// ------------------------------------------------------ the resident kernel
//
// A kernel that stays on the device while a server has work, and takes each
// request from the server's ring (rp_resident.h) as it arrives: a request
// starts as soon as a workgroup is free, at that workgroup's next request
// boundary, instead of at the next launch.  Every workgroup loops: claim the
// next entry in ring order, run it, report it, claim again.
//   * A request planned for one workgroup runs the workgroup rounds of the
//     batched form (rp_wg.h), its round state in the workgroup's LDS.
//   * A request planned for a gang of G workgroups runs the one-barrier
//     rounds above on G workgroups, its tables in device memory the server
//     allocated with it.  The workgroup that claims it (the leader) opens the
//     gang, idle workgroups join it before they claim anything else, and all
//     start once G have joined: every member is then running, so its flag
//     barriers complete.  One gang forms at a time.  A leader whose gang has
//     not formed within form_ticks closes it and reports the request as not
//     run, and the server posts it again.
//   * One workgroup at a time reads the host ring for new entries and
//     publishes what it finds (and the host's stop word) in device memory;
//     the other idle workgroups poll only device memory.
//   * The kernel ends when the host sets the stop word (every workgroup
//     finishes its request first), or by itself after idle_ticks with
//     nothing to claim.
constexpr uint32_t RES_WG = WG1;          // the one-barrier body's workgroup
using ResShape = rpwg::Shape<RES_WG>;
constexpr uint32_t RES_MASK = rpres::RING - 1;
constexpr int RES_IDLE_SLEEP = 32;        // idle poll interval, in units of 64 clocks

struct ResCtl {
    uint64_t head;          // next entry to claim
    uint64_t avail;         // entries below this are known to be posted
    uint64_t gang;          // forming gang: (entry + 1) << 24 | need << 12 | joined;
                            // joined = 0 while its leader is still claiming it
    uint32_t poll_owner;    // 1 while a workgroup reads the host ring
    uint32_t gang_left;     // members of the full gang that have seen it full
    uint32_t exitf;         // 1: claim nothing more and leave
    uint32_t pad[9];
    uint32_t need[rpres::RING];             // workgroups each posted entry needs
    uint64_t stats[rpres::RING][S_WORDS];   // a gang's statistics, per ring slot
};

struct ResParams {
    const rpres::Entry *ring;
    rpres::Result *res;
    const uint32_t *stop;
    ResCtl *ctl;
    uint64_t idle_ticks;
    uint64_t form_ticks;
};

enum : uint32_t { RCMD_EXIT = 0, RCMD_SINGLE = 1, RCMD_LEAD = 2, RCMD_JOIN = 3 };

template <typename T>
__device__ __forceinline__ T ld_sys(const T *p)
{
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename T>
__device__ __forceinline__ void st_sys(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename T>
__device__ __forceinline__ bool cas_agent(T *p, T expect, T v)
{
    return __hip_atomic_compare_exchange_strong(p, &expect, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T xchg_agent(T *p, T v, int order = __ATOMIC_RELAXED)
{
    return order == __ATOMIC_RELEASE
               ? __hip_atomic_exchange(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT)
               : __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t now_ticks()
{
    return __builtin_amdgcn_s_memrealtime();
}

__device__ __forceinline__ uint32_t rfl(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t rfl64(uint64_t v)
{
    return ((uint64_t)rfl((uint32_t)(v >> 32)) << 32) | rfl((uint32_t)v);
}

// Thread 0: what this workgroup does next.  A forming gang takes idle
// workgroups first; then the next posted entry is claimed; with nothing
// posted that is known, one workgroup at a time reads the host ring.
__device__ __forceinline__ uint32_t res_next(const ResParams &P, uint64_t *entry, uint32_t *rank)
{
    ResCtl *c = P.ctl;
    uint64_t t_last = now_ticks();
    for (;;) {
        const uint64_t W = ld(&c->gang);
        if (W != 0) {
            const uint32_t joined = (uint32_t)W & 0xFFFu;
            const uint32_t need = (uint32_t)(W >> 12) & 0xFFFu;
            if (joined != 0 && joined < need) {
                if (cas_agent(&c->gang, W, W + 1)) {
                    *entry = (W >> 24) - 1;
                    *rank = joined;
                    return RCMD_JOIN;
                }
                continue;
            }
            // locked by its leader or full: either lasts microseconds
            if (now_ticks() - t_last > P.idle_ticks) {
                (void)xchg_agent(&c->exitf, 1u);
                return RCMD_EXIT;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        if (ld(&c->exitf) != 0u)
            return RCMD_EXIT;
        const uint64_t h = ld(&c->head);
        const uint64_t a = __hip_atomic_load(&c->avail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (h < a) {
            const uint32_t nd = ld(&c->need[h & RES_MASK]);
            if (nd <= 1u) {
                if (cas_agent(&c->head, h, h + 1)) {
                    *entry = h;
                    *rank = 0;
                    return RCMD_SINGLE;
                }
                continue;
            }
            // A gang entry is claimed with the gang word locked for it, so
            // no workgroup joins before its leader owns the entry.
            const uint64_t Wl = ((h + 1) << 24) | ((uint64_t)nd << 12);
            if (cas_agent(&c->gang, (uint64_t)0, Wl)) {
                if (cas_agent(&c->head, h, h + 1)) {
                    *entry = h;
                    *rank = 0;
                    return RCMD_LEAD;
                }
                (void)xchg_agent(&c->gang, (uint64_t)0);  // h was stale; nobody joined
            }
            continue;
        }
        if (ld(&c->poll_owner) == 0u && xchg_agent(&c->poll_owner, 1u) == 0u) {
            uint64_t aa = a;
            while (aa - h < rpres::RING) {
                const rpres::Entry *e = &P.ring[aa & RES_MASK];
                if (__hip_atomic_load(const_cast<uint64_t *>(&e->seq), __ATOMIC_ACQUIRE,
                                      __HIP_MEMORY_SCOPE_SYSTEM) != aa + 1)
                    break;
                st(&c->need[aa & RES_MASK], ld_sys(&e->gang));
                aa++;
            }
            if (aa > a)
                (void)__hip_atomic_fetch_max(&c->avail, aa, __ATOMIC_RELEASE,
                                             __HIP_MEMORY_SCOPE_AGENT);
            const bool stop = ld_sys(P.stop) != 0u;
            if (stop)
                (void)xchg_agent(&c->exitf, 1u);
            (void)xchg_agent(&c->poll_owner, 0u, __ATOMIC_RELEASE);
            if (aa > a) {
                t_last = now_ticks();
                continue;
            }
            if (stop)
                return RCMD_EXIT;
        }
        if (now_ticks() - t_last > P.idle_ticks) {
            (void)xchg_agent(&c->exitf, 1u);
            return RCMD_EXIT;
        }
        __builtin_amdgcn_s_sleep(RES_IDLE_SLEEP);
    }
}

// Thread 0 of a gang member: wait until the gang of entry `e` has all `need`
// members.  The last member to see it full clears the gang word for the next
// gang.  The leader closes a gang that has not formed within form_ticks;
// then every member returns false.
__device__ __forceinline__ bool res_gang_wait(const ResParams &P, uint64_t e, uint32_t need,
                                              bool leader)
{
    ResCtl *c = P.ctl;
    const uint64_t id = ((e + 1) << 12) | need;
    const uint64_t t0 = now_ticks();
    for (;;) {
        const uint64_t W = ld(&c->gang);
        if ((W >> 12) != id)
            return false;   // closed before it filled
        if ((uint32_t)(W & 0xFFFu) == need) {
            if (__hip_atomic_fetch_add(&c->gang_left, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT) + 1u == need) {
                (void)xchg_agent(&c->gang_left, 0u);
                (void)xchg_agent(&c->gang, (uint64_t)0, __ATOMIC_RELEASE);
            }
            return true;
        }
        if (leader && now_ticks() - t0 > P.form_ticks && cas_agent(&c->gang, W, (uint64_t)0))
            return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

// Thread 0: report a ring slot's result; the records (and the result) are
// made visible beyond the device before the completion word.
__device__ __forceinline__ void res_publish(rpres::Result *out, uint64_t seq, uint64_t rounds,
                                            uint64_t attempts, int32_t status)
{
    st_sys(&out->rounds, rounds);
    st_sys(&out->attempts, attempts);
    st_sys(&out->status, status);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    st_sys(&out->done, seq);
}

// Records [first, n) stepping by `step`: A[r] = r (word 0 of a wider record,
// the other words 0), or a copy of src.  Coherent: device-scope stores, for
// a gang whose members on other compute units read the records next.  The
// source is read with system-scope loads: the kernel outlives the writes
// that produced it, so its caches may hold older copies of those lines.
template <bool COHERENT>
__device__ void res_fill(unsigned char *A, const void *src, uint32_t n, uint32_t eb,
                         uint32_t fill, uint64_t first, uint64_t step)
{
    if (fill == rpres::FILL_NONE)
        return;
    const bool copy = fill == rpres::FILL_COPY;
    for (uint64_t r = first; r < n; r += step) {
        if ((eb & 7u) == 0) {
            uint64_t *d = reinterpret_cast<uint64_t *>(A + r * eb);
            const uint64_t *s = reinterpret_cast<const uint64_t *>(
                static_cast<const unsigned char *>(src) + r * eb);
            for (uint32_t w = 0; w < eb / 8; w++) {
                const uint64_t v = copy ? ld_sys(s + w) : (w == 0 ? r : 0ull);
                if (COHERENT) st(d + w, v); else rpwg::as_global(d)[w] = v;
            }
        } else {
            uint32_t *d = reinterpret_cast<uint32_t *>(A + r * eb);
            const uint32_t *s = reinterpret_cast<const uint32_t *>(
                static_cast<const unsigned char *>(src) + r * eb);
            for (uint32_t w = 0; w < eb / 4; w++) {
                const uint32_t v = copy ? ld_sys(s + w) : (w == 0 ? (uint32_t)r : 0u);
                if (COHERENT) st(d + w, v); else rpwg::as_global(d)[w] = v;
            }
        }
    }
}

// (Flattened: calls would pass the request through scratch memory.)
__global__ __launch_bounds__(RES_WG) __attribute__((flatten)) void
rp_resident_kernel(ResParams P)
{
    __shared__ uint32_t lds[ResShape::LDS_WORDS];
    __shared__ uint32_t sh_scan[ResShape::WAVES];
    __shared__ uint64_t sh_red[ResShape::WAVES];
    __shared__ uint64_t sh_res[6];
    __shared__ uint64_t sh_e[sizeof(rpres::Entry) / 8];
    __shared__ uint64_t sh_idx;
    __shared__ uint32_t sh_cmd, sh_rank, sh_go;

    const uint32_t t = threadIdx.x;
    // Every value that steers these loops is made wave-uniform, and each
    // single-lane step is closed by a workgroup barrier before the loop's
    // back edge.
    for (;;) {
        if (t == 0) {
            uint64_t idx = 0;
            uint32_t rank = 0;
            const uint32_t cmd = res_next(P, &idx, &rank);
            if (cmd != RCMD_EXIT) {
                const uint64_t *q = reinterpret_cast<const uint64_t *>(&P.ring[idx & RES_MASK]);
                for (uint32_t i = 0; i < sizeof(rpres::Entry) / 8; i++)
                    sh_e[i] = ld_sys(q + i);
            }
            sh_cmd = cmd;
            sh_idx = idx;
            sh_rank = rank;
        }
        __syncthreads();
        const uint32_t cmd = rfl(sh_cmd);
        if (cmd == RCMD_EXIT)
            break;
        const uint64_t idx = rfl64(sh_idx);
        const uint32_t rank = rfl(sh_rank);
        const rpres::Entry &le = *reinterpret_cast<const rpres::Entry *>(sh_e);
        unsigned char *const A = reinterpret_cast<unsigned char *>(rfl64((uint64_t)le.A));
        unsigned char *const aux = reinterpret_cast<unsigned char *>(rfl64((uint64_t)le.aux));
        const void *const src = reinterpret_cast<const void *>(rfl64((uint64_t)le.src));
        const uint64_t seed = rfl64(le.seed), max_rounds = rfl64(le.max_rounds);
        const uint32_t n = rfl(le.n), eb = rfl(le.eb), k = rfl(le.k), T = rfl(le.T),
                       bmw = rfl(le.bmw), G = rfl(le.gang), cl = rfl(le.chunk_log2),
                       rank_cap = rfl(le.rank_cap), fill = rfl(le.fill);
        const uint64_t seq = idx + 1;
        rpres::Result *const out = &P.res[idx & RES_MASK];
        __syncthreads();

        if (cmd == RCMD_SINGLE) {
            if (t == 0)
                st_sys(&out->started, seq);
            res_fill<false>(A, src, n, eb, fill, t, RES_WG);
            __syncthreads();
            const rpwg::BatchReq r{A, nullptr, seed, n, eb, k, T, bmw, 1u,
                                   (uint32_t)(idx & RES_MASK), 0u};
            rpwg::WGGroup<RES_WG> wg;
            wg.lds = lds;
            wg.sh_scan = sh_scan;
            uint64_t rounds = 0, attempts = 0;
            uint32_t status = 0;
            if (n > 1) {
                if (eb == 4)
                    rpwg::run_request<4>(wg, r, max_rounds, false, &rounds, &attempts, &status);
                else if (eb == 8)
                    rpwg::run_request<8>(wg, r, max_rounds, false, &rounds, &attempts, &status);
                else
                    rpwg::run_request<0>(wg, r, max_rounds, false, &rounds, &attempts, &status);
            }
            attempts = rpwg::sum_over_group_wg<ResShape::WAVES>(attempts, sh_red);
            rounds = rpwg::sum_over_group_wg<ResShape::WAVES>(
                T == 0 ? rounds : (t == 0 ? rounds : 0), sh_red);
            if (t == 0)
                res_publish(out, seq, rounds, attempts, status ? -(int32_t)status : RP_OK);
            __syncthreads();
            continue;
        }

        // ---- a gang of G workgroups; this one is member `rank`
        Params p{};
        p.A = A;
        p.H = nullptr;
        p.seed = seed;
        p.n = n;
        p.eb = eb;
        p.k = k;
        p.T = T;
        p.bmw = bmw;
        p.choices = 1;
        p.variant = RP_VARIANT_FINAL;
        p.lds_tab = 0;
        p.R64 = nullptr;
        p.max_rounds = max_rounds;
        p.rank_cap = rank_cap;
        p.wg_first = 0;
        p.wg_count = G;
        p.chunk_log2 = cl;
        // the layout of aux_bytes_for1: slots, three window parities, the
        // gather flags, the error word
        unsigned char *cur = aux;
        p.slots = reinterpret_cast<uint32_t *>(cur);
        cur += ((uint64_t)T * 4 + 7) / 8 * 8;
        p.bm = reinterpret_cast<uint32_t *>(cur);
        cur += ((uint64_t)WPAR1 * bmw * 4 + 7) / 8 * 8;
        p.flags = reinterpret_cast<uint64_t *>(cur);
        cur += 2ull * G * 8;
        p.err = reinterpret_cast<uint32_t *>(cur);
        p.dstats = P.ctl->stats[idx & RES_MASK];
        if (cmd == RCMD_LEAD) {
            // Before anyone joins: the words the first barrier and the
            // statistics start from.
            if (t == 0)
                st_sys(&out->started, seq);
            for (uint32_t i = t; i < 2 * G; i += RES_WG)
                st(&p.flags[i], (uint64_t)0);
            if (t == 0)
                st(p.err, 0u);
            if (t < S_WORDS)
                (void)xchg_agent(&p.dstats[t], (uint64_t)0);
            wait_mem();
            __syncthreads();
            if (t == 0)
                (void)xchg_agent(&P.ctl->gang, ((idx + 1) << 24) | ((uint64_t)G << 12) | 1u,
                                 __ATOMIC_RELEASE);
        }
        if (t == 0)
            sh_go = res_gang_wait(P, idx, G, cmd == RCMD_LEAD) ? 1u : 0u;
        __syncthreads();
        if (rfl(sh_go) == 0u) {
            if (cmd == RCMD_LEAD && t == 0)
                res_publish(out, seq, 0, 0, RP_PENDING);
            __syncthreads();
            continue;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // This member's share of the input and of the tables, then a
        // barrier before the first round.
        res_fill<true>(A, src, n, eb, fill, (uint64_t)rank * RES_WG + t, (uint64_t)G * RES_WG);
        for (uint32_t i = rank + G * t; i < T; i += G * RES_WG)
            clear_rmw(&p.slots[i]);
        for (uint32_t i = rank + G * t; i < WPAR1 * bmw; i += G * RES_WG)
            clear_rmw(&p.bm[i]);
        // The records are read after the decision: with about 220 active swaps
        // per workgroup and one workgroup per compute unit, reading every
        // swap's records early cost more than it saved (2^26 int64 on 64
        // workgroups: 78.5 against 72.5 ms).
        bool ok = plain_barrier(p, rank, 1u, sh_res);
        if (ok) {
            uint32_t epoch;
            switch (eb) {
            case 4: epoch = rounds1_body<4, false>(p, rank, 1u); break;
            case 8: epoch = rounds1_body<8, false>(p, rank, 1u); break;
            case 16: epoch = rounds1_body<16, false>(p, rank, 1u); break;
            case 64: epoch = rounds1_body<64, false>(p, rank, 1u); break;
            default: epoch = rounds1_body<0, false>(p, rank, 1u); break;
            }
            // every member's statistics are in before the leader reads them
            ok = plain_barrier(p, rank, epoch + 1, sh_res);
        }
        if (rank == 0 && t == 0) {
            int32_t status = (int32_t)(int64_t)ld(&p.dstats[S_STATUS]);
            if (!ok || ld(p.err) != 0u)
                status = RP_ETIMEOUT;
            res_publish(out, seq, ld(&p.dstats[S_ROUNDS]), ld(&p.dstats[S_ATTEMPTS]), status);
        }
        __syncthreads();
    }
}

__global__ void rp_res_init_kernel(ResCtl *c, uint64_t first)
{
    // These words are later updated by read-modify-write atomics: reset them
    // with atomics too.
    if (threadIdx.x == 0) {
        (void)xchg_agent(&c->head, first);
        (void)xchg_agent(&c->avail, first);
        (void)xchg_agent(&c->gang, (uint64_t)0);
        (void)xchg_agent(&c->poll_owner, 0u);
        (void)xchg_agent(&c->gang_left, 0u);
        (void)xchg_agent(&c->exitf, 0u);
    }
}

// Several independent shuffles in one cooperative launch: shuffle i runs on
// workgroups [g[i].wg_first, g[i].wg_first + g[i].wg_count) with its own
// auxiliary words, its rounds synchronised among those workgroups only.
constexpr uint32_t GROUP_MAX = 16;
struct GroupParams {
    uint32_t count;
    uint32_t pad;
    Params g[GROUP_MAX];
};

template <int M, int EB>
__global__ __launch_bounds__(WG) void rp_rounds_group_kernel(GroupParams gp)
{
    uint32_t i = 0;
    while (i + 1 < gp.count && blockIdx.x >= gp.g[i].wg_first + gp.g[i].wg_count)
        i++;
    rounds_body<M, EB, false>(gp.g[i]);
}

// k = 1: a single active swap per round always commits, so the rounds are the
// sequential loop itself; used when the auxiliary bound cannot hold a table.
__global__ void rp_single_kernel(Params p)
{
    if (blockIdx.x != 0 || threadIdx.x != 0)
        return;
    uint64_t rounds = 0, selfl = 0;
    for (uint32_t i = p.n; i-- > 0;) {
        const uint32_t h = target_of(p, i);
        if (h == i) {
            selfl++;
            continue;
        }
        swap_generic(p.A, p.eb, i, h);
        rounds++;
    }
    st(&p.dstats[S_ROUNDS], rounds);
    st(&p.dstats[S_ATTEMPTS], rounds);
    st(&p.dstats[S_MAXACT], (uint64_t)(rounds ? 1 : 0));
    st(&p.dstats[S_SELF], selfl);
}

// Zero the auxiliary words and write the host-computed statistics.
__global__ void rp_init_kernel(uint32_t *aux, uint64_t words32, uint64_t *dstats,
                               rp_stats host)
{
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = i0; i < words32; i += (uint64_t)gridDim.x * blockDim.x)
        aux[i] = 0u;
    if (i0 == 0 && dstats != nullptr) {
        dstats[S_K] = host.k;
        dstats[S_AUX] = host.aux_words;
        dstats[S_BOUND] = host.aux_bound_words;
        dstats[S_ROUNDS] = 0;
        dstats[S_ATTEMPTS] = 0;
        dstats[S_RETRIES] = 0;
        dstats[S_MAXACT] = 0;
        dstats[S_SELF] = 0;
        dstats[S_GRID] = host.grid;
        dstats[S_SLOTS] = host.slots_per_lane;
        dstats[S_TABLE] = host.table_slots;
        dstats[S_STATUS] = 0;
        dstats[S_INFLIGHT] = host.inflight_words;
        dstats[S_THROTTLED] = 0;
    }
}

// H validation: err <- 1 if some H[i] > i.  Read-only on H and A.
__global__ void rp_check_targets_kernel(const uint64_t *H, uint64_t n, uint32_t *err)
{
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    for (uint64_t i = i0; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        bad = bad || (H[i] > i);
    if (bad)
        st(err, 1u);
}

__global__ void rp_seed_targets_kernel(const uint64_t *idx, uint64_t count,
                                       uint64_t seed, uint64_t *out)
{
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = i0; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = umod64(splitmix64(seed ^ idx[i]), idx[i] + 1);
}

// ------------------------------------------------------------- host planning

struct Plan {
    bool single;      // k = 1 path
    bool lds;         // one workgroup: slots and window in dynamic LDS
    bool onebar;      // one barrier per round (rp_rounds1_kernel, WG1 lanes)
    uint32_t chunk_log2;  // its chunks of fresh indices
    uint32_t G, M, k, T, bmw;
    uint32_t wpar;    // window parities: 2, or 3 with one barrier per round
    uint64_t bound, aux_bytes;
    int eb_class;     // 4, 8, 16 or 0
    int eb1;          // record size the one-barrier kernel holds: 4, 8, 16, 64 or 0
};

double table_ratio()
{
    const char *v = getenv("RP_TABLE_RATIO");
    const double r = (v && *v) ? atof(v) : TABLE_RATIO;
    return (r > 0.05 && r < 64.0) ? r : TABLE_RATIO;
}

// Device bytes the rounds path allocates for k active swaps on G workgroups,
// with `ratio` reservation slots per active swap.
// Entries per parity of the naive variant's table of H: a power of two, at
// least twice the active swaps.
uint64_t naive_cap(uint64_t k)
{
    uint64_t c = 2;
    while (c < 2 * k)
        c <<= 1;
    return c;
}

// Bytes of the array of H the flat and naive variants add for k active swaps.
uint64_t h_table_bytes(uint64_t k, int variant)
{
    if (variant == RP_VARIANT_FLAT)
        return (k * 4 + 7) / 8 * 8;
    if (variant == RP_VARIANT_NAIVE)
        return 2 * naive_cap(k) * 8;
    return 0;
}

uint64_t aux_bytes_for(uint64_t k, uint64_t G, uint64_t *T_out, uint64_t *bmw_out,
                       double ratio = table_ratio(), int variant = RP_VARIANT_FINAL)
{
    const uint64_t T = std::max<uint64_t>(2, (uint64_t)std::ceil(ratio * (double)k));
    const uint64_t bmw = std::max<uint64_t>(1, (2 * k + 31) / 32);
    if (T_out) *T_out = T;
    if (bmw_out) *bmw_out = bmw;
    uint64_t bytes = ((T * 4 + 7) / 8) * 8     // reservation array (padded)
                   + 2 * bmw * 4               // dense window (two parities)
                   + h_table_bytes(k, variant) // flat / naive: H of the active swaps
                   + 8;                        // error word (padded)
    if (G > 1)
        bytes += 2 * G * 8;                    // gather flags (two parities)
    return bytes;
}

int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

// The linear variant: exact n-word array, as many active swaps as the grid
// holds (up to n), no hashed slots or dense window.
int choose_linear_plan(uint64_t n, uint32_t eb, double eps, int cus, int occ_by_m[4],
                       Plan *pl)
{
    std::memset(pl, 0, sizeof(*pl));
    pl->bound = rp_aux_bound_words(n, eps);
    pl->eb_class = (eb == 4 || eb == 8 || eb == 16) ? (int)eb : 0;
    const int slot_opts[4] = {1, 2, 4, 8};
    int mi = 0;
    while (mi < 3 && n > (uint64_t)cus * occ_by_m[mi] * WG * slot_opts[mi])
        mi++;
    const uint64_t M = slot_opts[mi];
    const uint64_t gmax = std::min<uint64_t>(MAXG, (uint64_t)cus * occ_by_m[mi]);
    const uint64_t G = std::max<uint64_t>(1, std::min<uint64_t>(gmax, (n + WG * M - 1) / (WG * M)));
    pl->G = (uint32_t)G;
    pl->M = (uint32_t)M;
    pl->k = (uint32_t)std::min<uint64_t>(n, G * WG * M);
    pl->T = 0;
    pl->bmw = 0;
    pl->aux_bytes = n * 8 + (G > 1 ? 2 * G * 8 : 0) + 8;
    return RP_OK;
}

// Device bytes of the one-barrier path for a target of k active swaps on G
// workgroups (0: the default grid for k on `cus` compute units): the slot
// array, three window parities, the gather flags of the grid and the error
// word.
// Tuning overrides of the one-barrier plan (environment; defaults are the
// measured best): RP_WINDOW window keys per active swap, RP_PER_WG active
// swaps per workgroup (fixes the grid at k / RP_PER_WG).
double window_frac1()
{
    const char *v = getenv("RP_WINDOW");
    const double r = (v && *v) ? atof(v) : WFRAC1;
    return (r >= 0.25 && r <= 8.0) ? r : WFRAC1;
}

// The grid for k active swaps on `cus` compute units: PER_WG1 swaps per
// workgroup, unless that leaves most of the chip idle; then the grid widens
// to WIDE_NUM/WIDE_DEN of the compute units (at least MIN_PER_WG1 swaps per
// workgroup).  A round's memory operations are issued lane by lane, so a
// round is shorter when its swaps are spread over more compute units; the
// flag barrier grows with the grid, which is why it is not widened further
// (measured: n = 2^28 int64 at eps 0.5, 107 / 169 / 210 workgroups ->
// 101.6 / 100.0 / 104.9 ms; 2^26 records of 64 B, 54 / 105 / 205 ->
// 114.5 / 81.9 / 69.3 ms).
uint64_t grid1_for(uint64_t k, uint64_t cus)
{
    const int v = env_int("RP_PER_WG", 0);
    if (v >= 16 && v <= WG1 / 2)
        return (k + (uint64_t)v - 1) / (uint64_t)v;
    const uint64_t g_full = (k + PER_WG1 - 1) / PER_WG1;
    const uint64_t g_wide = std::min<uint64_t>((k + MIN_PER_WG1 - 1) / MIN_PER_WG1,
                                               cus * WIDE_NUM / WIDE_DEN);
    return std::max(g_full, g_wide);
}

uint64_t aux_bytes_for1(uint64_t k, uint64_t G, uint64_t cus, uint64_t *T_out,
                        uint64_t *bmw_out, uint64_t *G_out)
{
    if (G == 0)
        G = grid1_for(k, cus);
    const uint64_t T = std::max<uint64_t>(2, (uint64_t)std::ceil(table_ratio() * (double)k));
    const uint64_t bmw = std::max<uint64_t>(1, (uint64_t)std::ceil(window_frac1() * (double)k / 32.0));
    if (T_out) *T_out = T;
    if (bmw_out) *bmw_out = bmw;
    if (G_out) *G_out = G;
    // slot array and window padded to 8 bytes: the gather flags after them
    // are 64-bit words
    return ((T * 4 + 7) / 8) * 8 + ((WPAR1 * bmw * 4 + 7) / 8) * 8 + 8 + (G > 1 ? 2 * G * 8 : 0);
}

// The one-barrier plan, when it applies: the bound (not the grid) limits
// the active swaps, they need at least two workgroups of WG1 lanes and at
// most `wg_cap` of them, and no other launch shape was asked for.
bool choose_plan1(uint64_t n, uint32_t eb, uint64_t budget, uint64_t cus, uint64_t wg_cap,
                  Plan *pl)
{
    if (env_int("RP_ONEBAR", 1) == 0)
        return false;
    const int want_m = env_int("RP_SLOTS", 0), want_g = env_int("RP_GRID", 0);
    if (want_m > 1)
        return false;
    // A fixed grid (RP_GRID) is counted with its own gather flags.
    const uint64_t G_fixed = want_g > 0 ? (uint64_t)want_g : 0;
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) / 2;
        if (aux_bytes_for1(mid, G_fixed, cus, nullptr, nullptr, nullptr) <= budget) lo = mid;
        else hi = mid - 1;
    }
    uint64_t T, bmw, G;
    const uint64_t k = lo;
    const uint64_t aux = aux_bytes_for1(k, G_fixed, cus, &T, &bmw, &G);
    // every workgroup must keep room for its quota
    if (G_fixed > 0 && G_fixed * WG1 < 2 * k)
        return false;
    if (G < 2 || G > std::min<uint64_t>(MAXG, wg_cap))
        return false;
    pl->onebar = true;
    pl->chunk_log2 = 0;
    while (pl->chunk_log2 < MAX_CHUNK_LOG2 && (G << (pl->chunk_log2 + 1)) * 16 <= k)
        pl->chunk_log2++;
    pl->wpar = WPAR1;
    pl->k = (uint32_t)k;
    pl->G = (uint32_t)G;
    pl->M = 1;
    pl->T = (uint32_t)T;
    pl->bmw = (uint32_t)bmw;
    pl->aux_bytes = aux;
    pl->eb1 = (eb == 4 || eb == 8 || eb == 16 || eb == 64) ? (int)eb : 0;
    return true;
}

// occ1: workgroups of the one-barrier kernel a compute unit holds, or 0 when
// that path may not be used (group launches, variants).
int choose_plan2(uint64_t n, uint32_t eb, double eps, int cus, int occ_by_m[4], Plan *pl,
                 int variant = RP_VARIANT_FINAL);

// occ1 > 0: the one-barrier kernel may be used; it replaces the two-barrier
// plan unless that is the sequential loop (k = 1) or one workgroup with its
// tables in LDS, whose rounds cost only workgroup barriers (n = 2^28 at
// eps = 0.75: 4.7 s there against 9.0 s for four one-barrier workgroups).
int choose_plan(uint64_t n, uint32_t eb, double eps, int cus, int occ_by_m[4],
                Plan *pl, int occ1 = 0, int variant = RP_VARIANT_FINAL)
{
    const int rc = choose_plan2(n, eb, eps, cus, occ_by_m, pl, variant);
    if (rc != RP_OK || occ1 <= 0 || pl->single || pl->lds)
        return rc;
    Plan p1 = *pl;
    if (choose_plan1(n, eb, pl->bound * 8, (uint64_t)cus, (uint64_t)cus * occ1, &p1))
        *pl = p1;
    return RP_OK;
}

// The two-barrier plan (rounds_body).
int choose_plan2(uint64_t n, uint32_t eb, double eps, int cus, int occ_by_m[4], Plan *pl,
                 int variant)
{
    std::memset(pl, 0, sizeof(*pl));
    pl->bound = rp_aux_bound_words(n, eps);
    pl->eb_class = (eb == 4 || eb == 8 || eb == 16) ? (int)eb : 0;
    pl->wpar = 2;
    const uint64_t budget = pl->bound * 8;
    // The persistent path needs k >= 2.
    if (aux_bytes_for(2, 1, nullptr, nullptr, table_ratio(), variant) > budget) {
        pl->single = true;
        pl->k = 1;
        pl->G = 1;
        pl->M = 1;
        pl->aux_bytes = 8;  // the error word; budget >= 8 since bound >= 1
        return RP_OK;
    }
    // Largest k that fits on G workgroups with `ratio` slots per swap.
    auto kmax_for = [&](uint64_t G, double ratio = table_ratio()) {
        uint64_t lo = 0, hi = (uint64_t)n;  // k never needs to exceed n
        while (lo < hi) {
            const uint64_t mid = (lo + hi + 1) / 2;
            if (aux_bytes_for(mid, G, nullptr, nullptr, ratio, variant) <= budget) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    const int slot_opts[4] = {1, 2, 4, 8};
    const int want_m = env_int("RP_SLOTS", 0);
    const int want_g = env_int("RP_GRID", 0);
    uint64_t k0 = kmax_for(1);
    // Choose M then G: prefer one slot per lane with as many workgroups as
    // the chip holds, more slots per lane only when the grid is full.
    int mi = 0;
    if (want_m) {
        for (mi = 0; mi < 3 && slot_opts[mi] < want_m; mi++) {}
    } else {
        while (mi < 3 && k0 > (uint64_t)cus * occ_by_m[mi] * WG * slot_opts[mi]) mi++;
    }
    const uint64_t M = slot_opts[mi];
    const uint64_t gmax = std::min<uint64_t>(MAXG, (uint64_t)cus * occ_by_m[mi]);
    uint64_t G = want_g ? std::min<uint64_t>(want_g, gmax)
                        : std::min<uint64_t>(gmax, (k0 + WG * M - 1) / (WG * M));
    if (G < 1) G = 1;
    uint64_t k = std::min<uint64_t>(kmax_for(G), G * WG * M);
    while (k < 2 && G > 1) {
        G = std::max<uint64_t>(1, G / 2);
        k = std::min<uint64_t>(kmax_for(G), G * WG * M);
    }
    if (k < 2) {
        pl->single = true;
        pl->k = 1;
        pl->G = pl->M = 1;
        pl->aux_bytes = 8;
        return RP_OK;
    }
    // When the grid rather than the bound caps k, the spare words go to a
    // sparser reservation array: with r slots per swap a swap loses to a
    // collision with probability about 1 - r(1 - e^(-1/r)) (37 % at r = 1,
    // 12 % at r = 4), and every such loss costs another round's atomic and
    // record reads.  The largest r is taken for which k need not shrink by
    // more than a quarter: with k that large the rounds are cheap next to
    // the attempts, and r = 1.5 at 3/4 of k already completes about as many
    // swaps per round as r = 1 at the full k.
    double ratio = table_ratio();
    const char *fixed = getenv("RP_TABLE_RATIO");
    if (!(fixed && *fixed) && k < kmax_for(G)) {
        for (const double r : {SPARE_RATIO_MAX, 3.0, 2.0, 1.5, 1.25}) {
            if (r <= ratio)
                break;
            const uint64_t kr = std::min<uint64_t>(k, kmax_for(G, r));
            if (kr >= 2 && kr * 4 >= k * 3) {
                k = kr;
                ratio = r;
                break;
            }
        }
    }
    uint64_t T, bmw;
    pl->aux_bytes = aux_bytes_for(k, G, &T, &bmw, ratio, variant);
    pl->k = (uint32_t)k;
    pl->G = (uint32_t)G;
    pl->M = (uint32_t)M;
    pl->T = (uint32_t)T;
    pl->bmw = (uint32_t)bmw;
    pl->lds = G == 1 && M == 1 && (T + 2 * bmw) * 4 <= LDS_TAB_BYTES;
    return RP_OK;
}

int validate(void *A, uint64_t n, uint32_t eb, double eps)
{
    if (!(eps > 0.0 && eps < 1.0))
        return RP_EINVAL;
    if (eb == 0 || (eb & 3u) != 0 || eb > 256)
        return RP_EINVAL;
    if (n >= (1ull << 32))
        return RP_EINVAL;
    if (A == nullptr && n > 1)
        return RP_EINVAL;
    if (n > 1 && (reinterpret_cast<uintptr_t>(A) & (record_alignment(eb) - 1u)) != 0)
        return RP_EINVAL;
    return RP_OK;
}

using KernelFn = void (*)(Params);

template <int M>
KernelFn pick_eb(int ebc, bool hx)
{
    if (hx) {
        switch (ebc) {
        case 4: return rp_rounds_kernel<M, 4, false, true>;
        case 8: return rp_rounds_kernel<M, 8, false, true>;
        case 16: return rp_rounds_kernel<M, 16, false, true>;
        default: return rp_rounds_kernel<M, 0, false, true>;
        }
    }
    switch (ebc) {
    case 4: return rp_rounds_kernel<M, 4, false>;
    case 8: return rp_rounds_kernel<M, 8, false>;
    case 16: return rp_rounds_kernel<M, 16, false>;
    default: return rp_rounds_kernel<M, 0, false>;
    }
}

// One workgroup, one slot per lane, tables in LDS.
KernelFn pick_lds_kernel(int ebc, bool hx = false)
{
    if (hx) {
        switch (ebc) {
        case 4: return rp_rounds_kernel<1, 4, true, true>;
        case 8: return rp_rounds_kernel<1, 8, true, true>;
        case 16: return rp_rounds_kernel<1, 16, true, true>;
        default: return rp_rounds_kernel<1, 0, true, true>;
        }
    }
    switch (ebc) {
    case 4: return rp_rounds_kernel<1, 4, true>;
    case 8: return rp_rounds_kernel<1, 8, true>;
    case 16: return rp_rounds_kernel<1, 16, true>;
    default: return rp_rounds_kernel<1, 0, true>;
    }
}

using GroupFn = void (*)(GroupParams);

// Group launches: one slot per lane (a shuffle that needs more fills the
// device by itself and has nothing to share a launch with).
GroupFn pick_group_kernel(int ebc)
{
    switch (ebc) {
    case 4: return rp_rounds_group_kernel<1, 4>;
    case 8: return rp_rounds_group_kernel<1, 8>;
    case 16: return rp_rounds_group_kernel<1, 16>;
    default: return rp_rounds_group_kernel<1, 0>;
    }
}

KernelFn pick_kernel(int M, int ebc, bool hx = false)
{
    switch (M) {
    case 1: return pick_eb<1>(ebc, hx);
    case 2: return pick_eb<2>(ebc, hx);
    case 4: return pick_eb<4>(ebc, hx);
    default: return pick_eb<8>(ebc, hx);
    }
}

struct DevInfo {
    bool ok = false;
    int cus = 256;
    int occ[4][5] = {};  // [M index][eb class index] co-resident WGs per CU
    int occx[4][5] = {}; // the same for the flat and naive variants' kernels
    int occ1[5] = {};    // one-barrier kernel (both record timings), by eb1 index
};

using KernelFn1 = void (*)(Params);

KernelFn1 pick_kernel1(int eb1, bool early)
{
    if (early) {
        switch (eb1) {
        case 4: return rp_rounds1_kernel<4, true>;
        case 8: return rp_rounds1_kernel<8, true>;
        case 16: return rp_rounds1_kernel<16, true>;
        case 64: return rp_rounds1_kernel<64, true>;
        default: return rp_rounds1_kernel<0, true>;
        }
    }
    switch (eb1) {
    case 4: return rp_rounds1_kernel<4, false>;
    case 8: return rp_rounds1_kernel<8, false>;
    case 16: return rp_rounds1_kernel<16, false>;
    case 64: return rp_rounds1_kernel<64, false>;
    default: return rp_rounds1_kernel<0, false>;
    }
}

int eb1_index(int eb1) { return eb1 == 4 ? 0 : eb1 == 8 ? 1 : eb1 == 16 ? 2 : eb1 == 64 ? 3 : 4; }
int eb1_of(uint32_t eb) { return (eb == 4 || eb == 8 || eb == 16 || eb == 64) ? (int)eb : 0; }

std::mutex g_mu;
std::vector<DevInfo> g_dev;

int eb_index(int ebc) { return ebc == 4 ? 0 : ebc == 8 ? 1 : ebc == 16 ? 2 : 3; }

int device_info(int dev, DevInfo *out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_dev.size() <= dev)
        g_dev.resize(dev + 1);
    DevInfo &d = g_dev[dev];
    if (!d.ok) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return RP_EDEVICE;
        d.cus = prop.multiProcessorCount;
        const int ms[4] = {1, 2, 4, 8}, ebs[4] = {4, 8, 16, 0};
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                int occ = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &occ, reinterpret_cast<const void *>(pick_kernel(ms[a], ebs[b])),
                        WG, 0) != hipSuccess)
                    return RP_EDEVICE;
                d.occ[a][b] = std::max(occ, 1);
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &occ, reinterpret_cast<const void *>(pick_kernel(ms[a], ebs[b], true)),
                        WG, 0) != hipSuccess)
                    return RP_EDEVICE;
                d.occx[a][b] = std::max(occ, 1);
            }
        const int eb1s[5] = {4, 8, 16, 64, 0};
        for (int b = 0; b < 5; b++) {
            int occ = 0, occe = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &occ, reinterpret_cast<const void *>(pick_kernel1(eb1s[b], false)), WG1,
                    0) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &occe, reinterpret_cast<const void *>(pick_kernel1(eb1s[b], true)), WG1,
                    0) != hipSuccess)
                return RP_EDEVICE;
            d.occ1[b] = std::min(occ, occe);
        }
        d.ok = true;
    }
    *out = d;
    return RP_OK;
}

// Register-held state of the active swaps: source and target (4 bytes each)
// and, for records moved through registers (4, 8, 16 bytes), both records.
uint64_t inflight_words_for(uint64_t k, int eb_class)
{
    const uint64_t per_swap = 8 + 2 * (uint64_t)eb_class;  // eb_class 0: none held
    return (k * per_swap + 7) / 8;
}

void fill_host_stats(const Plan &pl, rp_stats *s)
{
    std::memset(s, 0, sizeof(*s));
    s->k = pl.k;
    s->inflight_words = inflight_words_for(pl.k, pl.single ? 0 : pl.onebar ? pl.eb1 : pl.eb_class);
    s->aux_words = (pl.aux_bytes + 7) / 8;
    s->aux_bound_words = pl.bound;
    s->grid = pl.G;
    s->slots_per_lane = pl.M;
    s->table_slots = pl.T;
}

}  // namespace

extern "C" {

uint64_t rp_aux_bound_words(uint64_t n, double eps)
{
    if (n == 0 || !(eps > 0.0 && eps < 1.0))
        return 0;
    const long double x = powl((long double)n, 1.0L - (long double)eps);
    long double w = floorl(x);
    // Snap values that are an integer up to rounding (e.g. (2^20)^0.5).
    if (x - w > 1.0L - 1e-12L * std::max<long double>(1.0L, x))
        w += 1.0L;
    if (w < 1.0L)
        w = 1.0L;  // n^(1-eps) >= 1 for n >= 1
    return (uint64_t)w;
}

int rp_plan(uint64_t n, uint32_t elem_bytes, double eps, int device,
            rp_stats *stats_out)
{
    // Sizing only: any non-null, suitably aligned stand-in for A.
    int rc = validate(reinterpret_cast<void *>(uintptr_t{256}), n, elem_bytes, eps);
    if (rc != RP_OK)
        return rc;
    int occ[4];
    int cus = 256, occ1 = 1;
    const int ebc = (elem_bytes == 4 || elem_bytes == 8 || elem_bytes == 16) ? (int)elem_bytes : 0;
    if (device >= 0) {
        DevInfo d;
        rc = device_info(device, &d);
        if (rc != RP_OK)
            return rc;
        cus = d.cus;
        for (int a = 0; a < 4; a++)
            occ[a] = d.occ[a][eb_index(ebc)];
        occ1 = d.occ1[eb1_index(eb1_of(elem_bytes))];
    } else {
        for (int a = 0; a < 4; a++)
            occ[a] = 2;
    }
    Plan pl;
    rc = choose_plan(n, elem_bytes, eps, cus, occ, &pl, occ1);
    if (rc != RP_OK)
        return rc;
    if (stats_out)
        fill_host_stats(pl, stats_out);
    return RP_OK;
}

}  // extern "C"

namespace rpint {

// The workgroups rp_shuffle_group gives a shuffle of these arguments, for
// packing group launches (0 when it would not be part of a group: k = 1, or
// more than one slot per lane).
int group_grid(uint64_t n, uint32_t elem_bytes, double eps, int device, uint64_t *grid)
{
    int rc = validate(reinterpret_cast<void *>(uintptr_t{256}), n, elem_bytes, eps);
    if (rc != RP_OK)
        return rc;
    DevInfo d;
    rc = device_info(device, &d);
    if (rc != RP_OK)
        return rc;
    const int ebc = (elem_bytes == 4 || elem_bytes == 8 || elem_bytes == 16) ? (int)elem_bytes : 0;
    int occ[4];
    for (int a = 0; a < 4; a++)
        occ[a] = d.occ[a][eb_index(ebc)];
    Plan pl;
    rc = choose_plan(n, elem_bytes, eps, d.cus, occ, &pl);
    if (rc != RP_OK)
        return rc;
    *grid = (pl.single || pl.M != 1) ? 0 : pl.G;
    return RP_OK;
}

uint64_t resident_ctl_bytes()
{
    return sizeof(ResCtl);
}

int resident_grid(int device, uint32_t *grid)
{
    DevInfo d;
    const int rc = device_info(device, &d);
    if (rc != RP_OK)
        return rc;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, reinterpret_cast<const void *>(rp_resident_kernel), RES_WG, 0) != hipSuccess ||
        occ < 1)
        return RP_EDEVICE;
    // One workgroup per compute unit: the rest of each unit stays free for
    // the device's other work.
    *grid = (uint32_t)d.cus;
    return RP_OK;
}

int resident_plan(uint64_t n, uint32_t eb, double eps, uint32_t max_gang, int device,
                  bool allow_gang, rpres::Entry *e, uint64_t *aux_bytes)
{
    if (e == nullptr || aux_bytes == nullptr || n == 0 || n >= (1ull << 32) ||
        !(eps > 0.0 && eps < 1.0) || eb == 0 || (eb & 3u) != 0 || eb > 256)
        return RP_EINVAL;
    std::memset(e, 0, sizeof(*e));
    e->n = (uint32_t)n;
    e->eb = eb;
    e->max_rounds = n + 64;
    e->rank_cap = RANKMAX;
    e->gang = 1;
    *aux_bytes = 0;
    const uint64_t gmax = std::min<uint64_t>({(uint64_t)max_gang, rpres::MAX_GANG, MAXG});
    if (allow_gang && gmax >= 2 && n > 1) {
        DevInfo d;
        const int rc = device_info(device, &d);
        if (rc != RP_OK)
            return rc;
        const uint64_t cus = (uint64_t)d.cus;
        const uint64_t budget = rp_aux_bound_words(n, eps) * 8;
        // The largest k whose tables fit the bound on a gang of
        // min(grid1_for(k), gmax) workgroups with room for every workgroup's
        // quota (true up to some k, false beyond it).
        auto gang_for = [&](uint64_t k) { return std::min<uint64_t>(grid1_for(k, cus), gmax); };
        auto fits = [&](uint64_t k) {
            const uint64_t G = gang_for(k);
            return G * WG1 >= 2 * k && aux_bytes_for1(k, G, cus, nullptr, nullptr, nullptr) <= budget;
        };
        uint64_t lo = 0, hi = n;
        while (lo < hi) {
            const uint64_t mid = (lo + hi + 1) / 2;
            if (fits(mid)) lo = mid;
            else hi = mid - 1;
        }
        const uint64_t k = lo, G = gang_for(k);
        if (k >= 2 && G >= 2) {
            uint64_t T, bmw, Gx;
            const uint64_t aux = aux_bytes_for1(k, G, cus, &T, &bmw, &Gx);
            uint32_t cl = 0;
            while (cl < MAX_CHUNK_LOG2 && (G << (cl + 1)) * 16 <= k)
                cl++;
            e->gang = (uint32_t)G;
            e->k = (uint32_t)k;
            e->T = (uint32_t)T;
            e->bmw = (uint32_t)bmw;
            e->chunk_log2 = cl;
            e->aux_words = (uint32_t)((aux + 7) / 8);
            *aux_bytes = aux;
            return RP_OK;
        }
    }
    uint32_t k, T, bmw;
    rpwg::plan_request(n, eps, 1.0, RES_WG, ResShape::LDS_WORDS, &k, &T, &bmw);
    e->k = k;
    e->T = T;
    e->bmw = bmw;
    e->aux_words = (uint32_t)(((uint64_t)(T + 2 * bmw) * 4 + 7) / 8);
    return RP_OK;
}

int resident_launch(const rpres::Launch &L, hipStream_t stream)
{
    if (L.ring == nullptr || L.res == nullptr || L.stop == nullptr || L.ctl == nullptr ||
        L.grid == 0)
        return RP_EINVAL;
    ResCtl *c = static_cast<ResCtl *>(L.ctl);
    hipLaunchKernelGGL(rp_res_init_kernel, dim3(1), dim3(64), 0, stream, c, L.first);
    if (hipGetLastError() != hipSuccess)
        return RP_EDEVICE;
    ResParams P{L.ring, L.res, L.stop, c, L.idle_ticks, L.form_ticks};
    hipLaunchKernelGGL(rp_resident_kernel, dim3(L.grid), dim3(RES_WG), 0, stream, P);
    return hipGetLastError() == hipSuccess ? RP_OK : RP_EDEVICE;
}

}  // namespace rpint

namespace {

// The launch parameters of one shuffle planned as `pl`, with its counted
// words at `base` and its statistics record at `dstats`.  The counted words
// are carved as [slots | bm | flags | err], or for the linear variant
// [R (n words) | flags | err]; the LDS variant holds slots and window in LDS.
void setup_params(Params &p, const Plan &pl, int variant, bool lds_tab, void *A, uint64_t n,
                  uint32_t elem_bytes, const uint64_t *H, uint64_t seed, unsigned char *base,
                  uint64_t *dstats)
{
    p.A = static_cast<unsigned char *>(A);
    p.H = H;
    p.seed = seed;
    p.n = (uint32_t)n;
    p.eb = elem_bytes;
    p.k = pl.k;
    p.T = pl.T;
    p.choices = variant == RP_VARIANT_FINAL
                    ? (uint32_t)std::max(1, std::min(2, env_int("RP_CHOICES", 1)))
                    : 1u;
    p.variant = (uint32_t)variant;
    p.lds_tab = lds_tab ? 1u : 0u;
    p.bmw = pl.bmw;
    p.dstats = dstats;
    // RP_MAX_ROUNDS (environment) lowers the round limit, to exercise the
    // watchdog path: every workgroup leaves at that round and the call
    // reports RP_ETIMEOUT with A holding a permutation of its input.
    const int max_rounds = env_int("RP_MAX_ROUNDS", 0);
    p.max_rounds = max_rounds > 0 ? (uint64_t)max_rounds : n + 64;
    // RP_RANK_CAP (environment) lowers the refill throttle's rank limit so
    // that tests can make it engage at small n; any value >= 1 gives the
    // same permutation.
    const int rank_cap = env_int("RP_RANK_CAP", 0);
    p.rank_cap = (rank_cap > 0 && (uint32_t)rank_cap < RANKMAX) ? (uint32_t)rank_cap : RANKMAX;
    p.wg_first = 0;
    p.wg_count = pl.G;
    p.chunk_log2 = pl.chunk_log2;
    unsigned char *cur = base;
    if (variant == RP_VARIANT_LINEAR) {
        p.R64 = reinterpret_cast<uint64_t *>(cur);
        cur += n * 8;
        if (pl.G > 1) {
            p.flags = reinterpret_cast<uint64_t *>(cur);
            cur += 2ull * pl.G * 8;
        }
    } else if (!pl.single) {
        if (!lds_tab) {
            p.slots = reinterpret_cast<uint32_t *>(cur);
            cur += ((uint64_t)pl.T * 4 + 7) / 8 * 8;
            p.bm = reinterpret_cast<uint32_t *>(cur);
            cur += ((uint64_t)pl.wpar * pl.bmw * 4 + 7) / 8 * 8;
        }
        if (variant == RP_VARIANT_FLAT) {
            p.hflat = reinterpret_cast<uint32_t *>(cur);
            cur += h_table_bytes(pl.k, variant);
        } else if (variant == RP_VARIANT_NAIVE) {
            p.htab = reinterpret_cast<uint64_t *>(cur);
            p.hcap = (uint32_t)naive_cap(pl.k);
            cur += h_table_bytes(pl.k, variant);
        }
        if (pl.G > 1) {
            p.flags = reinterpret_cast<uint64_t *>(cur);
            cur += 2ull * pl.G * 8;
        }
    }
    p.err = reinterpret_cast<uint32_t *>(cur);
}

// What the calling thread's last shuffle call obtained as auxiliary memory,
// recorded where it is obtained (allocation calls and the launch's dynamic
// LDS), independently of the plan's own count.
struct AuxLedger {
    uint64_t device_bytes = 0;
    uint64_t lds_bytes = 0;
};
thread_local AuxLedger g_ledger;

// Every counted device allocation of a shuffle call goes through here.
// RP_FAIL_ALLOC (environment, non-zero) makes it fail, to exercise the
// RP_ENOMEM path without exhausting the device.
hipError_t aux_alloc(void **ptr, uint64_t bytes, hipStream_t stream)
{
    if (env_int("RP_FAIL_ALLOC", 0) != 0)
        return hipErrorOutOfMemory;
    const hipError_t e = hipMallocAsync(ptr, bytes, stream);
    if (e == hipSuccess)
        g_ledger.device_bytes += bytes;
    return e;
}

// The device memory a call works in: obtained per call (hipMallocAsync, freed
// stream-ordered at its end), or a caller-supplied region that is neither
// allocated nor freed here (the no-allocation entry point's static scratch).
struct CallMemory {
    unsigned char *fixed = nullptr;
    uint64_t fixed_bytes = 0;
};

int shuffle_impl(void *A, uint64_t n, uint32_t elem_bytes, const uint64_t *H, uint64_t seed,
                 double eps, int variant, void *stream_, rp_stats *stats,
                 const CallMemory &cm = CallMemory{})
{
    g_ledger = AuxLedger{};
    int rc = validate(A, n, elem_bytes, eps);
    if (rc != RP_OK)
        return rc;
    if (variant < RP_VARIANT_FINAL || variant > RP_VARIANT_NAIVE)
        return RP_EINVAL;
    if (H != nullptr && (reinterpret_cast<uintptr_t>(H) & 7u) != 0)
        return RP_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    if (n <= 1) {
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->aux_bound_words = rp_aux_bound_words(n ? n : 1, eps);
        }
        return RP_OK;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return RP_EDEVICE;
    DevInfo di;
    rc = device_info(dev, &di);
    if (rc != RP_OK)
        return rc;
    const int ebc = (elem_bytes == 4 || elem_bytes == 8 || elem_bytes == 16) ? (int)elem_bytes : 0;
    const bool hx_plan = variant == RP_VARIANT_FLAT || variant == RP_VARIANT_NAIVE;
    int occ[4];
    for (int a = 0; a < 4; a++)
        occ[a] = hx_plan ? di.occx[a][eb_index(ebc)] : di.occ[a][eb_index(ebc)];
    Plan pl;
    const int occ1 = variant == RP_VARIANT_FINAL ? di.occ1[eb1_index(eb1_of(elem_bytes))] : 0;
    rc = variant == RP_VARIANT_LINEAR ? choose_linear_plan(n, elem_bytes, eps, di.cus, occ, &pl)
                                      : choose_plan(n, elem_bytes, eps, di.cus, occ, &pl, occ1,
                                                    variant);
    if (rc != RP_OK)
        return rc;

    // Auxiliary words (counted), and apart from them the statistics record
    // (output, not counted).  The LDS variant holds its slot array and window
    // in LDS instead, so only the rest of the counted words are allocated.
    const bool lds_tab = variant != RP_VARIANT_LINEAR && pl.lds;
    const uint64_t tab_bytes = ((uint64_t)pl.T * 4 + 7) / 8 * 8 + 2ull * pl.bmw * 4;
    const uint64_t aux_bytes = lds_tab ? pl.aux_bytes - tab_bytes : pl.aux_bytes;  // multiple of 8
    void *mem = nullptr, *smem = nullptr;
    if (cm.fixed != nullptr) {
        // [aux words | statistics record], both inside the fixed region.
        const uint64_t aux_span = (aux_bytes + 255) / 256 * 256;
        if (aux_span + S_WORDS * 8 > cm.fixed_bytes)
            return RP_ETOOBIG;
        mem = cm.fixed;
        smem = cm.fixed + aux_span;
        g_ledger.device_bytes += aux_bytes;
    } else {
        if (aux_alloc(&mem, aux_bytes, stream) != hipSuccess) {
            (void)hipGetLastError();
            return RP_ENOMEM;
        }
        if (hipMallocAsync(&smem, S_WORDS * 8, stream) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFreeAsync(mem, stream);
            return RP_ENOMEM;
        }
    }
    auto release = [&]() {
        if (cm.fixed != nullptr)
            return hipSuccess;
        (void)hipFreeAsync(smem, stream);
        return hipFreeAsync(mem, stream);
    };
    unsigned char *base = static_cast<unsigned char *>(mem);
    uint64_t *dstats = static_cast<uint64_t *>(smem);
    rp_stats hs;
    fill_host_stats(pl, &hs);
    const uint32_t init_blocks =
        (uint32_t)std::min<uint64_t>(8192, std::max<uint64_t>(64, aux_bytes / 4 / (256 * 16)));
    rp_init_kernel<<<init_blocks, 256, 0, stream>>>(reinterpret_cast<uint32_t *>(base),
                                                    aux_bytes / 4, dstats, hs);
    if (hipGetLastError() != hipSuccess) {
        (void)release();
        return RP_EDEVICE;
    }

    Params p{};
    setup_params(p, pl, variant, lds_tab, A, n, elem_bytes, H, seed, base, dstats);
    // The gather flags are 64-bit atomics and must be naturally aligned.
    if ((reinterpret_cast<uintptr_t>(p.flags) & 7u) != 0) {
        (void)release();
        return RP_EDEVICE;
    }

    if (H != nullptr) {
        // H mode: reject H[i] > i before anything moves.
        rp_check_targets_kernel<<<1024, 256, 0, stream>>>(H, n, p.err);
        uint32_t herr = 0;
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&herr, p.err, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess) {
            (void)release();
            return RP_EDEVICE;
        }
        if (herr != 0) {
            (void)release();
            return RP_EINVAL;
        }
    }

    if (pl.single) {
        rp_single_kernel<<<1, 64, 0, stream>>>(p);
        if (hipGetLastError() != hipSuccess) {
            (void)release();
            return RP_EDEVICE;
        }
    } else if (pl.onebar) {
        void *args[] = {&p};
        const bool early = early_recs_for(n, elem_bytes) != 0;
        if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(pick_kernel1(pl.eb1, early)),
                                       dim3(pl.G), dim3(WG1), args, 0, stream) != hipSuccess) {
            (void)hipGetLastError();
            (void)release();
            return RP_EDEVICE;
        }
    } else {
        const bool hx = variant == RP_VARIANT_FLAT || variant == RP_VARIANT_NAIVE;
        KernelFn fn = p.lds_tab ? pick_lds_kernel(pl.eb_class, hx)
                                : pick_kernel((int)pl.M, pl.eb_class, hx);
        void *args[] = {&p};
        const size_t lds_bytes = p.lds_tab ? ((size_t)pl.T + 2 * (size_t)pl.bmw) * 4 : 0;
        g_ledger.lds_bytes = lds_bytes;
        if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3(pl.G),
                                       dim3(WG), args, lds_bytes, stream) != hipSuccess) {
            (void)hipGetLastError();
            (void)release();
            return RP_EDEVICE;
        }
    }
    if (stats) {
        if (hipMemcpyAsync(stats, dstats, sizeof(rp_stats), hipMemcpyDeviceToHost,
                           stream) != hipSuccess) {
            (void)release();
            return RP_EDEVICE;
        }
    }
    if (release() != hipSuccess)
        return RP_EDEVICE;
    return RP_OK;
}

}  // namespace

extern "C" {

int rp_shuffle_inplace(void *A, uint64_t n, uint32_t elem_bytes,
                       const uint64_t *H, uint64_t seed, double eps,
                       void *stream, rp_stats *stats)
{
    return shuffle_impl(A, n, elem_bytes, H, seed, eps, RP_VARIANT_FINAL, stream, stats);
}

int rp_shuffle_variant(void *A, uint64_t n, uint32_t elem_bytes,
                       const uint64_t *H, uint64_t seed, double eps, int variant,
                       void *stream, rp_stats *stats)
{
    return shuffle_impl(A, n, elem_bytes, H, seed, eps, variant, stream, stats);
}

}  // extern "C"

namespace {

// Device memory of the no-allocation entry point: one copy of this array per
// device, held until the process ends.  On the host, `scratch` names a
// host-side stand-in, never the device array: its device address is taken
// once per device with hipGetSymbolAddress (with that device current) and
// only that address is handed to kernels.  Every call on a device shares that
// device's copy; it keeps the last call's contents, and rp_init_kernel clears
// the words a call needs before its rounds start.
__device__ __align__(256) unsigned char scratch[RP_NOALLOC_SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[SCRATCH_DEVICES] = {};

// The device address of `scratch` on the current device, looked up (and the
// device's launch parameters queried) on the first call there.
int scratch_of_current_device(unsigned char **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_DEVICES)
        return RP_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        DevInfo di;
        const int rc = device_info(dev, &di);
        if (rc != RP_OK)
            return rc;
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return RP_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return RP_OK;
}

}  // namespace

extern "C" {

int rp_shuffle_inplace_noalloc(void *A, uint64_t n, uint32_t elem_bytes,
                               const uint64_t *H, uint64_t seed, double eps,
                               void *stream, rp_stats *stats)
{
    g_ledger = AuxLedger{};
    int rc = validate(A, n, elem_bytes, eps);
    if (rc != RP_OK)
        return rc;
    if (n <= 1)
        return shuffle_impl(A, n, elem_bytes, H, seed, eps, RP_VARIANT_FINAL, stream, stats);
    unsigned char *base = nullptr;
    rc = scratch_of_current_device(&base);
    if (rc != RP_OK)
        return rc;
    CallMemory cm;
    cm.fixed = base;
    cm.fixed_bytes = RP_NOALLOC_SCRATCH_BYTES;
    return shuffle_impl(A, n, elem_bytes, H, seed, eps, RP_VARIANT_FINAL, stream, stats, cm);
}

uint64_t rp_last_call_aux_bytes(void)
{
    return g_ledger.device_bytes + g_ledger.lds_bytes;
}

int rp_group_capacity(uint32_t elem_bytes, int device, uint64_t *workgroups)
{
    if (workgroups == nullptr || elem_bytes == 0 || (elem_bytes & 3u) != 0 || elem_bytes > 256)
        return RP_EINVAL;
    DevInfo di;
    int rc = device_info(device, &di);
    if (rc != RP_OK)
        return rc;
    const int ebc = (elem_bytes == 4 || elem_bytes == 8 || elem_bytes == 16) ? (int)elem_bytes : 0;
    int gocc = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &gocc, reinterpret_cast<const void *>(pick_group_kernel(ebc)), WG, 0) != hipSuccess)
        return RP_EDEVICE;
    *workgroups = (uint64_t)di.cus * (uint64_t)std::max(gocc, 1);
    return RP_OK;
}

int rp_shuffle_group(const rp_batch_request *reqs, uint32_t count, void *stream_,
                     rp_stats *stats)
{
    g_ledger = AuxLedger{};
    if (count == 0)
        return RP_OK;
    if (reqs == nullptr || count > GROUP_MAX)
        return RP_EINVAL;
    const uint32_t eb = reqs[0].elem_bytes;
    for (uint32_t i = 0; i < count; i++) {
        const rp_batch_request &q = reqs[i];
        if (q.elem_bytes != eb || q.n >= (1ull << 32))
            return RP_EINVAL;
        const int rc = validate(q.A, q.n, q.elem_bytes, q.eps);
        if (rc != RP_OK)
            return rc;
        if (q.H != nullptr && (reinterpret_cast<uintptr_t>(q.H) & 7u) != 0)
            return RP_EINVAL;
    }
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return RP_EDEVICE;
    DevInfo di;
    int rc = device_info(dev, &di);
    if (rc != RP_OK)
        return rc;
    const int ebc = (eb == 4 || eb == 8 || eb == 16) ? (int)eb : 0;
    int occ[4];
    for (int a = 0; a < 4; a++)
        occ[a] = di.occ[a][eb_index(ebc)];
    const GroupFn fn = pick_group_kernel(ebc);
    int gocc = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &gocc, reinterpret_cast<const void *>(fn), WG, 0) != hipSuccess)
        return RP_EDEVICE;
    const uint64_t capacity = (uint64_t)di.cus * (uint64_t)std::max(gocc, 1);

    // Each shuffle is planned exactly as a call of its own would be; the
    // workgroups of all of them must be resident together.
    std::vector<Plan> pl(count);
    std::vector<uint64_t> off(count, 0);
    uint64_t aux_total = 0, wg_total = 0;
    for (uint32_t i = 0; i < count; i++) {
        if (reqs[i].n <= 1)
            continue;
        rc = choose_plan(reqs[i].n, eb, reqs[i].eps, di.cus, occ, &pl[i]);
        if (rc != RP_OK)
            return rc;
        if (!pl[i].single && pl[i].M != 1)
            return RP_EINVAL;
        off[i] = aux_total;
        aux_total += pl[i].aux_bytes;
        if (!pl[i].single)
            wg_total += pl[i].G;
    }
    if (wg_total > capacity)
        return RP_EINVAL;
    if (stats)
        for (uint32_t i = 0; i < count; i++) {
            std::memset(&stats[i], 0, sizeof(rp_stats));
            stats[i].aux_bound_words = rp_aux_bound_words(reqs[i].n ? reqs[i].n : 1, reqs[i].eps);
        }
    if (aux_total == 0)
        return RP_OK;

    void *mem = nullptr, *smem = nullptr;
    if (aux_alloc(&mem, aux_total, stream) != hipSuccess) {
        (void)hipGetLastError();
        return RP_ENOMEM;
    }
    if (hipMallocAsync(&smem, (uint64_t)count * S_WORDS * 8, stream) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFreeAsync(mem, stream);
        return RP_ENOMEM;
    }
    auto release = [&]() {
        (void)hipFreeAsync(smem, stream);
        return hipFreeAsync(mem, stream);
    };
    unsigned char *base = static_cast<unsigned char *>(mem);
    uint64_t *dstats = static_cast<uint64_t *>(smem);
    // Shuffles whose bound holds no table (k = 1) run as the sequential
    // single-lane kernel ahead of the group; the others form the group.
    GroupParams gp{};
    std::vector<Params> singles(count);
    std::vector<uint32_t> slot_of(count, GROUP_MAX);
    std::vector<bool> single(count, false);
    uint32_t first = 0;
    for (uint32_t i = 0; i < count; i++) {
        if (reqs[i].n <= 1)
            continue;
        rp_stats hs;
        fill_host_stats(pl[i], &hs);
        const uint64_t words32 = pl[i].aux_bytes / 4;
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(
            8192, std::max<uint64_t>(64, words32 / (256 * 16)));
        rp_init_kernel<<<blocks, 256, 0, stream>>>(reinterpret_cast<uint32_t *>(base + off[i]),
                                                   words32, dstats + (uint64_t)i * S_WORDS, hs);
        Params &p = pl[i].single ? singles[i] : gp.g[gp.count];
        setup_params(p, pl[i], RP_VARIANT_FINAL, false, reqs[i].A, reqs[i].n, eb, reqs[i].H,
                     reqs[i].seed, base + off[i], dstats + (uint64_t)i * S_WORDS);
        if (pl[i].single) {
            single[i] = true;
            continue;
        }
        p.wg_first = first;
        p.wg_count = pl[i].G;
        first += pl[i].G;
        slot_of[i] = gp.count++;
    }
    if (hipGetLastError() != hipSuccess) {
        (void)release();
        return RP_EDEVICE;
    }
    // Explicit targets: reject the whole group if any H[i] > i, before
    // anything moves.
    auto err_of = [&](uint32_t i) {
        return single[i] ? singles[i].err : gp.g[slot_of[i]].err;
    };
    bool any_h = false;
    for (uint32_t i = 0; i < count; i++)
        if (reqs[i].H != nullptr && reqs[i].n > 1) {
            any_h = true;
            rp_check_targets_kernel<<<1024, 256, 0, stream>>>(reqs[i].H, reqs[i].n, err_of(i));
        }
    if (any_h) {
        uint32_t bad = 0;
        for (uint32_t i = 0; i < count && rc == RP_OK; i++) {
            if (reqs[i].H == nullptr || reqs[i].n <= 1)
                continue;
            uint32_t e = 0;
            if (hipMemcpyAsync(&e, err_of(i), 4, hipMemcpyDeviceToHost, stream) !=
                    hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess)
                rc = RP_EDEVICE;
            bad |= e;
        }
        if (rc == RP_OK && hipGetLastError() != hipSuccess)
            rc = RP_EDEVICE;
        if (rc != RP_OK || bad != 0) {
            (void)release();
            return rc != RP_OK ? rc : RP_EINVAL;
        }
    }
    for (uint32_t i = 0; i < count; i++)
        if (single[i])
            rp_single_kernel<<<1, 64, 0, stream>>>(singles[i]);
    if (hipGetLastError() != hipSuccess) {
        (void)release();
        return RP_EDEVICE;
    }
    void *args[] = {&gp};
    if (gp.count > 0 &&
        hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3((uint32_t)wg_total),
                                   dim3(WG), args, 0, stream) != hipSuccess) {
        (void)hipGetLastError();
        (void)release();
        return RP_EDEVICE;
    }
    if (stats)
        for (uint32_t i = 0; i < count; i++)
            if (reqs[i].n > 1 &&
                hipMemcpyAsync(&stats[i], dstats + (uint64_t)i * S_WORDS, sizeof(rp_stats),
                               hipMemcpyDeviceToHost, stream) != hipSuccess) {
                (void)release();
                return RP_EDEVICE;
            }
    if (release() != hipSuccess)
        return RP_EDEVICE;
    return RP_OK;
}

int rp_seed_targets(const uint64_t *idx, uint64_t count, uint64_t seed,
                    uint64_t *out, void *stream_)
{
    if (count == 0)
        return RP_OK;
    if (idx == nullptr || out == nullptr)
        return RP_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    const uint64_t blocks = std::min<uint64_t>(4096, (count + 255) / 256);
    rp_seed_targets_kernel<<<(unsigned)blocks, 256, 0, stream>>>(idx, count, seed, out);
    return hipGetLastError() == hipSuccess ? RP_OK : RP_EDEVICE;
}

}  // extern "C"

// ------------------------------------------------------ measurement probes
//
// Microbenchmarks of the device costs the rounds are built from: the data
// movement of the shuffle alone (every swap's two reads and two writes at its
// real addresses, with no reservation, so the output is not a permutation), a
// streaming copy, the flag barrier of the rounds kernel, and device-scope
// atomic max into a reservation-sized table.  They give the ceilings the
// shuffle's time is compared with; none is used by the shuffle itself.

namespace {

template <int EB>
__global__ __launch_bounds__(256) void rp_probe_rmw_kernel(unsigned char *A, uint32_t n,
                                                           uint64_t seed)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
        const uint32_t h = seed_target(seed, s);
        if constexpr (EB == 64) {
            uint4 *ps = reinterpret_cast<uint4 *>(A) + 4ull * s;
            uint4 *ph = reinterpret_cast<uint4 *>(A) + 4ull * h;
            uint4 a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                a[u] = ps[u];
                b[u] = ph[u];
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                ps[u] = b[u];
                ph[u] = a[u];
            }
        } else {
            Rec<EB> a, b;
            a.load(A, s);
            b.load(A, h);
            b.store(A, s);
            a.store(A, h);
        }
    }
}

__global__ __launch_bounds__(256) void rp_probe_copy_kernel(uint4 *dst, const uint4 *src,
                                                            uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

// `rounds` flag barriers on the launch's workgroups, each preceded by the
// same wait for memory operations and workgroup barrier as in the rounds.
__global__ __launch_bounds__(WG) void rp_probe_barrier_kernel(Params p, uint32_t rounds)
{
    __shared__ uint64_t sh_res[5];
    for (uint32_t r = 0; r < rounds; r++)
        if (!plain_barrier(p, blockIdx.x, r + 1, sh_res))
            return;
}

// Each lane issues `per_lane` atomic max operations on pseudo-random slots of
// a `T`-slot table: fire-and-forget (the wave waits for all of them at the
// end), or each on the result of the previous one (latency).
__global__ __launch_bounds__(256) void rp_probe_atomic_kernel(uint32_t *tab, uint32_t T,
                                                              uint32_t per_lane,
                                                              uint32_t chained, uint32_t *sink)
{
    const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t x = id * 0x9E3779B9u + 1u, acc = 0;
    for (uint32_t j = 0; j < per_lane; j++) {
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        const uint32_t slot = (uint32_t)(((uint64_t)(x ^ (chained ? acc & 1u : 0u)) * T) >> 32);
        if (chained)
            acc += __hip_atomic_fetch_max(&tab[slot], x, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        else
            __hip_atomic_fetch_max(&tab[slot], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    wait_mem();
    if (acc == 0xFFFFFFFFu)
        st(sink, acc);
}

int probe_time(hipStream_t stream, hipEvent_t a, hipEvent_t b, double *ms)
{
    float f = 0;
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&f, a, b) != hipSuccess)
        return RP_EDEVICE;
    *ms = f;
    (void)stream;
    return RP_OK;
}

}  // namespace

extern "C" {

int rp_probe_random_rmw(void *A, uint64_t n, uint32_t elem_bytes, uint64_t seed, void *stream_)
{
    if (n == 0)
        return RP_OK;
    if (A == nullptr || n >= (1ull << 32) ||
        !(elem_bytes == 4 || elem_bytes == 8 || elem_bytes == 16 || elem_bytes == 64))
        return RP_EINVAL;
    if ((reinterpret_cast<uintptr_t>(A) & (elem_bytes >= 16 ? 15u : elem_bytes - 1u)) != 0)
        return RP_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    int dev = 0;
    DevInfo di;
    if (hipGetDevice(&dev) != hipSuccess || device_info(dev, &di) != RP_OK)
        return RP_EDEVICE;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((uint64_t)di.cus * 8,
                                                         (n + 255) / 256);
    unsigned char *a = static_cast<unsigned char *>(A);
    switch (elem_bytes) {
    case 4: rp_probe_rmw_kernel<4><<<blocks, 256, 0, stream>>>(a, (uint32_t)n, seed); break;
    case 8: rp_probe_rmw_kernel<8><<<blocks, 256, 0, stream>>>(a, (uint32_t)n, seed); break;
    case 16: rp_probe_rmw_kernel<16><<<blocks, 256, 0, stream>>>(a, (uint32_t)n, seed); break;
    default: rp_probe_rmw_kernel<64><<<blocks, 256, 0, stream>>>(a, (uint32_t)n, seed); break;
    }
    return hipGetLastError() == hipSuccess ? RP_OK : RP_EDEVICE;
}

int rp_probe_copy(void *dst, const void *src, uint64_t bytes, void *stream_)
{
    if (bytes == 0)
        return RP_OK;
    if (dst == nullptr || src == nullptr || (bytes & 15u) != 0 ||
        ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u) != 0)
        return RP_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    int dev = 0;
    DevInfo di;
    if (hipGetDevice(&dev) != hipSuccess || device_info(dev, &di) != RP_OK)
        return RP_EDEVICE;
    const uint64_t n16 = bytes / 16;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((uint64_t)di.cus * 16, (n16 + 255) / 256);
    rp_probe_copy_kernel<<<blocks, 256, 0, stream>>>(static_cast<uint4 *>(dst),
                                                     static_cast<const uint4 *>(src), n16);
    return hipGetLastError() == hipSuccess ? RP_OK : RP_EDEVICE;
}

int rp_probe_barrier(uint32_t grid, uint32_t rounds, void *stream_, double *us_per_barrier)
{
    if (grid < 2 || grid > MAXG || rounds == 0 || us_per_barrier == nullptr)
        return RP_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    void *mem = nullptr;
    const uint64_t bytes = 2ull * grid * 8 + 8;
    if (hipMallocAsync(&mem, bytes, stream) != hipSuccess) {
        (void)hipGetLastError();
        return RP_ENOMEM;
    }
    hipEvent_t a = nullptr, b = nullptr;
    int rc = RP_EDEVICE;
    if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
        rp_init_kernel<<<64, 256, 0, stream>>>(static_cast<uint32_t *>(mem), bytes / 4,
                                               nullptr, rp_stats{});
        Params p{};
        p.flags = static_cast<uint64_t *>(mem);
        p.err = reinterpret_cast<uint32_t *>(static_cast<unsigned char *>(mem) + 2ull * grid * 8);
        p.wg_first = 0;
        p.wg_count = grid;
        void *args[] = {&p, &rounds};
        double ms = 0;
        if (hipGetLastError() == hipSuccess && hipEventRecord(a, stream) == hipSuccess &&
            hipLaunchCooperativeKernel(reinterpret_cast<const void *>(rp_probe_barrier_kernel),
                                       dim3(grid), dim3(WG), args, 0, stream) == hipSuccess &&
            hipEventRecord(b, stream) == hipSuccess && probe_time(stream, a, b, &ms) == RP_OK) {
            *us_per_barrier = ms * 1e3 / rounds;
            rc = RP_OK;
        }
        (void)hipGetLastError();
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFreeAsync(mem, stream);
    (void)hipStreamSynchronize(stream);
    return rc;
}

int rp_probe_atomics(uint32_t table_slots, uint32_t grid, uint32_t per_lane, int chained,
                     void *stream_, double *ns_total)
{
    if (table_slots == 0 || grid == 0 || per_lane == 0 || ns_total == nullptr)
        return RP_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    void *mem = nullptr;
    const uint64_t bytes = (uint64_t)table_slots * 4 + 8;
    if (hipMallocAsync(&mem, bytes, stream) != hipSuccess) {
        (void)hipGetLastError();
        return RP_ENOMEM;
    }
    hipEvent_t a = nullptr, b = nullptr;
    int rc = RP_EDEVICE;
    if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
        uint32_t *tab = static_cast<uint32_t *>(mem);
        rp_init_kernel<<<64, 256, 0, stream>>>(tab, bytes / 4, nullptr, rp_stats{});
        double ms = 0;
        if (hipGetLastError() == hipSuccess && hipEventRecord(a, stream) == hipSuccess) {
            rp_probe_atomic_kernel<<<grid, 256, 0, stream>>>(tab, table_slots, per_lane,
                                                             chained ? 1u : 0u,
                                                             tab + table_slots);
            if (hipGetLastError() == hipSuccess && hipEventRecord(b, stream) == hipSuccess &&
                probe_time(stream, a, b, &ms) == RP_OK) {
                *ns_total = ms * 1e6;
                rc = RP_OK;
            }
        }
        (void)hipGetLastError();
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFreeAsync(mem, stream);
    (void)hipStreamSynchronize(stream);
    return rc;
}

}  // extern "C"
