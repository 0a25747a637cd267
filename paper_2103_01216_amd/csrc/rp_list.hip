// List ranking by in-place list contraction (Gu, Obeya, Shun, "Parallel
// In-Place Algorithms: Theory and Practice", Section 4.2).
//
// Contraction: the elements are taken in blocks of k = floor(n^(1-eps)) in
// index order; inside a block, Algorithm 2 (Shun et al.'s parallel list
// contraction) runs in rounds: every element of the block whose key is below
// both current neighbours' keys is spliced out, and the rest stay for the
// next round.  Keys are (block, priority, index); list heads and the NIL ends
// are above every key, and so are the elements of later blocks, so a block
// is contracted completely before the next one starts.  List heads are never
// spliced: they anchor the ranks.
//
// In place: every element's two 64-bit pointer words carry the algorithm's
// state and then its record in the contraction tree (Section 4.2 stores the
// tree over the input's pointers):
//   word 0 (prev):  low 32 = previous element (NIL at a head);
//                   after the splice: low 32 = left neighbour L at the splice,
//                   high 32 = offset, the distance from L to this element
//   word 1 (next):  low 32 = next element (NIL at a tail), high 32 = weight,
//                   the distance to the current next element;
//                   after the splice: low 32 = right neighbour R at the
//                   splice, high 32 = the round of its block it went in.
// A splice of i between L and R links L and R and adds i's weight to L's.
//
// Reconstruction: blocks in reverse, rounds of a block in reverse:
// rank(i) = rank(L) + offset(i), heads at rank 0.
//
// One cooperative persistent kernel; each element of the current block is
// held by a lane (M per lane).  Rounds are separated by grid-wide flag
// barriers that also carry the counts the loop needs.  Auxiliary memory: the
// barrier flags and an error word.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "rp.h"
#include "rp_device.h"

namespace {

using namespace rpdev;

constexpr int LWG = 256;
constexpr int LWAVES = LWG / 64;
constexpr int LM_MAX = 4;                   // block elements per lane, at most
constexpr uint32_t NILI = 0xFFFFFFFFu;
constexpr uint32_t LMAXG = 2048;
constexpr uint32_t LPOLL = 8;               // barrier flags a lane loads at once
constexpr uint64_t LWATCHDOG = 500000000ull;  // 5 s at 100 MHz

struct LParams {
    uint64_t *rec;          // 2 words per element
    uint64_t *rank;         // output, n entries
    const uint64_t *prio;   // nullptr: seed mode
    uint64_t seed;
    uint64_t n;
    uint64_t k;             // block size
    uint64_t *flags;        // 2 * G words
    uint32_t *err;          // 0 ok, 1 watchdog, 2 no progress (malformed)
    uint64_t *out;          // phases, contract rounds, rebuild rounds
};

__device__ __forceinline__ void st64(uint64_t *a, uint64_t v) { st<uint64_t>(a, v); }

__device__ __forceinline__ uint64_t prio_of(const LParams &p, uint32_t i)
{
    return p.prio ? ld(&p.prio[i]) : splitmix64(p.seed ^ (uint64_t)i);
}

// key(a) < key(b) for an element a of the block ending at b1; a current
// neighbour b is NIL, a head, or an element of this block or a later one
// (earlier blocks are gone).
__device__ __forceinline__ bool below(const LParams &p, uint64_t b1, uint32_t a, uint64_t pa,
                                      uint32_t b, bool b_head)
{
    if (b == NILI || b_head || b >= b1)
        return true;
    const uint64_t pb = prio_of(p, b);
    if (pa != pb)
        return pa < pb;
    return a < b;
}

// Grid barrier carrying a 48-bit payload per workgroup (wave 0 only).  Flags
// hold epoch:16 | payload:48, double-buffered by epoch parity, so a
// workgroup cannot reuse a flag before every workgroup has read it.  Every
// workgroup's memory operations are complete (each wave waited for them, then
// a workgroup barrier) before its flag is raised.  Returns the sum of the
// payload fields (two 24-bit counts are summed independently) and false if
// the watchdog fired or another workgroup reported an error; *max_lo is the
// largest low field.
__device__ bool lgather(const LParams &p, uint32_t epoch, uint64_t payload, uint64_t *sum_lo,
                        uint64_t *sum_hi, uint64_t *max_lo)
{
    const uint32_t G = gridDim.x, lane = threadIdx.x & 63;
    const uint32_t e16 = epoch & 0xFFFFu;
    uint64_t *fl = p.flags + (uint64_t)(epoch & 1u) * G;
    if (lane == 0)
        st(&fl[blockIdx.x], ((uint64_t)e16 << 48) | payload);
    uint64_t lo = 0, hi = 0;
    uint32_t mx = 0;
    bool ok = true;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    // The flags of lane l are l, l + 64, ...; every sweep loads all of its
    // pending ones before checking any (one load latency per sweep).
    const uint32_t nj = (G + 63u) / 64u;   // <= 32
    uint32_t pending = 0;
    for (uint32_t j = 0; j < nj; j++)
        pending |= (lane + 64u * j < G) ? (1u << j) : 0u;
    for (uint32_t sweep = 1; pending; sweep++) {
#pragma unroll 1
        for (uint32_t j0 = 0; j0 < nj; j0 += LPOLL) {
            uint64_t f[LPOLL];
#pragma unroll
            for (uint32_t u = 0; u < LPOLL; u++) {
                const uint32_t j = j0 + u;
                f[u] = (j < nj && (pending & (1u << j))) ? ld(&fl[lane + 64u * j]) : 0ull;
            }
#pragma unroll
            for (uint32_t u = 0; u < LPOLL; u++) {
                const uint32_t j = j0 + u;
                if (j < nj && (pending & (1u << j)) && (uint32_t)(f[u] >> 48) == e16) {
                    pending &= ~(1u << j);
                    lo += f[u] & 0xFFFFFFull;
                    hi += (f[u] >> 24) & 0xFFFFFFull;
                    mx = max(mx, (uint32_t)(f[u] & 0xFFFFFFull));
                }
            }
        }
        if (pending && (sweep & 63u) == 0 &&
            (__builtin_amdgcn_s_memrealtime() - t0 > LWATCHDOG || ld(p.err) != 0u)) {
            ok = false;
            break;
        }
        if (pending)
            __builtin_amdgcn_s_sleep(1);
    }
    *sum_lo = wave_sum64(lo);
    *sum_hi = wave_sum64(hi);
    *max_lo = wave_max(mx);
    return __all(ok);
}

// Workgroup-wide: sum (lo, hi) over every lane of the grid -- or, with
// take_max, the maximum of lo -- as wave-uniform values; false on error.
// Every lane passes values below 2^24 / (lanes of the grid) for sums.
__device__ bool grid_sum(const LParams &p, uint32_t *epoch, uint32_t lo, uint32_t hi,
                         uint64_t *tot_lo, uint64_t *tot_hi, uint64_t *sh, bool take_max = false)
{
    __shared__ uint32_t s_lo[LWAVES], s_hi[LWAVES];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t wl = take_max ? wave_max(lo) : wave_sum64(lo), wh = wave_sum64(hi);
    if (lane == 0) {
        s_lo[wave] = (uint32_t)wl;
        s_hi[wave] = (uint32_t)wh;
    }
    wait_mem();
    __syncthreads();
    ++*epoch;
    if (wave == 0) {
        uint64_t a = 0, b = 0;
        for (int i = 0; i < LWAVES; i++) {
            a = take_max ? max(a, (uint64_t)s_lo[i]) : a + s_lo[i];
            b += s_hi[i];
        }
        bool ok = true;
        if (gridDim.x > 1) {
            uint64_t m = 0;
            ok = lgather(p, *epoch, (b << 24) | a, &a, &b, &m);
            if (take_max)
                a = m;
            if (!ok && lane == 0)
                st(p.err, 1u);
        }
        if (lane == 0) {
            sh[0] = a;
            sh[1] = b;
            sh[2] = ok ? 0u : 1u;
        }
    }
    __syncthreads();
    // wave-uniform (scalar) values: every loop decision below depends on them
    const uint64_t a = sh[0], b = sh[1];
    *tot_lo = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) << 32) |
              __builtin_amdgcn_readfirstlane((uint32_t)a);
    *tot_hi = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32)) << 32) |
              __builtin_amdgcn_readfirstlane((uint32_t)b);
    return __builtin_amdgcn_readfirstlane((uint32_t)sh[2]) == 0;
}

// LM: block elements per lane (1, 2 or 4): the fewest that hold a block on
// the grid, so that a small block is spread over as many workgroups as it
// fills.
template <int LM>
__global__ __launch_bounds__(LWG) void rp_list_kernel(LParams p)
{
    __shared__ uint64_t sh[3];
    const uint32_t G = gridDim.x, w = blockIdx.x, t = threadIdx.x;
    const uint64_t nth = (uint64_t)G * LWG;
    uint32_t epoch = 0;
    uint64_t lo, hi;

    // ---- init: weights 1, offsets 0, head ranks 0
    for (uint64_t i = (uint64_t)w * LWG + t; i < p.n; i += nth) {
        const uint64_t pw = ld(&p.rec[2 * i]), nw = ld(&p.rec[2 * i + 1]);
        st64(&p.rec[2 * i], pw & 0xFFFFFFFFull);
        st64(&p.rec[2 * i + 1], (nw & 0xFFFFFFFFull) | (1ull << 32));
        if ((uint32_t)pw == NILI)
            st64(&p.rank[i], 0ull);
    }
    if (!grid_sum(p, &epoch, 0, 0, &lo, &hi, sh))
        return;

    // ---- contraction, block by block
    uint64_t phases = 0, crounds = 0;
    for (uint64_t b0 = 0; b0 < p.n; b0 += p.k) {
        const uint64_t b1 = min(b0 + p.k, p.n);
        uint32_t idx[LM];
        bool alive[LM];
#pragma unroll
        for (int m = 0; m < LM; m++) {
            const uint64_t i = b0 + (uint64_t)m * nth + (uint64_t)w * LWG + t;
            idx[m] = (uint32_t)i;
            alive[m] = i < b1 && (uint32_t)ld(&p.rec[2 * i]) != NILI;
        }
        for (uint32_t r = 0;; r++) {
            uint32_t na = 0;
#pragma unroll
            for (int m = 0; m < LM; m++)
                na += alive[m] ? 1u : 0u;
            // Which of mine are below both neighbours (all reads first: the
            // neighbours' words of this round are only written after the
            // barrier below).
            bool go[LM];
            uint64_t pw[LM], nw[LM];
#pragma unroll
            for (int m = 0; m < LM; m++) {
                go[m] = false;
                if (!alive[m])
                    continue;
                const uint32_t i = idx[m];
                pw[m] = ld(&p.rec[2 * (uint64_t)i]);
                nw[m] = ld(&p.rec[2 * (uint64_t)i + 1]);
                const uint32_t L = (uint32_t)pw[m], R = (uint32_t)nw[m];
                // L is a head iff its own previous pointer is NIL; a
                // successor is never a head.
                const bool l_head = (uint32_t)ld(&p.rec[2 * (uint64_t)L]) == NILI;
                const uint64_t pi = prio_of(p, i);
                go[m] = below(p, b1, i, pi, L, l_head) && below(p, b1, i, pi, R, false);
            }
            uint32_t ns = 0;
#pragma unroll
            for (int m = 0; m < LM; m++)
                ns += go[m] ? 1u : 0u;
            // Everyone has decided before anyone splices.
            if (!grid_sum(p, &epoch, na, ns, &lo, &hi, sh))
                return;
            if (lo == 0)
                break;              // block done (na counted before this round)
            if (hi == 0) {          // alive elements but no local minimum
                if (t == 0 && w == 0)
                    st(p.err, 2u);
                return;
            }
            // Splice: i's left neighbour L and right neighbour R are not
            // spliced this round (their keys are higher), and no other
            // spliced element touches the words written here.
            // (all weight loads first, then the stores: one load latency)
            uint32_t wls[LM];
#pragma unroll
            for (int m = 0; m < LM; m++)
                wls[m] = go[m] ? (uint32_t)(ld(&p.rec[2 * (uint64_t)(uint32_t)pw[m] + 1]) >> 32)
                               : 0u;
#pragma unroll
            for (int m = 0; m < LM; m++) {
                if (!go[m])
                    continue;
                const uint64_t i = idx[m];
                const uint32_t L = (uint32_t)pw[m], R = (uint32_t)nw[m];
                const uint64_t wi = nw[m] >> 32;
                const uint64_t wl = wls[m];
                st64(&p.rec[2 * (uint64_t)L + 1], (uint64_t)R | ((wl + wi) << 32));
                if (R != NILI)
                    st64(&p.rec[2 * (uint64_t)R], (uint64_t)L);
                st64(&p.rec[2 * i], (uint64_t)L | (wl << 32));
                st64(&p.rec[2 * i + 1], (uint64_t)R | ((uint64_t)r << 32));
                alive[m] = false;
            }
            // The splices must be visible before the next round's reads.
            if (!grid_sum(p, &epoch, 0, 0, &lo, &hi, sh))
                return;
            crounds++;
        }
        phases++;
    }

    // ---- reconstruction: blocks in reverse, rounds in reverse
    uint64_t rrounds = 0;
    const uint64_t nblocks = (p.n + p.k - 1) / p.k;
    for (uint64_t bj = nblocks; bj-- > 0;) {
        const uint64_t b0 = bj * p.k, b1 = min(b0 + p.k, p.n);
        uint32_t idx[LM], rr[LM], left[LM], off[LM];
        uint32_t mymax = 0;
#pragma unroll
        for (int m = 0; m < LM; m++) {
            const uint64_t i = b0 + (uint64_t)m * nth + (uint64_t)w * LWG + t;
            idx[m] = (uint32_t)i;
            rr[m] = NILI;
            if (i < b1) {
                const uint64_t pw = ld(&p.rec[2 * i]);
                if ((uint32_t)pw != NILI) {   // heads keep rank 0
                    left[m] = (uint32_t)pw;
                    off[m] = (uint32_t)(pw >> 32);
                    rr[m] = (uint32_t)(ld(&p.rec[2 * i + 1]) >> 32);
                    mymax = max(mymax, rr[m] + 1);
                }
            }
        }
        // rounds of this block = the largest (round + 1) over its elements
        if (!grid_sum(p, &epoch, mymax, 0, &lo, &hi, sh, true))
            return;
        const uint32_t R = (uint32_t)lo;
        for (uint32_t r = R; r-- > 0;) {
            uint64_t lr[LM];
#pragma unroll
            for (int m = 0; m < LM; m++)
                lr[m] = rr[m] == r ? ld(&p.rank[left[m]]) : 0ull;
#pragma unroll
            for (int m = 0; m < LM; m++)
                if (rr[m] == r)
                    st64(&p.rank[idx[m]], lr[m] + off[m]);
            if (!grid_sum(p, &epoch, 0, 0, &lo, &hi, sh))
                return;
            rrounds++;
        }
    }
    if (w == 0 && t == 0) {
        st64(&p.out[0], phases);
        st64(&p.out[1], crounds);
        st64(&p.out[2], rrounds);
    }
}

// Consistency of the links: next[prev[i]] == i and prev[next[i]] == i,
// indices in range.  Sets *bad on the first violation found.
__global__ void rp_list_check_kernel(const uint64_t *rec, uint64_t n, uint32_t *bad)
{
    const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) {
        const uint32_t P = (uint32_t)rec[2 * i], N = (uint32_t)rec[2 * i + 1];
        bool ok = true;
        if (P != NILI)
            ok = P < n && P != i && (uint32_t)rec[2 * (uint64_t)P + 1] == (uint32_t)i;
        if (ok && N != NILI)
            ok = N < n && N != i && (uint32_t)rec[2 * (uint64_t)N] == (uint32_t)i;
        if (!ok)
            __hip_atomic_store(bad, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace

extern "C" {

int rp_list_rank(uint64_t *rec, uint64_t n, const uint64_t *prio, uint64_t seed, double eps,
                 uint64_t *rank, void *stream_, rp_list_stats *stats)
{
    if (!(eps > 0.0 && eps < 1.0) || n >= (1ull << 32) - 1)
        return RP_EINVAL;
    if (n > 0 && (rec == nullptr || rank == nullptr))
        return RP_EINVAL;
    if (((reinterpret_cast<uintptr_t>(rec) | reinterpret_cast<uintptr_t>(rank) |
          reinterpret_cast<uintptr_t>(prio)) & 7u) != 0)
        return RP_EINVAL;   // 64-bit words
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    if (stats)
        std::memset(stats, 0, sizeof(*stats));
    if (n == 0)
        return RP_OK;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return RP_EDEVICE;
    // k = floor(n^(1-eps)) elements per block; the grid holds LM per lane,
    // the fewest of 1, 2, 4 that hold a whole block (more workgroups with
    // fewer elements each keep more memory operations in flight per round).
    const uint64_t bound = rp_aux_bound_words(n, eps);
    const void *const fns[3] = {reinterpret_cast<const void *>(rp_list_kernel<1>),
                                reinterpret_cast<const void *>(rp_list_kernel<2>),
                                reinterpret_cast<const void *>(rp_list_kernel<LM_MAX>)};
    const uint64_t lms[3] = {1, 2, LM_MAX};
    int li = 0;
    uint64_t gmax = 1;
    for (;; li++) {
        int occ = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fns[li], LWG, 0) != hipSuccess)
            return RP_EDEVICE;
        gmax = std::min<uint64_t>(LMAXG, (uint64_t)prop.multiProcessorCount * std::max(occ, 1));
        if (li == 2 || bound <= gmax * LWG * lms[li])
            break;
    }
    const uint64_t LM = lms[li];
    // Auxiliary words: flags (two parities) + error word + 3 result words.
    // The grid is limited so that they fit in the bound too.
    uint64_t G = std::min<uint64_t>(gmax, (bound + LWG * LM - 1) / (LWG * LM));
    while (G > 1 && 2 * G + 2 > bound)
        G /= 2;
    G = std::max<uint64_t>(1, G);
    const uint64_t k = std::max<uint64_t>(1, std::min<uint64_t>(bound, G * LWG * LM));
    const uint64_t aux_words = (G > 1 ? 2 * G : 0) + 1 + 3;
    if (stats) {
        stats->k = k;
        stats->aux_words = aux_words;
        stats->aux_bound_words = bound;
        stats->grid = G;
    }

    void *mem = nullptr;
    if (hipMallocAsync(&mem, aux_words * 8, stream) != hipSuccess) {
        (void)hipGetLastError();
        return RP_ENOMEM;
    }
    if (hipMemsetAsync(mem, 0, aux_words * 8, stream) != hipSuccess) {
        (void)hipFreeAsync(mem, stream);
        return RP_EDEVICE;
    }
    uint64_t *words = static_cast<uint64_t *>(mem);
    LParams p{};
    p.rec = rec;
    p.rank = rank;
    p.prio = prio;
    p.seed = seed;
    p.n = n;
    p.k = k;
    p.flags = G > 1 ? words : nullptr;
    p.err = reinterpret_cast<uint32_t *>(words + (G > 1 ? 2 * G : 0));
    p.out = words + (G > 1 ? 2 * G : 0) + 1;

    // Reject inconsistent links before anything is written.
    rp_list_check_kernel<<<1024, 256, 0, stream>>>(rec, n, p.err);
    uint32_t bad = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&bad, p.err, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipFreeAsync(mem, stream);
        return RP_EDEVICE;
    }
    if (bad) {
        (void)hipFreeAsync(mem, stream);
        return RP_EINVAL;
    }
    void *args[] = {&p};
    if (hipLaunchCooperativeKernel(fns[li], dim3((uint32_t)G),
                                   dim3(LWG), args, 0, stream) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFreeAsync(mem, stream);
        return RP_EDEVICE;
    }
    int rc = RP_OK;
    if (stats) {
        uint64_t host[4] = {0, 0, 0, 0};
        if (hipMemcpyAsync(host, p.err, 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipMemcpyAsync(host + 1, p.out, 24, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess) {
            rc = RP_EDEVICE;
        } else {
            const uint32_t e = (uint32_t)host[0];
            stats->status = e == 0 ? RP_OK : e == 2 ? RP_EINVAL : RP_ETIMEOUT;
            stats->phases = host[1];
            stats->contract_rounds = host[2];
            stats->rebuild_rounds = host[3];
        }
    }
    if (hipFreeAsync(mem, stream) != hipSuccess)
        return RP_EDEVICE;
    return rc;
}

}  // extern "C"
