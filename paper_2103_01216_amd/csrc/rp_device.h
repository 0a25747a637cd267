// rp_device.h -- device helpers shared by the kernels of librp (rp.hip,
// rp_batch.hip): device-coherent memory operations, the exact integer path
// for seed-mode swap targets, the reservation-slot hashes, wave reductions and
// register-held records.  Internal to the library; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rpdev {

constexpr uint32_t EMPTY = 0xFFFFFFFFu;
constexpr uint32_t RANKB = 24;          // priority = tag:8 | rank:24
constexpr uint32_t RANKMAX = (1u << RANKB) - 1u;

// ---------------------------------------------------------------- memory ops

template <typename T>
__device__ __forceinline__ T ld(const T *p)
{
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reset a word that is otherwise only updated by read-modify-write atomics.
// It must be written by an atomic RMW too: on gfx950 the RMW atomics and a
// plain device-scope store to the same word are not ordered with each other,
// and a store-based reset was observed to be lost.
__device__ __forceinline__ void clear_rmw(uint32_t *p)
{
    (void)__hip_atomic_exchange(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Alignment a record array needs: records whose size is a multiple of 8
// bytes are moved in 8-byte words, the others in 4-byte words.
__host__ __device__ inline uint32_t record_alignment(uint32_t eb)
{
    return (eb & 7u) == 0 ? 8u : 4u;
}

__device__ __forceinline__ void wait_mem()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Wait until at most N of this wave's vector memory operations are still
// outstanding.  They complete in the order they were issued (the counter the
// compiler's own waits rely on), so this waits for every operation issued
// before the last N.
template <int N>
__device__ __forceinline__ void wait_mem_but()
{
    static_assert(N >= 0 && N < 64, "the vector memory counter has 6 bits");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}


// ------------------------------------------------------- exact integer math

// SplitMix64 output function (Steele, Lea, Flood 2014): add the golden-ratio
// increment, two xor-shift-multiply rounds, final xor-shift, all mod 2^64.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Exact x mod d for 1 <= d <= 2^32 without an integer divider.  Quotient
// estimate from an IEEE-754 double reciprocal, then one exact correction in
// 64-bit integers: the estimate q is within 8193 of x/d (three roundings of
// relative size 2^-53 on a value below 2^64, a clamp of at most 2048 and a
// truncation), so r = x - q*d lies in (-2^46, 2^46) and is exact in int64;
// r/d is then resolved in doubles to within 2^-39, which leaves r within one
// d of [0, d) -- two conditional corrections each way finish it.
__device__ __forceinline__ uint64_t umod64(uint64_t x, uint64_t d)
{
    const double rd = 1.0 / (double)d;
    double qf = (double)x * rd;
    qf = fmin(qf, 18446744073709549568.0);  // largest double below 2^64
    const uint64_t q = (uint64_t)qf;
    int64_t r = (int64_t)(x - q * d);
    const int64_t q2 = (int64_t)((double)r * rd);
    r -= q2 * (int64_t)d;
    const int64_t sd = (int64_t)d;
    if (r < 0) r += sd;
    if (r < 0) r += sd;
    if (r >= sd) r -= sd;
    if (r >= sd) r -= sd;
    return (uint64_t)r;
}

// Swap target of iteration i in seed mode, i < 2^32.
__device__ __forceinline__ uint32_t seed_target(uint64_t seed, uint64_t i)
{
    return (uint32_t)umod64(splitmix64(seed ^ i), i + 1);
}


// The two reservation slots of key x: multiplicative hashing with two odd
// 64-bit constants, scaled to [0, T).
__device__ __forceinline__ uint32_t slot1(uint32_t key, uint32_t T)
{
    const uint32_t h = (uint32_t)(((uint64_t)key * 0x9E3779B97F4A7C15ull) >> 32);
    return (uint32_t)(((uint64_t)h * T) >> 32);
}

__device__ __forceinline__ uint32_t slot2(uint32_t key, uint32_t T)
{
    const uint32_t h = (uint32_t)(((uint64_t)key * 0xC2B2AE3D27D4EB4Full) >> 32);
    return (uint32_t)(((uint64_t)h * T) >> 32);
}

// ----------------------------------------------------------- wave helpers

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o)
            v += u;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------------ record moves

// Records of EB bytes held in registers (EB = 4, 8, 16).
template <int EB> struct Rec;
// LOADS: vector memory instructions one load issues.
template <> struct Rec<4> {
    static constexpr int LOADS = 1;
    uint32_t w;
    __device__ void load(const unsigned char *A, uint32_t i)
    { w = ld(reinterpret_cast<const uint32_t *>(A) + i); }
    __device__ void store(unsigned char *A, uint32_t i) const
    { st(reinterpret_cast<uint32_t *>(A) + i, w); }
};
template <> struct Rec<8> {
    static constexpr int LOADS = 1;
    uint64_t w;
    __device__ void load(const unsigned char *A, uint32_t i)
    { w = ld(reinterpret_cast<const uint64_t *>(A) + i); }
    __device__ void store(unsigned char *A, uint32_t i) const
    { st(reinterpret_cast<uint64_t *>(A) + i, w); }
};
template <> struct Rec<16> {
    static constexpr int LOADS = 2;
    uint64_t w0, w1;
    __device__ void load(const unsigned char *A, uint32_t i)
    {
        const uint64_t *q = reinterpret_cast<const uint64_t *>(A) + 2ull * i;
        w0 = ld(q);
        w1 = ld(q + 1);
    }
    __device__ void store(unsigned char *A, uint32_t i) const
    {
        uint64_t *q = reinterpret_cast<uint64_t *>(A) + 2ull * i;
        st(q, w0);
        st(q + 1, w1);
    }
};

template <> struct Rec<64> {
    static constexpr int LOADS = 8;
    uint64_t w[8];
    __device__ void load(const unsigned char *A, uint32_t i)
    {
        const uint64_t *q = reinterpret_cast<const uint64_t *>(A) + 8ull * i;
#pragma unroll
        for (int u = 0; u < 8; u++)
            w[u] = ld(q + u);
    }
    __device__ void store(unsigned char *A, uint32_t i) const
    {
        uint64_t *q = reinterpret_cast<uint64_t *>(A) + 8ull * i;
#pragma unroll
        for (int u = 0; u < 8; u++)
            st(q + u, w[u]);
    }
};

// Swap two records of eb bytes (multiple of 4) word by word.
__device__ __forceinline__ void swap_generic(unsigned char *A, uint32_t eb,
                                             uint32_t a, uint32_t b)
{
    if ((eb & 7u) == 0) {
        uint64_t *pa = reinterpret_cast<uint64_t *>(A + (uint64_t)a * eb);
        uint64_t *pb = reinterpret_cast<uint64_t *>(A + (uint64_t)b * eb);
        for (uint32_t j = 0; j < eb / 8; j += 4) {
            uint64_t x[4], y[4];
            const uint32_t m = min(4u, eb / 8 - j);
#pragma unroll
            for (uint32_t u = 0; u < 4; u++)
                if (u < m) { x[u] = ld(pa + j + u); y[u] = ld(pb + j + u); }
#pragma unroll
            for (uint32_t u = 0; u < 4; u++)
                if (u < m) { st(pa + j + u, y[u]); st(pb + j + u, x[u]); }
        }
    } else {
        uint32_t *pa = reinterpret_cast<uint32_t *>(A + (uint64_t)a * eb);
        uint32_t *pb = reinterpret_cast<uint32_t *>(A + (uint64_t)b * eb);
        for (uint32_t j = 0; j < eb / 4; j++) {
            const uint32_t x = ld(pa + j), y = ld(pb + j);
            st(pa + j, y);
            st(pb + j, x);
        }
    }
}

// Reductions over the 64 lanes of a (converged) wave with DPP moves: quad
// permutes, half-row and row mirrors, then the two row broadcasts; the
// result forms in lane 63 and is read back as a uniform value.  A few VALU
// cycles per step instead of a cross-lane permute through LDS.
template <typename Op>
__device__ __forceinline__ uint32_t wave_reduce_dpp(uint32_t v, Op op)
{
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint32_t wave_sum_dpp(uint32_t v)
{
    return wave_reduce_dpp(v, [](uint32_t a, uint32_t b) { return a + b; });
}

__device__ __forceinline__ uint32_t wave_max_dpp(uint32_t v)
{
    return wave_reduce_dpp(v, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
}

// Number of lanes below this one whose bit is set in the wave mask m.
__device__ __forceinline__ uint32_t lane_rank(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, (uint32_t)__shfl_xor(v, o, 64));
    return v;
}

}  // namespace rpdev
