/*
 * rp.h -- C ABI of librp: parallel in-place random permutation on one
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (Gu, Obeya, Shun, "Parallel In-Place Algorithms: Theory and
 * Practice", Section 4.1, the Knuth-Shuffle listing): given an array A of n
 * records and swap targets H with 0 <= H[i] <= i, apply
 *
 *     for i = n-1 down to 0:  swap(A[i], A[H[i]])
 *
 * (the paper writes it 1-based, i = n..1 and H[i] in [1, i]).  The library
 * computes exactly this permutation, bit for bit, with the relaxed-PIP
 * algorithm of Section 4.1 (rounds over the first k unfinished swaps, k about
 * n^(1-eps), Theorem on relaxed-PIP random permutation via the Decomposable
 * Property of Section 4) implemented in the RP-Final form of Section 7.4 and
 * Appendix A.2 (single reservation on R[H[i]], dense array for the keys of
 * the swaps added in the current round; the reservation array R itself is
 * hashed into O(k) priority slots written with atomic max).  Auxiliary
 * space is O(n^(1-eps)) words: every byte of device memory a call allocates
 * is counted and the total never exceeds 8 * floor(n^(1-eps)) bytes.
 *
 * Conventions
 *   - A word is 8 bytes.
 *   - Pointers are device pointers unless a comment says "host".
 *   - hipStream_t is passed as void* so this header needs no HIP headers;
 *     NULL means the null (default) stream.
 *   - Calls are stream-ordered: the permutation is complete when the stream
 *     reaches the work the call enqueued.  Unless a comment says otherwise a
 *     call does not wait for the GPU.
 *   - Every call that returns an error leaves A untouched.
 *   - n must be below 2^32 (indices are packed into 32-bit slots).
 */
#ifndef RP_H
#define RP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define RP_OK 0
#define RP_PENDING 1   /* rp_batch_poll: not finished yet */
#define RP_EINVAL (-1) /* bad argument, or some H[i] > i */
#define RP_ENOMEM (-2) /* device memory or the auxiliary budget cannot be met */
#define RP_EDEVICE (-3) /* a HIP runtime call failed */
#define RP_ETIMEOUT (-4) /* device watchdog fired (a barrier or the round count
                            exceeded its bound); reported through stats */
#define RP_ECANCELED (-5) /* rp_server_destroy: the request was never launched */
#define RP_ETOOBIG (-6) /* rp_shuffle_inplace_noalloc: the call needs more
                           auxiliary memory than the static scratch holds */

/*
 * Per-call statistics, written by the device and copied into caller memory
 * (host) when the stream reaches the end of the call.
 *   k                 active swaps per round the call plans for (the prefix
 *                     size); with one barrier per round the refill aims
 *                     at k without knowing the round's commits yet, so a
 *                     round may hold a few more (see max_active)
 *   aux_words         auxiliary memory of the call, in 8-byte words
 *                     (rounded up): the device memory it allocated for
 *                     tables, bitmaps, barrier flags and counters, plus the
 *                     LDS that holds the table and window of a
 *                     one-workgroup launch (which then allocates none)
 *   aux_bound_words   floor(n^(1-eps))
 *   rounds            reserve/commit rounds executed
 *   attempts          swap attempts summed over rounds (self-loops excluded)
 *   retries           attempts that lost and were carried to the next round
 *   max_active        largest number of swaps attempted in one round
 *                     (rounds, attempts, retries and max_active may differ
 *                     slightly between runs of one input: a workgroup's
 *                     reservation for the next round can make a slower
 *                     workgroup's check lose once more; the permutation
 *                     itself never differs)
 *   self_loops        swaps with H[i] = i, retired without a reservation
 *   grid, slots_per_lane, table_slots   launch shape and number of 32-bit
 *                     slots of the hashed reservation array
 *   status            RP_OK, or RP_ETIMEOUT if the device watchdog fired
 *   inflight_words    state the active swaps hold in registers (the
 *                     larger of k and max_active swaps), in 8-byte
 *                     words: per swap its source and target (4 bytes each)
 *                     and, for records of 4, 8 or 16 bytes (and 64 with one
 *                     barrier per round), both records; other record sizes
 *                     are moved word by word and hold none.  Not device
 *                     memory and not part of aux_words; reported so that the
 *                     whole working set of a round can be compared with the
 *                     bound (Section 4.1 keeps the prefix's H values inside
 *                     its O(n^(1-eps)) table).
 *   throttled_rounds  rounds whose refill was cut short so that every active
 *                     swap's rank (its distance above the round's lowest
 *                     fresh index) fits the 24-bit priority field
 */
typedef struct rp_stats {
    uint64_t k;
    uint64_t aux_words;
    uint64_t aux_bound_words;
    uint64_t rounds;
    uint64_t attempts;
    uint64_t retries;
    uint64_t max_active;
    uint64_t self_loops;
    uint64_t grid;
    uint64_t slots_per_lane;
    uint64_t table_slots;
    int64_t status;
    uint64_t inflight_words;
    uint64_t throttled_rounds;
} rp_stats;

/*
 * floor(n^(1-eps)): the auxiliary-space bound in words (Section 3.2, the
 * relaxed PIP model's O(n^(1-eps)) auxiliary space; Section 4.1's prefix of
 * n^(1-eps) swaps).  Pure host arithmetic, no GPU.  Returns 0 for n == 0 or
 * eps outside (0, 1).
 */
uint64_t rp_aux_bound_words(uint64_t n, double eps);

/*
 * Plan a call without running it (host only, no GPU): fills *stats_out
 * (host) with the k, aux_words, aux_bound_words, grid, slots_per_lane and
 * table_slots that rp_shuffle_inplace would use on device `device` for these
 * arguments; the other fields are zero.  Returns RP_OK, RP_EINVAL, or
 * RP_EDEVICE when `device` cannot be queried.  A bound too small for even the
 * smallest table gives k = 1 (one active swap: the sequential loop, which
 * needs one word).  device < 0 assumes an MI355X with 256 compute units.
 */
int rp_plan(uint64_t n, uint32_t elem_bytes, double eps, int device,
            rp_stats *stats_out);

/*
 * Shuffle A in place (Section 4.1; the RP-Final implementation of
 * Section 7.4 / Appendix A.2).
 *   A           n records of elem_bytes bytes each, contiguous (device),
 *               aligned to 8 bytes when elem_bytes is a multiple of 8 and to
 *               4 otherwise.  Permuted in place; the caller owns it.
 *   n           number of records, n < 2^32.  n <= 1 is a successful no-op.
 *   elem_bytes  record size: a multiple of 4 in [4, 256].
 *   H           swap targets, n uint64 values with H[i] <= i (device,
 *               8-byte aligned, read-only, not counted as auxiliary space), or NULL for
 *               seed mode: H[i] = splitmix64(seed ^ i) mod (i + 1), with
 *               SplitMix64 as published by Steele, Lea and Flood (2014).
 *   seed        used only in seed mode.
 *   eps         in (0, 1); auxiliary space is at most floor(n^(1-eps))
 *               words.
 *   stream      hipStream_t (as void*), or NULL.
 *   stats       host memory (pinned, or pageable at the cost of a
 *               synchronous copy) receiving rp_stats when the stream reaches
 *               the end of the call; may be NULL.
 * Errors: RP_EINVAL for A == NULL with n > 1, a bad elem_bytes or eps,
 * n >= 2^32, a misaligned A or H (checked on the host, before any device
 * work), or (H mode) some H[i] > i -- H mode validates H on the device
 * first and, for that check only, waits for the stream before returning.
 * RP_ENOMEM if device memory for the auxiliary structures cannot be had.
 * RP_EDEVICE if a HIP call fails.  A is untouched whenever an error is
 * returned.  A device watchdog error is reported in stats->status.
 */
int rp_shuffle_inplace(void *A, uint64_t n, uint32_t elem_bytes,
                       const uint64_t *H, uint64_t seed, double eps,
                       void *stream, rp_stats *stats);

/*
 * Reservation variants of the same operation, for comparing design choices
 * (Section 7.4 and the appendix on the random permutation implementations:
 * the versions differ in how the reservation array R is held and how many
 * reservations a swap makes per round).  Every variant computes exactly the
 * permutation of rp_shuffle_inplace; only rounds, retries and memory traffic
 * differ.
 *   RP_VARIANT_FINAL   the path of rp_shuffle_inplace: one reservation, on
 *                      H[s], in a hashed slot array; the round's consecutive
 *                      keys are checked in a dense window array
 *   RP_VARIANT_ONERES  one reservation on H[s]; the source check also goes
 *                      through the hashed slots (no dense window)
 *   RP_VARIANT_TWORES  Algorithm 1 as printed: reservations on both s and
 *                      H[s] (hashed); a swap commits when both hold its own
 *                      priority; H[s] of every active swap held in registers
 *   RP_VARIANT_FLAT    as RP_VARIANT_TWORES, with H[s] of the active swaps in
 *                      an array of the prefix's size (one word per swap slot,
 *                      written when the swap enters, read back to reserve and
 *                      to commit)
 *   RP_VARIANT_NAIVE   as RP_VARIANT_TWORES, with H[s] of the active swaps in
 *                      a hashed table keyed by s (open addressing, twice the
 *                      prefix's size, two parities cleared whole in turn):
 *                      set every round, read back to commit
 *   RP_VARIANT_LINEAR  the non-in-place scheme: R is an array of n 8-byte
 *                      words (exact, never cleaned: the round number is part
 *                      of every priority) and k is the largest the grid
 *                      holds; eps does not bound its memory
 * Arguments and errors as rp_shuffle_inplace; RP_EINVAL for an unknown
 * variant.  stats->aux_words counts what the variant allocated (for
 * RP_VARIANT_LINEAR it exceeds aux_bound_words).
 */
#define RP_VARIANT_FINAL 0
#define RP_VARIANT_ONERES 1
#define RP_VARIANT_TWORES 2
#define RP_VARIANT_LINEAR 3
#define RP_VARIANT_FLAT 4
#define RP_VARIANT_NAIVE 5

int rp_shuffle_variant(void *A, uint64_t n, uint32_t elem_bytes,
                       const uint64_t *H, uint64_t seed, double eps, int variant,
                       void *stream, rp_stats *stats);

/*
 * rp_shuffle_inplace for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operation, arguments, kernels and result, but the
 * auxiliary words and the statistics record live in a static device array of
 * RP_NOALLOC_SCRATCH_BYTES bytes (one per device, held until the process
 * ends) instead of memory obtained per call.  The call allocates nothing: no
 * hipMalloc/hipFree of any kind.  Its first call on a device looks up that
 * device's array (and queries the device) once.
 *   - Rejects, with RP_ETOOBIG and A untouched, a call whose plan needs more
 *     than the array holds (256 bytes of alignment slack and the 112-byte
 *     statistics record included).  1 MiB covers every eps at which
 *     floor(n^(1-eps)) <= 131000 words, e.g. n = 2^30 at eps = 0.5
 *     (256 KiB); n = 2^28 at eps = 0.25 (16 MiB) is rejected.
 *   - Every call on a device shares that device's array and leaves its
 *     contents behind; each call clears the words it uses before its rounds.
 *     Calls that overlap on one device (other streams, other threads, the
 *     same graph launched twice at once) race on the array and give wrong
 *     results: serialise them.
 *   - Otherwise as rp_shuffle_inplace (errors, stats, stream order; H mode
 *     still waits for the stream after its validation pass).
 */
#define RP_NOALLOC_SCRATCH_BYTES (1u << 20)

int rp_shuffle_inplace_noalloc(void *A, uint64_t n, uint32_t elem_bytes,
                               const uint64_t *H, uint64_t seed, double eps,
                               void *stream, rp_stats *stats);

/*
 * The auxiliary memory that the calling thread's last rp_shuffle_inplace or
 * rp_shuffle_variant call obtained, in bytes, as recorded where it was
 * obtained: the sizes passed to its device allocation calls (the statistics
 * record excluded) plus the dynamic LDS of its launch.  Lets a caller check
 * the floor(n^(1-eps))-word bound of Section 3.2 independently of
 * rp_stats.aux_words.  0 before the first call and after a call that
 * allocated nothing (n <= 1, or an error before allocating).  Host only;
 * no device work.
 *
 * Two environment variables exercise the error paths of these calls from
 * the host: RP_FAIL_ALLOC=1 makes the auxiliary allocation fail (the call
 * returns RP_ENOMEM and A is untouched); RP_MAX_ROUNDS=r lowers the round
 * limit to r (the call completes with stats->status = RP_ETIMEOUT after r
 * rounds, and A then holds a permutation of its input, not the shuffle).
 */
uint64_t rp_last_call_aux_bytes(void);

/*
 * Seed-mode swap targets on the device, for testing the exact integer path:
 * out[j] = splitmix64(seed ^ idx[j]) mod (idx[j] + 1) for j < count, with
 * idx[j] < 2^32.  idx and out are device arrays.  Stream-ordered.
 */
int rp_seed_targets(const uint64_t *idx, uint64_t count, uint64_t seed,
                    uint64_t *out, void *stream);

/* ------------------------------------------------------------------------
 * Measurement probes: the device costs a round is made of, measured in
 * isolation, to compare the shuffle's time with.  Section 7.4 counts the
 * sequential and random accesses a swap makes per round; these give the
 * price of each kind on this device.  None of them is part of the shuffle.
 * ------------------------------------------------------------------------ */

/*
 * The data movement of a shuffle with nothing else: for every s < n (in no
 * particular order, unsynchronised) read A[s] and A[H[s]], H[s] the seed-mode
 * target, and write them back exchanged.  Swaps that share a location race,
 * so A afterwards is NOT a permutation of its input: re-initialise it.
 * Moves the shuffle's algorithmic bytes (4 * elem_bytes per element) at its
 * real addresses.  elem_bytes 4, 8, 16 or 64; A aligned to
 * min(elem_bytes, 16) bytes; n < 2^32.  Stream-ordered, non-blocking; time it
 * with events.  RP_EINVAL, RP_EDEVICE.
 */
int rp_probe_random_rmw(void *A, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                        void *stream);

/* Streaming copy of `bytes` (multiple of 16; both pointers 16-byte aligned,
 * device) in 16-byte accesses: the bandwidth reference, and the kernel of
 * known traffic that hardware byte counters are scaled by.  Stream-ordered,
 * non-blocking.  RP_EINVAL, RP_EDEVICE. */
int rp_probe_copy(void *dst, const void *src, uint64_t bytes, void *stream);

/* Microseconds per grid-wide flag barrier (the barrier between the phases
 * of a round) on `grid` workgroups of 256 lanes, averaged over `rounds`
 * barriers of one cooperative launch.  Allocates its flags, waits for the
 * stream; *us_per_barrier (host) receives the result.  2 <= grid <= 2048.
 * RP_EINVAL, RP_ENOMEM, RP_EDEVICE. */
int rp_probe_barrier(uint32_t grid, uint32_t rounds, void *stream, double *us_per_barrier);

/* Device-scope 32-bit atomic max (the reservation's operation): grid
 * workgroups of 256 lanes each issue per_lane atomics on pseudo-random slots
 * of a table of table_slots words, either all in flight at once
 * (chained = 0: throughput) or each after the previous one returned
 * (chained = 1: latency).  *ns_total (host) receives the launch's time in
 * nanoseconds.  Allocates the table, waits for the stream.  RP_EINVAL,
 * RP_ENOMEM, RP_EDEVICE. */
int rp_probe_atomics(uint32_t table_slots, uint32_t grid, uint32_t per_lane, int chained,
                     void *stream, double *ns_total);

/* ------------------------------------------------------------------------
 * Batched form: many independent shuffles in one persistent launch.
 *
 * Each request is an independent call of the operation above on its own array
 * (same semantics and the same auxiliary bound per request, floor(n^(1-eps))
 * words, here held in the on-chip LDS of the lanes that run it).  Requests of
 * one batch share one record size; n < 2^32 per request.  The batch is
 * stream-ordered; completion can be observed without blocking.
 */
typedef struct rp_batch_request {
    void *A;                 /* device records, permuted in place (caller-owned);
                                aligned as for rp_shuffle_inplace */
    uint64_t n;              /* number of records, < 2^32 */
    uint32_t elem_bytes;     /* multiple of 4 in [4, 256]; equal for the batch */
    uint32_t reserved;       /* 0 */
    const uint64_t *H;       /* device targets (H[i] <= i, 8-byte aligned) or NULL:
                                seed mode */
    uint64_t seed;           /* seed mode: H[i] = splitmix64(seed ^ i) mod (i+1) */
    double eps;              /* in (0, 1) */
} rp_batch_request;

typedef struct rp_batch_result {
    uint64_t rounds;         /* rounds run for this request */
    uint64_t attempts;       /* swap attempts summed over its rounds */
    int32_t status;          /* RP_OK, RP_EINVAL (some H[i] > i; A untouched),
                                RP_ETIMEOUT */
    uint32_t aux_words;      /* 8-byte words of round state it used */
} rp_batch_result;

/* Schedule of a batch launch (chosen by rp_batch_autotune, or defaults):
 * requests with n >= wave_cutoff run one per workgroup, smaller ones one per
 * wave; table_ratio_x16 = 16 * reservation slots per active swap;
 * workgroups_per_cu = resident workgroups per compute unit (at most what the
 * workgroup size allows); workgroup_lanes = 256 or 1024 (0: 256) -- a
 * 1024-lane workgroup holds four times as many active swaps of one request,
 * so a large request needs a quarter of the rounds; late_loads = 1 reads a
 * swap's two records only once it has won its round (fewer random reads,
 * longer rounds), 0 reads them before the decision. */
typedef struct rp_batch_schedule {
    uint32_t wave_cutoff;
    uint32_t table_ratio_x16;
    uint32_t workgroups_per_cu;
    uint32_t tuned_ms_x1000;  /* out: best trial time in microseconds */
    uint32_t workgroup_lanes;
    uint32_t late_loads;
} rp_batch_schedule;

/*
 * Choose a schedule for batches shaped like reqs (host array of count
 * requests): times trial launches of candidate schedules on scratch copies of
 * an evenly spaced sample of the requests (seed mode; the caller's arrays are
 * not touched), waits for them, writes the fastest to *out (host) and makes it
 * the default of later rp_batch_submit calls that pass no schedule.  The
 * choice is remembered in a text file with the device (architecture and
 * compute units), the record size, the eps values and the sample's size mix
 * (share of requests per octave of n); a later call on the same kind of
 * device, for the same record size and eps values and a size mix whose
 * cumulative shares over the octaves stay within 0.15 of a remembered one
 * (batches drawn from one distribution), takes the closest remembered
 * schedule without trial runs.  The file is $RP_TUNE_CACHE, or
 * $HOME/.cache/librp/batch_schedules.txt; RP_TUNE_CACHE set to the empty
 * string turns this off.  A file that cannot be read or written is ignored.
 * Returns RP_OK, RP_EINVAL, RP_ENOMEM.
 */
int rp_batch_autotune(const rp_batch_request *reqs, uint32_t count, void *stream,
                      rp_batch_schedule *out);

/*
 * Enqueue a batch (reqs is a host array, copied before return; sched may be
 * NULL for the tuned or default schedule).  Does not wait for the GPU.  Writes
 * a batch id to *batch_id (host).  RP_EINVAL for a malformed request (no
 * request runs then); requests whose H fails validation finish with status
 * RP_EINVAL and untouched arrays while the rest of the batch runs.
 */
int rp_batch_submit(const rp_batch_request *reqs, uint32_t count,
                    const rp_batch_schedule *sched, void *stream, uint64_t *batch_id);

/* Non-blocking: *n_done (host, may be NULL) = finished requests; returns
 * RP_OK when all are finished, RP_PENDING otherwise, RP_EINVAL for an unknown
 * id. */
int rp_batch_poll(uint64_t batch_id, uint32_t *n_done);

/* Non-blocking: RP_OK if request `index` (caller's order) has finished and its
 * array may be read by later stream work, RP_PENDING if not. */
int rp_batch_request_done(uint64_t batch_id, uint32_t index);

/* Waits for the batch and copies count results (caller's order) to out
 * (host, may be NULL). */
int rp_batch_results(uint64_t batch_id, rp_batch_result *out);

/* Waits for the batch and frees its bookkeeping; the id becomes invalid. */
int rp_batch_release(uint64_t batch_id);

/*
 * Several independent shuffles in one cooperative launch, each on all the
 * workgroups it would get alone: for running a few large shuffles side by
 * side (one cooperative launch at a time is what the device runs).  Each
 * request is the operation of rp_shuffle_inplace on its own array, planned
 * exactly as a call of its own would be (the same k and auxiliary words,
 * floor(n^(1-eps)) per request, allocated apart for each), on its own group
 * of workgroups whose rounds are synchronised among themselves only; the
 * result of each is its Knuth shuffle, whatever else runs in the group.  A
 * request whose bound holds no table (k = 1) runs as the sequential loop
 * ahead of the group, as it would alone.
 *   reqs    host array of count requests (fields as for rp_batch_submit),
 *           count <= 16, one elem_bytes for all.
 *   stream  hipStream_t (as void*), or NULL.  Stream-ordered.
 *   stats   host array of count rp_stats, filled when the stream reaches the
 *           end of the call, or NULL.
 * Errors: RP_EINVAL for a request rp_shuffle_inplace would reject, mixed
 * record sizes, count > 16, a request whose plan needs more than one swap
 * slot per lane (it fills the device by itself), groups whose planned grids
 * (rp_plan's grid) add up to more than rp_group_capacity, or (explicit
 * targets) some H[i] > i in any
 * request (checked first; the call then waits for the stream).  RP_ENOMEM,
 * RP_EDEVICE.  Every A is untouched whenever an error is returned.
 * rp_last_call_aux_bytes reports the sum over the group.
 */
int rp_shuffle_group(const rp_batch_request *reqs, uint32_t count, void *stream,
                     rp_stats *stats);

/*
 * The most workgroups the planned grids of one rp_shuffle_group call may add
 * up to on `device` for records of elem_bytes (the workgroups of its kernel
 * that can be resident at once).  Host only; *workgroups receives it.
 * RP_EINVAL for a bad elem_bytes or NULL; RP_EDEVICE.
 */
int rp_group_capacity(uint32_t elem_bytes, int device, uint64_t *workgroups);

/* ------------------------------------------------------------------------
 * List ranking by in-place list contraction (Section 4.2: list contraction
 * has the Decomposable Property, so Algorithm 2 can be applied to
 * n^(1-eps) elements at a time).
 *
 * rec: device array of 2n words, element i's (prev, next) pair (rec, rank
 * and prio are 8-byte aligned; RP_EINVAL otherwise).  On input
 * the low 32 bits of rec[2i] and rec[2i+1] are the previous and next
 * element (0xFFFFFFFF = none; any number of disjoint lists; the high bits
 * are ignored).  The elements are contracted in blocks of
 * k = floor(n^(1-eps)) indices (block j = [jk, (j+1)k)); inside a block,
 * rounds of Algorithm 2 splice out every element whose key
 * (block, priority, index) is below both current neighbours' keys; list
 * heads are never spliced.  Priorities: prio[i] (device, may be NULL) or
 * splitmix64(seed ^ i).  On return the pair of every non-head element holds
 * its record in the contraction tree, overwriting the input pointers:
 *   rec[2i]   = L | (offset << 32): L = left neighbour when it was spliced,
 *               offset = its distance from L in the list
 *   rec[2i+1] = R | (round << 32): R = right neighbour when it was spliced,
 *               round = the round of its block in which it went
 * A head's rec[2h] is unchanged and rec[2h+1] = 0xFFFFFFFF | (length << 32),
 * the number of elements of its list.
 * rank (device, n words, caller-owned) receives every element's position in
 * its list (heads 0).
 * Auxiliary memory: barrier flags and four words, at most
 * max(floor(n^(1-eps)), 4) 8-byte words.  Errors: RP_EINVAL for bad
 * arguments or inconsistent links (checked before anything is written);
 * RP_ENOMEM; RP_EDEVICE.  A cycle (links consistent, no head) is found
 * during the contraction: stats->status = RP_EINVAL, rec partly rewritten.
 * With stats != NULL (host) the call waits for the stream to fill it.
 * ------------------------------------------------------------------------ */
typedef struct rp_list_stats {
    uint64_t k;                  /* block size */
    uint64_t aux_words;          /* 8-byte words allocated */
    uint64_t aux_bound_words;    /* floor(n^(1-eps)) */
    uint64_t phases;             /* blocks contracted */
    uint64_t contract_rounds;    /* rounds of Algorithm 2, all blocks */
    uint64_t rebuild_rounds;     /* reconstruction steps */
    uint64_t grid;               /* workgroups */
    int64_t status;              /* RP_OK, RP_EINVAL (cycle), RP_ETIMEOUT */
} rp_list_stats;

int rp_list_rank(uint64_t *rec, uint64_t n, const uint64_t *prio, uint64_t seed, double eps,
                 uint64_t *rank, void *stream, rp_list_stats *stats);

/* ------------------------------------------------------------------------
 * Serving form: a request loop on one device.
 *
 * The paper motivates in-place algorithms by the limited memory of a single
 * machine (Section 1) and reports the memory each algorithm holds beyond its
 * input (Section 7.6).  A server applies that to a stream of shuffle
 * requests: it owns a device arena of a fixed budget, admits requests in
 * arrival order while their arrays fit in the free part of the arena, fills
 * each admitted array on the device, and runs admitted requests as batched
 * launches (the batched form above) that overlap on the device with launches
 * still running, or through one resident kernel that takes each request as
 * it arrives.  Each request's result is the Knuth shuffle of its array with
 * its seed, whatever else runs beside it.  One host thread per server does
 * all device work; the calls below only exchange bookkeeping with it and
 * never block on the GPU (rp_server_destroy excepted).
 *
 * Resident mode: while the server has work, one kernel (one 512-lane
 * workgroup per compute unit) stays on the device and takes admitted
 * requests from a ring in host memory as they arrive, so a request starts on
 * the next free workgroup instead of with the next launch (admission at the
 * granularity of a workgroup's request boundary).  A request below
 * 2^large_log2 elements (2^20 by default) runs on one workgroup with its
 * round state in LDS; a larger one on a gang of idle workgroups (at most a
 * quarter of them and half of those the posted requests leave free; on one
 * workgroup when fewer than 8 would be left) that runs the one-barrier rounds
 * with its tables in the arena, counted against the admission budget and the
 * auxiliary bound of its eps.  The kernel fills each array itself (identity,
 * or a copy from device or pinned host memory: rp_server_submit rejects any
 * other source with RP_EINVAL), leaves 20 ms after the server runs out of
 * work (every wave reaches a stop word the host sets) and is launched again
 * when work arrives.  It runs on the server's own stream; device work that
 * other code puts on a stream sharing its hardware queue may wait until it
 * leaves.
 * ------------------------------------------------------------------------ */

#define RP_SERVE_BATCHED 0  /* admitted requests go out as batched launches */
#define RP_SERVE_PLAIN 1    /* one rp_shuffle_inplace per request, in order */
#define RP_SERVE_RESIDENT 2 /* admitted requests go to a resident kernel */

#define RP_INIT_IDENTITY 0  /* A[i] = i (elem_bytes 4 or 8: the integer i;
                               other sizes: word 0 = i, other words 0) */
#define RP_INIT_COPY 1      /* A = n * elem_bytes bytes copied from src
                               (device or pinned host memory) */

#define RP_REQ_QUEUED 0     /* waiting for arena space */
#define RP_REQ_ADMITTED 1   /* array allocated, not launched yet */
#define RP_REQ_RUNNING 2    /* launched */
#define RP_REQ_DONE 3       /* finished; A holds the result until released */

typedef struct rp_server_config {
    uint64_t mem_budget_bytes;   /* arena size: bound on the bytes of all
                                    admitted, unreleased arrays; 0: the
                                    process default (rp_set_mem_budget) */
    uint32_t mode;               /* RP_SERVE_BATCHED, RP_SERVE_PLAIN or
                                    RP_SERVE_RESIDENT */
    uint32_t max_batch;          /* requests per launch; 0: no limit */
    uint32_t large_log2;         /* n >= 2^large_log2 uses the large-request
                                    streams (resident mode: may run on a
                                    gang); 0: 22 (resident mode: 20) */
    uint32_t tick_us;            /* dispatcher poll interval; 0: 50 */
    uint32_t auto_release;       /* 1: free each array as soon as it is done
                                    (results are not kept) */
    uint32_t large_alone;        /* 1: run large requests, in arrival
                                    order, on the workgroups a call of their
                                    own gets instead of in one workgroup of a
                                    batched launch: as many as fit one
                                    cooperative launch together in one
                                    rp_shuffle_group call (or one alone with
                                    rp_shuffle_inplace), launch after launch;
                                    when more than 16 wait, batch them */
    rp_batch_schedule schedule;  /* small requests' schedule; all zero: 1024-lane
                                    workgroups, two per compute unit, the
                                    shortest launches (lowest latency) */
} rp_server_config;

typedef struct rp_server_request {
    uint64_t n;                  /* records, 1 <= n < 2^32 */
    uint32_t elem_bytes;         /* multiple of 4 in [4, 256] */
    uint32_t init;               /* RP_INIT_IDENTITY or RP_INIT_COPY */
    const void *src;             /* RP_INIT_COPY: source records; the caller
                                    keeps them valid until the request runs */
    uint64_t seed;               /* H[i] = splitmix64(seed ^ i) mod (i+1) */
    double eps;                  /* in (0, 1) */
} rp_server_request;

typedef struct rp_server_ticket_info {
    int32_t state;               /* RP_REQ_* */
    int32_t status;              /* RP_OK, or the request's error once done */
    uint64_t t_submit_ns;        /* steady-clock times (ns) of each step; */
    uint64_t t_admit_ns;         /* 0 when not reached yet */
    uint64_t t_launch_ns;
    uint64_t t_done_ns;          /* when the dispatcher saw completion */
    void *A;                     /* device array (NULL until admitted, and
                                    after release) */
    uint64_t rounds;             /* rounds run (batched and resident modes) */
    uint32_t aux_words;          /* round-state words used */
    uint32_t workgroups;         /* resident mode: workgroups it ran on (1,
                                    or its gang's size); 0 in other modes */
} rp_server_ticket_info;

typedef struct rp_server_stats {
    uint64_t submitted, admitted, done, launches;
    uint64_t bytes_in_use;       /* arena bytes held by admitted requests */
    uint64_t peak_bytes;         /* maximum of bytes_in_use so far */
    uint64_t elements_done;      /* sum of n over finished requests */
} rp_server_stats;

/* Process-wide default admission budget (bytes of device memory for request
 * arrays) of servers created with mem_budget_bytes = 0.  Host only.  The
 * initial default is 64 GiB.  RP_EINVAL for 0. */
int rp_set_mem_budget(uint64_t bytes);

/* Create a server on the current device: allocates the arena and starts the
 * dispatcher thread.  *server (host) receives its handle.  RP_EINVAL for a bad
 * config, RP_ENOMEM when the arena cannot be allocated. */
int rp_server_create(const rp_server_config *cfg, uint64_t *server);

/* Queue a request (host struct, copied).  Never blocks.  RP_EINVAL for a bad
 * request or one larger than the whole budget.  *ticket (host) identifies it. */
int rp_server_submit(uint64_t server, const rp_server_request *req, uint64_t *ticket);

/* Snapshot of a request's state (host struct).  RP_EINVAL for an unknown or
 * released ticket. */
int rp_server_info(uint64_t server, uint64_t ticket, rp_server_ticket_info *info);

/* Tickets finished since the last call, oldest first: up to max of them are
 * written to tickets (host) and *count (host) says how many. */
int rp_server_completed(uint64_t server, uint64_t *tickets, uint32_t max, uint32_t *count);

/* Enqueue, on `stream`, a copy of a finished request's n * elem_bytes result
 * bytes to dst (device or pinned host memory, caller-owned).  RP_PENDING if
 * the request has not finished; RP_EINVAL for an unknown ticket or one whose
 * array was already freed (auto_release).  Release the ticket only after the
 * copy has completed on `stream`. */
int rp_server_copy_out(uint64_t server, uint64_t ticket, void *dst, void *stream);

/* Free a finished request's array (its space returns to the arena) and forget
 * the ticket.  RP_PENDING if the request has not finished yet. */
int rp_server_release(uint64_t server, uint64_t ticket);

/* Counters (host struct). */
int rp_server_stats_get(uint64_t server, rp_server_stats *out);

/* Stop accepting requests, let running ones finish, cancel the ones not yet
 * launched (status RP_ECANCELED), free all memory and end the dispatcher
 * thread.  Blocks until done. */
int rp_server_destroy(uint64_t server);

#ifdef __cplusplus
}
#endif

#endif /* RP_H */
