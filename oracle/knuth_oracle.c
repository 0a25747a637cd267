/*
 * knuth_oracle.c -- CPU oracle for the in-place random permutation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file: only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP library; it has its own SplitMix64.
 *
 * What it computes (Gu, Obeya, Shun, "Parallel In-Place Algorithms: Theory
 * and Practice", Section 4.1, the sequential Knuth-Shuffle listing): for i
 * from n down to 1, swap A[i] with A[H[i]], where H[i] is drawn uniformly
 * from [1, i].  This file uses 0-based indices throughout: i runs from n-1
 * down to 0 and 0 <= H[i] <= i.  The parallel and in-place algorithms of the
 * paper (Algorithm 1 and its relaxed-PIP form in Section 4.1, the RP-Final
 * implementation of Section 7.4 / Appendix A.2) compute exactly this result,
 * so the plain sequential loop is the oracle; there is no tolerance.
 *
 * Elements are opaque records of elem_bytes bytes; the loop moves bytes and
 * never looks at them.  The listing's first loop (A[i] <- i) is not part of
 * the shuffle of a given array: callers pass whatever A they want permuted.
 *
 * Seed mode draws H[i] = splitmix64(seed XOR i) mod (i + 1), with
 * SplitMix64 as published by Steele, Lea and Flood (OOPSLA 2014) in the form
 * of Vigna's public-domain reference: add the golden-ratio increment, then
 * the two xor-shift-multiply steps and a final xor-shift, all mod 2^64.
 *
 * Parity: pinned by the tests (paper's worked example, closed forms,
 * bijection over all H for n <= 8, chi-square uniformity, published
 * SplitMix64 outputs).  No function here is "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* SplitMix64 output function applied to one 64-bit input x. */
uint64_t oracle_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Swap target of iteration i in seed mode: uniform-ish draw from [0, i]. */
uint64_t oracle_seed_target(uint64_t seed, uint64_t i)
{
    return oracle_splitmix64(seed ^ i) % (i + 1);
}

/* Fill H[0..n) with the seed-mode swap targets. */
void oracle_seed_targets(uint64_t n, uint64_t seed, uint64_t *H)
{
    for (uint64_t i = 0; i < n; i++)
        H[i] = oracle_seed_target(seed, i);
}

static void swap_records(unsigned char *A, uint64_t a, uint64_t b,
                         uint32_t eb, unsigned char *tmp)
{
    if (a == b)
        return;
    memcpy(tmp, A + a * eb, eb);
    memcpy(A + a * eb, A + b * eb, eb);
    memcpy(A + b * eb, tmp, eb);
}

/*
 * Sequential Knuth shuffle with explicit targets (Section 4.1 listing).
 * Returns 0, or -1 if some H[i] > i (checked before anything moves) or the
 * arguments are unusable.  A is modified in place.
 */
int oracle_knuth_shuffle(void *A, uint64_t n, uint32_t elem_bytes,
                         const uint64_t *H)
{
    if (n == 0)
        return 0;
    if (A == NULL || H == NULL || elem_bytes == 0)
        return -1;
    for (uint64_t i = 0; i < n; i++)
        if (H[i] > i)
            return -1;
    unsigned char *tmp = (unsigned char *)malloc(elem_bytes);
    if (tmp == NULL)
        return -1;
    for (uint64_t i = n; i-- > 0;)
        swap_records((unsigned char *)A, i, H[i], elem_bytes, tmp);
    free(tmp);
    return 0;
}

/* Same loop with the targets drawn from the seed as it goes. */
int oracle_knuth_shuffle_seed(void *A, uint64_t n, uint32_t elem_bytes,
                              uint64_t seed)
{
    if (n == 0)
        return 0;
    if (A == NULL || elem_bytes == 0)
        return -1;
    unsigned char *tmp = (unsigned char *)malloc(elem_bytes);
    if (tmp == NULL)
        return -1;
    for (uint64_t i = n; i-- > 0;)
        swap_records((unsigned char *)A, i, oracle_seed_target(seed, i),
                     elem_bytes, tmp);
    free(tmp);
    return 0;
}

/*
 * Sampled form of the same result, for arrays too large to shuffle on the
 * host: for each requested output position p, the index q such that the
 * shuffled array holds at p the record that was at q before the shuffle.
 *
 * Derivation from the loop above.  Step p (the swap of iteration p) moves
 * into position p the record that sits at position H[p] just before step p,
 * and p is never touched again (every later step j < p has H[j] <= j < p).
 * Walking back in time from step p, the record at position c (c <= p) last
 * moved at the earliest-executed step j > p that touched c; since j > c such
 * a step has H[j] = c, and it brought the record from position j.  Steps
 * execute in decreasing j, so scanning j = p+1, p+2, ... upward visits them
 * newest-first and the first hit is the right one; after the hit the record
 * came from j, and any step touching j must itself come later in the scan.
 * When the scan ends, the record never moved again and q = c.
 *
 * One upward scan of H serves all samples: a sample becomes active at
 * j = p, and at every j the active samples whose current c equals H[j]
 * move to c = j.  Active samples track distinct records at the same moment,
 * so their c values are distinct and a small hash map c -> sample suffices.
 * Cost: one pass over j (n target draws) plus O(1) expected per step.
 * Returns 0, or -1 on bad arguments (a position >= n, H[j] > j) or no memory.
 */
struct smap {
    uint64_t *key; /* current position c of an active sample, or EMPTY */
    uint64_t *val; /* sample index */
    uint64_t mask;
};
#define SMAP_EMPTY UINT64_MAX

static uint64_t smap_slot(const struct smap *m, uint64_t c)
{
    uint64_t h = oracle_splitmix64(c) & m->mask;
    while (m->key[h] != SMAP_EMPTY && m->key[h] != c)
        h = (h + 1) & m->mask;
    return h;
}

/* Remove the entry in slot h and re-seat the rest of its probe run. */
static void smap_erase(struct smap *m, uint64_t h)
{
    m->key[h] = SMAP_EMPTY;
    uint64_t j = (h + 1) & m->mask;
    while (m->key[j] != SMAP_EMPTY) {
        uint64_t k = m->key[j], v = m->val[j];
        m->key[j] = SMAP_EMPTY;
        uint64_t t = smap_slot(m, k);
        m->key[t] = k;
        m->val[t] = v;
        j = (j + 1) & m->mask;
    }
}

static int sample_impl(uint64_t n, const uint64_t *H, uint64_t seed,
                       const uint64_t *pos, uint64_t count, uint64_t *src)
{
    if (count == 0)
        return 0;
    for (uint64_t s = 0; s < count; s++)
        if (pos[s] >= n)
            return -1;
    /* order[] lists sample indices by increasing position (insertion sort on
     * a copy is enough for the few samples the callers ask for). */
    uint64_t *order = (uint64_t *)malloc(count * sizeof(uint64_t));
    uint64_t cap = 4;
    while (cap < 2 * count)
        cap <<= 1;
    struct smap m;
    m.key = (uint64_t *)malloc(cap * sizeof(uint64_t));
    m.val = (uint64_t *)malloc(cap * sizeof(uint64_t));
    m.mask = cap - 1;
    int rc = -1;
    if (order == NULL || m.key == NULL || m.val == NULL)
        goto out;
    for (uint64_t s = 0; s < count; s++) {
        uint64_t t = s;
        while (t > 0 && pos[order[t - 1]] > pos[s]) {
            order[t] = order[t - 1];
            t--;
        }
        order[t] = s;
    }
    for (uint64_t h = 0; h < cap; h++)
        m.key[h] = SMAP_EMPTY;

    uint64_t next = 0; /* next sample (in order[]) to activate */
    for (uint64_t j = pos[order[0]]; j < n; j++) {
        uint64_t h = H ? H[j] : oracle_seed_target(seed, j);
        if (h > j)
            goto out;
        /* Step j: an active sample whose record sits at h came from j. */
        uint64_t slot = smap_slot(&m, h);
        if (m.key[slot] == h) {
            uint64_t s = m.val[slot];
            smap_erase(&m, slot);
            uint64_t t = smap_slot(&m, j);
            m.key[t] = j;
            m.val[t] = s;
        }
        /* Samples whose position is j start here, holding position H[j].
         * Duplicated positions get the same answer. */
        while (next < count && pos[order[next]] == j) {
            uint64_t s = order[next++];
            if (next >= 2 && pos[order[next - 2]] == j) {
                src[s] = UINT64_MAX; /* filled from its twin below */
                continue;
            }
            uint64_t t = smap_slot(&m, h);
            m.key[t] = h;
            m.val[t] = s;
        }
    }
    /* Whatever is still active never moved again. */
    for (uint64_t t = 0; t < cap; t++)
        if (m.key[t] != SMAP_EMPTY)
            src[m.val[t]] = m.key[t];
    for (uint64_t i = 1; i < count; i++)
        if (pos[order[i]] == pos[order[i - 1]])
            src[order[i]] = src[order[i - 1]];
    rc = 0;
out:
    free(order);
    free(m.key);
    free(m.val);
    return rc;
}

int oracle_sample_sources(uint64_t n, const uint64_t *H, const uint64_t *pos,
                          uint64_t count, uint64_t *src)
{
    if (H == NULL)
        return -1;
    return sample_impl(n, H, 0, pos, count, src);
}

int oracle_sample_sources_seed(uint64_t n, uint64_t seed, const uint64_t *pos,
                               uint64_t count, uint64_t *src)
{
    return sample_impl(n, NULL, seed, pos, count, src);
}
