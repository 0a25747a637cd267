/*
 * list_oracle.c -- CPU oracle for list ranking and the in-place list
 * contraction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file: only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP library; it has its own SplitMix64.
 *
 * Lists: n elements with prev[i] and next[i] (0-based indices, NIL =
 * 0xFFFFFFFF at the ends); any number of disjoint lists.  A head has
 * prev = NIL.
 *
 * oracle_list_rank -- the definition of list ranking (Section 4.2: the
 * position of each element in its list): walk every list from its head,
 * counting.  No tolerance; integers only.
 *
 * oracle_list_contract -- the relaxed-PIP list contraction of Section 4.2,
 * step by step: Algorithm 2 (the parallel list contraction of Shun et al.:
 * every uncontracted element whose priority is below both neighbours'
 * priorities is spliced out, the leftover elements are packed, repeat) is
 * applied to one block of k elements at a time, the blocks taken in index
 * order (elements [jk, (j+1)k) form block j), until every block is
 * contracted.  List heads are never spliced: they carry the ranks' origin.
 * Inside block j the elements of later blocks, the heads and the NIL ends
 * count as having higher priority, which is the same as comparing the key
 * (block, priority, index) with heads and NIL above every key.  Each splice
 * of element i between its current neighbours L and R records
 *   left[i] = L, right[i] = R, round[i] = the round of its block,
 *   offset[i] = the distance from L to i in the original list,
 * where every element keeps w = the distance to its current successor (1 at
 * the start) and a splice adds w(i) to w(L) (the weight bookkeeping of list
 * ranking by contraction).  These per-element records are the contraction
 * tree that Section 4.2 stores over the input's pointers.
 *
 * Priorities: prio[i] when a priority array is given, else
 * splitmix64(seed XOR i) (SplitMix64 as published by Steele, Lea and Flood,
 * OOPSLA 2014, in the form of Vigna's public-domain reference).
 *
 * Parity: pinned by the tests -- ranks by brute-force list walks and
 * permutations, the contraction against the nearest-higher-key neighbours
 * (an independent stack computation), the ranks rebuilt from the
 * contraction records, and round counts of closed-form cases.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NIL 0xFFFFFFFFu

static uint64_t sm64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* 0 on success; -1 if the links are inconsistent or an element is not
 * reached from a head (a cycle). */
int oracle_list_rank(const uint32_t *prev, const uint32_t *next, uint64_t n, uint64_t *rank)
{
    uint64_t seen = 0;
    for (uint64_t i = 0; i < n; i++)
        rank[i] = UINT64_MAX;
    for (uint64_t h = 0; h < n; h++) {
        if (prev[h] != NIL)
            continue;
        uint64_t r = 0;
        uint64_t x = h;
        for (;;) {
            if (rank[x] != UINT64_MAX)
                return -1;
            rank[x] = r++;
            seen++;
            const uint32_t y = next[x];
            if (y == NIL)
                break;
            if (y >= n || prev[y] != x)
                return -1;
            x = y;
        }
    }
    return seen == n ? 0 : -1;
}

/* Key order of Section 4.2's contraction inside block j: a < b. */
static int key_less(uint64_t a, uint64_t b, const uint64_t *pr, uint64_t k,
                    const unsigned char *head)
{
    /* NIL and heads are above every key */
    if (b == NIL || head[b])
        return a != NIL && !head[a];
    if (a == NIL || head[a])
        return 0;
    const uint64_t ba = a / k, bb = b / k;
    if (ba != bb)
        return ba < bb;
    if (pr[a] != pr[b])
        return pr[a] < pr[b];
    return a < b;
}

/* Returns 0, or -1 if a block cannot be finished (no element of it is below
 * both neighbours: only possible for a malformed list).  *n_rounds receives
 * the total number of rounds over all blocks. */
int oracle_list_contract(const uint32_t *prev, const uint32_t *next, const uint64_t *prio,
                         uint64_t seed, uint64_t n, uint64_t k, uint32_t *left,
                         uint32_t *right, uint64_t *offset, uint32_t *round,
                         uint64_t *n_rounds)
{
    uint32_t *P = malloc(n * sizeof *P), *N = malloc(n * sizeof *N);
    uint64_t *w = malloc(n * sizeof *w), *pr = malloc(n * sizeof *pr);
    unsigned char *head = malloc(n), *alive = malloc(n), *go = malloc(n);
    uint64_t *members = malloc((k ? k : 1) * sizeof *members);
    int rc = 0;
    uint64_t total = 0;
    if (!P || !N || !w || !pr || !head || !alive || !go || !members || k == 0) {
        rc = -1;
        goto out;
    }
    for (uint64_t i = 0; i < n; i++) {
        P[i] = prev[i];
        N[i] = next[i];
        w[i] = 1;
        pr[i] = prio ? prio[i] : sm64(seed ^ i);
        head[i] = prev[i] == NIL;
        alive[i] = !head[i];
        left[i] = NIL;
        right[i] = NIL;
        offset[i] = 0;
        round[i] = 0;
    }
    for (uint64_t b0 = 0; b0 < n; b0 += k) {
        const uint64_t b1 = b0 + k < n ? b0 + k : n;
        uint64_t m = 0;
        for (uint64_t i = b0; i < b1; i++)
            if (alive[i])
                members[m++] = i;
        for (uint32_t r = 0; m > 0; r++) {
            /* which members are below both current neighbours */
            uint64_t nsplice = 0;
            for (uint64_t t = 0; t < m; t++) {
                const uint64_t i = members[t];
                go[i] = key_less(i, P[i], pr, k, head) && key_less(i, N[i], pr, k, head);
                nsplice += go[i];
            }
            if (nsplice == 0) {
                rc = -1;
                goto out;
            }
            /* splice them out together (no two are adjacent) */
            for (uint64_t t = 0; t < m; t++) {
                const uint64_t i = members[t];
                if (!go[i])
                    continue;
                const uint32_t L = P[i], R = N[i];
                left[i] = L;
                right[i] = R;
                offset[i] = w[L];
                round[i] = r;
                w[L] += w[i];
                N[L] = R;
                if (R != NIL)
                    P[R] = L;
                alive[i] = 0;
            }
            /* pack the leftover elements */
            uint64_t m2 = 0;
            for (uint64_t t = 0; t < m; t++)
                if (alive[members[t]])
                    members[m2++] = members[t];
            m = m2;
            total++;
        }
    }
out:
    if (n_rounds)
        *n_rounds = total;
    free(P);
    free(N);
    free(w);
    free(pr);
    free(head);
    free(alive);
    free(go);
    free(members);
    return rc;
}
