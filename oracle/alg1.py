"""Round structure of the parallel Knuth shuffle -- TEST INFRASTRUCTURE ONLY.

A plain, sequential simulation of the paper's Algorithm 1 (Section 4.1,
"Parallel Knuth-Shuffle", deterministic reservations) for small inputs, in the
paper's notation but 0-based (H[i] in [0, i], swaps taken from i = n-1 down).

* Every unfinished swap (s, H[s]) writes R[s] <- max(R[s], s) and
  R[H[s]] <- max(R[H[s]], s); then every unfinished swap with R[s] = s and
  R[H[s]] = s swaps A[s] and A[H[s]]; the rest are kept for the next round and
  R is reset.  "max" is the priority write: the larger index is earlier in the
  sequential order and wins.
* ``prefix`` limits each round to the first ``prefix`` unfinished swaps in the
  sequential order (the relaxed-PIP form of Section 4.1, which always works on
  the first n^(1-eps) unfinished swaps; the deterministic-reservations
  framework of Section 7.3 / Appendix A.1 refills the prefix after every
  round).  ``prefix=None`` takes all unfinished swaps each round.
* ``rule="alg1"`` is the two-reservation test of Algorithm 1.
  ``rule="oneres"`` is the single-reservation test of Appendix A.2 (RP-OneRes,
  also used by RP-Final): only R[H[s]] is written, and s commits iff
  (R[s] is unset or R[s] = s) and R[H[s]] = s.

The per-round sets are what the paper's worked example (Section 4.1, the
figure for H = [1, 1, 2, 4, 2, 3, 4, 2]) describes; the final array must equal
the sequential loop in ``knuth_oracle.c``.
"""
from __future__ import annotations


def parallel_knuth_rounds(A, H, prefix=None, rule="alg1"):
    """Return (final A as a list, list of per-round committed swaps).

    Each round's entry is the sorted list of (s, H[s]) pairs that committed.
    Plain Python; meant for n up to a few thousand.
    """
    n = len(A)
    A = list(A)
    H = [int(h) for h in H]
    for i, h in enumerate(H):
        if not 0 <= h <= i:
            raise ValueError("H[i] must lie in [0, i]")
    if rule not in ("alg1", "oneres"):
        raise ValueError("rule must be 'alg1' or 'oneres'")
    unfinished = list(range(n - 1, -1, -1))  # sequential order: n-1 first
    rounds = []
    while unfinished:
        take = len(unfinished) if prefix is None else min(prefix, len(unfinished))
        active = unfinished[:take]
        R = {}  # reservation array restricted to the touched keys; unset = bottom
        for s in active:  # reserve phase
            if rule == "alg1":
                R[s] = max(R.get(s, -1), s)
            R[H[s]] = max(R.get(H[s], -1), s)
        won = []
        for s in active:  # commit test, all against the same R
            if rule == "alg1":
                ok = R.get(s) == s and R.get(H[s]) == s
            else:
                ok = R.get(s, -1) in (-1, s) and R.get(H[s]) == s
            if ok:
                won.append(s)
        for s in won:  # commit phase: winners touch disjoint locations
            A[s], A[H[s]] = A[H[s]], A[s]
        wonset = set(won)
        unfinished = [s for s in unfinished if s not in wonset]
        rounds.append(sorted((s, H[s]) for s in won))
    return A, rounds
