// A host-thread model of the one-barrier rounds of the shuffle
// (rounds1_body in rp.hip), for checking the protocol on the CPU under many
// interleavings.  Each thread plays one workgroup of L lanes; between two
// barriers it checks and commits round r and refills and reserves round r+1,
// with nothing to keep a fast workgroup's reservations of round r+1 from
// landing before a slow workgroup's checks of round r:
//   * reservations: atomic max of (round tag | rank) into a hashed slot of a
//     T-slot table per target key, rank = source - the round's cursor; the
//     table is reset between two extra barriers every `tag_cycle` rounds;
//   * dense window: one bit per key over [cursor, cursor + W), three
//     parities: round r+1 sets parity (r+1) mod 3 and clears (r+2) mod 3;
//   * decision: the target's slot still holds exactly the swap's priority,
//     and no active swap targets the source (its window bit, or the slot of
//     the source key not above the swap's priority); the top active swap
//     (its rank gathered at the barrier) commits regardless;
//   * refill by quota: every workgroup derives the same quota from the
//     gathered counts; workgroup w takes the fresh indices cursor-1-o for
//     the o dealt to it in chunks, round robin;
//   * records: read with the check loads (early) or by the winners after
//     the decision (late), written back swapped after the reservations.
// An adversarial schedule holds workgroup 0's checks of a round back until
// every other workgroup has reserved the next round and cleared its window
// parity; elsewhere random yields widen the interleavings.  Memory
// operations are sequentially consistent std::atomic accesses: this checks
// the protocol's logic, not the device's memory ordering.
//
// Checked: the output equals the sequential Knuth shuffle of the identity
// with the same targets (decreasing i, swap A[i] and A[H[i]]); every active
// rank stays within the rank limit (or the first refill's size, which is not
// throttled); the rounds end, within 2n + 64.  Prints "ok: ..." and
// exits 0, or prints the first violation and exits 1.
//
// usage: rounds1_model <seed> <n> <workgroups> <lanes> <k> <table_slots>
//                      <chunk_log2> <tag_cycle> <rank_cap> <early> <adversarial>
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

namespace {

constexpr uint32_t EMPTY = 0xFFFFFFFFu;
constexpr uint32_t RANKB = 24;          // priority = tag:8 | rank:24
constexpr uint32_t RANKMAX = (1u << RANKB) - 1u;
constexpr uint32_t PAR = 3;             // window parities

struct Cfg {
    uint64_t seed = 1;
    uint32_t n = 0, G = 1, L = 64, k = 1, T = 1, cl = 0, tag_cycle = 256, rank_cap = RANKMAX;
    bool early = false, adversarial = false;
    uint32_t bmw = 1, W = 32;
};

Cfg C;
std::vector<uint32_t> H;                         // targets
std::vector<std::atomic<uint32_t>> *slots, *bm;  // table, window (PAR * bmw words)
std::vector<std::atomic<uint64_t>> *A;           // the records
std::atomic<int> g_fail{0};

// gather barrier: payload per workgroup, double-buffered by epoch parity
struct Pay {
    uint32_t act = 0, won = 0, age = 0;
};
std::vector<Pay> *g_pay[2];
std::vector<std::atomic<uint64_t>> *g_arrived;   // last epoch each workgroup reached
std::atomic<uint64_t> g_reserved{0};             // reservation steps done, all workgroups
std::atomic<uint64_t> g_rounds{0}, g_attempts{0}, g_retries{0}, g_throttled{0}, g_maxact{0};

void fail(const char *what, uint64_t a, uint64_t b)
{
    if (g_fail.exchange(1) == 0)
        std::printf("violation: %s (%llu, %llu)\n", what, (unsigned long long)a,
                    (unsigned long long)b);
}

uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint32_t slot_of(uint32_t key)
{
    return (uint32_t)((splitmix64(key) >> 11) % C.T);
}

void jitter(std::mt19937_64 &rng)
{
    const uint32_t r = (uint32_t)(rng() % 64);
    if (r < 6)
        std::this_thread::yield();
    else if (r == 6)
        std::this_thread::sleep_for(std::chrono::microseconds(rng() % 50));
}

// Publish this workgroup's payload for `epoch` and wait until every workgroup
// reached it; returns false if the model failed meanwhile.
bool barrier(uint32_t w, uint64_t epoch, const Pay &mine, Pay *sum, uint32_t *maxact)
{
    (*g_pay[epoch & 1])[w] = mine;
    (*g_arrived)[w].store(epoch);
    for (uint32_t i = 0; i < C.G; i++)
        while ((*g_arrived)[i].load() < epoch) {
            if (g_fail.load())
                return false;
            std::this_thread::yield();
        }
    Pay s;
    uint32_t mx = 0;
    for (uint32_t i = 0; i < C.G; i++) {
        const Pay &p = (*g_pay[epoch & 1])[i];
        s.act += p.act;
        s.won += p.won;
        s.age = std::max(s.age, p.age);
        mx = std::max(mx, p.act);
    }
    if (sum)
        *sum = s;
    if (maxact)
        *maxact = mx;
    return true;
}

uint32_t fresh_ord(uint32_t w, uint32_t j)
{
    return ((w + C.G * (j >> C.cl)) << C.cl) + (j & ((1u << C.cl) - 1u));
}

void workgroup(uint32_t w)
{
    std::mt19937_64 rng(C.seed * 7919 + w);
    const uint32_t G = C.G, L = C.L, W = C.W, bmw = C.bmw;
    std::vector<uint32_t> src(L, EMPTY), tgt(L, 0), t1(L), q1(L), sh_h(L);
    std::vector<uint64_t> rs(L), rh(L);
    std::vector<char> won(L);
    uint64_t epoch = 0, rr = 0, prevA = 0, g_act = 0, g_won = 0;
    uint32_t cursor = C.n, g_maxa = 0, g_age = 0, top = EMPTY;
    uint32_t q = std::min<uint32_t>((C.k + G - 1) / G, L);
    q = std::max(q >> C.cl, 1u) << C.cl;
    uint32_t take = (uint32_t)std::min<uint64_t>((uint64_t)G * q, C.n);
    const double rG = 1.0 / (double)G;
    // Every round with an active swap commits at least its top one; a round
    // can start with nothing active only after a refill of self-loops or a
    // quota of zero, and the next refill takes at least one index.  So the
    // rounds stay below 2n + 64 for any parameters (the kernel's plans, with
    // k in the hundreds or more, need about 2n/k).
    const uint64_t max_rounds = 2 * (uint64_t)C.n + 64;
    // The first refill is not throttled: ranks stay within the larger of the
    // rank limit and its size.
    const uint32_t rank_lim = std::max(C.rank_cap, take - 1u);

    for (;;) {
        const bool reset_now = rr > 0 && rr % C.tag_cycle == 0;
        // Adversarial: workgroup 0 checks only after every other workgroup
        // reserved the next round (not when the table reset's barriers come
        // first: they wait for workgroup 0).
        if (C.adversarial && w == 0 && rr > 0 && !reset_now && (splitmix64(rr ^ C.seed) & 1)) {
            const uint64_t want = rr + (uint64_t)(G - 1) * (rr + 1);
            while (g_reserved.load() < want) {
                if (g_fail.load())
                    return;
                std::this_thread::yield();
            }
        }
        // ---- check round rr-1: the loads the decision needs
        for (uint32_t l = 0; l < L; l++) {
            if (src[l] == EMPTY)
                continue;
            const uint32_t ds = src[l] - cursor;
            const uint32_t par = (uint32_t)((rr - 1) % PAR);
            t1[l] = (*slots)[slot_of(tgt[l])].load();
            jitter(rng);
            q1[l] = ds < W ? (*bm)[(uint64_t)par * bmw + (ds >> 5)].load()
                           : (*slots)[slot_of(src[l])].load();
            if (C.early) {
                rs[l] = (*A)[src[l]].load();
                rh[l] = (*A)[tgt[l]].load();
            }
            jitter(rng);
        }
        if (rr > 0) {
            // ---- quota (identical in every workgroup)
            top = g_act ? g_age : EMPTY;
            const uint32_t a32 = (uint32_t)g_act;
            const uint32_t expect_w =
                prevA ? (uint32_t)((double)g_act * (double)g_won / (double)prevA) : a32 / 2u;
            prevA = g_act;
            const uint32_t want = C.k + expect_w > a32 ? C.k + expect_w - a32 : 0u;
            const uint32_t Cc = 1u << C.cl;
            uint32_t qq = ((uint32_t)std::ceil((double)want * rG) + Cc / 2) / Cc * Cc;
            qq = std::min(qq, (L - g_maxa) / Cc * Cc);
            const uint32_t room =
                g_age < C.rank_cap ? (uint32_t)((double)(C.rank_cap - g_age) * rG) / Cc * Cc : 0u;
            if (qq > room) {
                qq = room;
                if (w == 0)
                    g_throttled++;
            }
            if (qq == 0 && g_act == 0 && cursor > 0)
                qq = Cc;
            q = qq;
            take = (uint32_t)std::min<uint64_t>((uint64_t)G * q, cursor);
        }
        for (uint32_t j = 0; j < q && j < L; j++) {
            const uint32_t o = fresh_ord(w, j);
            if (o < take)
                sh_h[j] = H[cursor - 1u - o];
        }
        // ---- decide
        uint32_t nwon = 0;
        for (uint32_t l = 0; l < L; l++) {
            won[l] = 0;
            if (src[l] == EMPTY)
                continue;
            const uint32_t ds = src[l] - cursor;
            const uint32_t tag = (uint32_t)((rr - 1) % C.tag_cycle);
            const uint32_t v = (tag << RANKB) | ds;
            bool win = t1[l] == v;
            if (ds < W)
                win = win && !((q1[l] >> (ds & 31u)) & 1u);
            else
                win = win && q1[l] <= v;
            win = win || ds == top;
            g_attempts++;
            if (win) {
                won[l] = 1;
                nwon++;
                if (!C.early) {
                    rs[l] = (*A)[src[l]].load();
                    rh[l] = (*A)[tgt[l]].load();
                }
            } else {
                g_retries++;
            }
        }
        // winners keep their source and target until they write; their lanes
        // are free for the refill
        std::vector<uint32_t> ws(src), wt(tgt);
        for (uint32_t l = 0; l < L; l++)
            if (won[l])
                src[l] = EMPTY;
        // ---- refill: the free lanes take the fresh indices in lane order
        uint32_t j = 0;
        for (uint32_t l = 0; l < L; l++) {
            if (src[l] != EMPTY)
                continue;
            const uint32_t oj = fresh_ord(w, j);
            if (j < q && oj < take) {
                const uint32_t s = cursor - 1u - oj;
                if (sh_h[j] != s) {
                    src[l] = s;
                    tgt[l] = sh_h[j];
                }
            }
            j++;
        }
        cursor -= take;
        const uint32_t tag = (uint32_t)(rr % C.tag_cycle);
        if (reset_now) {
            if (!barrier(w, ++epoch, Pay{}, nullptr, nullptr))
                return;
            for (uint32_t i = w; i < C.T; i += G)
                (*slots)[i].store(0);
            if (!barrier(w, ++epoch, Pay{}, nullptr, nullptr))
                return;
        }
        // ---- reserve round rr (and clear the parity two rounds ahead)
        {
            const uint32_t cp = (uint32_t)((rr + 1) % PAR);
            for (uint32_t i = w; i < bmw; i += G)
                (*bm)[(uint64_t)cp * bmw + i].store(0);
        }
        uint32_t act = 0, age = 0;
        for (uint32_t l = 0; l < L; l++) {
            if (src[l] == EMPTY)
                continue;
            const uint32_t rank = src[l] - cursor;
            if (rank > rank_lim)
                fail("rank beyond the limit", rank, rank_lim);
            const uint32_t v = (tag << RANKB) | rank;
            std::atomic<uint32_t> &sl = (*slots)[slot_of(tgt[l])];
            uint32_t cur = sl.load();
            while (cur < v && !sl.compare_exchange_weak(cur, v)) {
            }
            const uint32_t d = tgt[l] - cursor;
            if (tgt[l] >= cursor && d < W)
                (*bm)[(uint64_t)(rr % PAR) * bmw + (d >> 5)].fetch_or(1u << (d & 31u));
            act++;
            age = std::max(age, rank);
            jitter(rng);
        }
        g_reserved++;
        rr++;
        // ---- winners of the round just checked exchange their records
        for (uint32_t l = 0; l < L; l++) {
            if (!won[l])
                continue;
            (*A)[ws[l]].store(rh[l]);
            (*A)[wt[l]].store(rs[l]);
            jitter(rng);
        }
        // ---- barrier
        Pay s;
        if (!barrier(w, ++epoch, Pay{act, nwon, age}, &s, &g_maxa))
            return;
        g_act = s.act;
        g_won = s.won;
        g_age = s.age;
        if (w == 0)
            g_maxact.store(std::max<uint64_t>(g_maxact.load(), g_act));
        if (cursor == 0 && g_act == 0)
            break;
        if (rr > max_rounds) {
            fail("rounds beyond the limit", rr, max_rounds);
            return;
        }
    }
    if (w == 0)
        g_rounds.store(rr > 0 ? rr - 1 : 0);
}

}  // namespace

int main(int argc, char **argv)
{
    if (argc != 12) {
        std::fprintf(stderr,
                     "usage: rounds1_model seed n workgroups lanes k table_slots chunk_log2 "
                     "tag_cycle rank_cap early adversarial\n");
        return 2;
    }
    C.seed = std::strtoull(argv[1], nullptr, 10);
    C.n = (uint32_t)std::strtoul(argv[2], nullptr, 10);
    C.G = (uint32_t)std::strtoul(argv[3], nullptr, 10);
    C.L = (uint32_t)std::strtoul(argv[4], nullptr, 10);
    C.k = (uint32_t)std::strtoul(argv[5], nullptr, 10);
    C.T = (uint32_t)std::strtoul(argv[6], nullptr, 10);
    C.cl = (uint32_t)std::strtoul(argv[7], nullptr, 10);
    C.tag_cycle = (uint32_t)std::strtoul(argv[8], nullptr, 10);
    C.rank_cap = (uint32_t)std::strtoul(argv[9], nullptr, 10);
    C.early = std::atoi(argv[10]) != 0;
    C.adversarial = std::atoi(argv[11]) != 0;
    if (C.n < 2 || C.G < 1 || C.L < 2 || C.k < 1 || C.T < 1 || C.tag_cycle < 2 ||
        C.tag_cycle > 256 || C.rank_cap < 1 || C.rank_cap > RANKMAX || (C.L >> C.cl) == 0) {
        std::fprintf(stderr, "bad arguments\n");
        return 2;
    }
    C.bmw = std::max<uint32_t>(1, (uint32_t)std::ceil(1.5 * (double)C.k / 32.0));
    C.W = C.bmw * 32;

    H.resize(C.n);
    for (uint32_t i = 0; i < C.n; i++)
        H[i] = (uint32_t)(splitmix64(C.seed ^ ((uint64_t)i << 20)) % ((uint64_t)i + 1));
    std::vector<std::atomic<uint32_t>> slots_v(C.T), bm_v((size_t)PAR * C.bmw);
    std::vector<std::atomic<uint64_t>> A_v(C.n);
    for (uint32_t i = 0; i < C.n; i++)
        A_v[i].store(i);
    std::vector<Pay> p0(C.G), p1(C.G);
    std::vector<std::atomic<uint64_t>> arrived(C.G);
    slots = &slots_v;
    bm = &bm_v;
    A = &A_v;
    g_pay[0] = &p0;
    g_pay[1] = &p1;
    g_arrived = &arrived;

    std::vector<std::thread> th;
    for (uint32_t w = 0; w < C.G; w++)
        th.emplace_back(workgroup, w);
    for (auto &t : th)
        t.join();
    if (g_fail.load())
        return 1;

    // the sequential Knuth shuffle of the identity with the same targets
    std::vector<uint64_t> want(C.n);
    for (uint32_t i = 0; i < C.n; i++)
        want[i] = i;
    for (uint32_t i = C.n; i-- > 0;)
        std::swap(want[i], want[H[i]]);
    for (uint32_t i = 0; i < C.n; i++)
        if (A_v[i].load() != want[i]) {
            fail("output differs from the sequential shuffle at", i, A_v[i].load());
            return 1;
        }
    std::printf("ok: %llu rounds, %llu attempts, %llu retries, %llu throttled, max active %llu\n",
                (unsigned long long)g_rounds.load(), (unsigned long long)g_attempts.load(),
                (unsigned long long)g_retries.load(), (unsigned long long)g_throttled.load(),
                (unsigned long long)g_maxact.load());
    return 0;
}
