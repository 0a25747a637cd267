// A host-thread model of the resident serving kernel's claim and gang
// protocol (rp_resident_kernel in rp.hip: res_next, res_gang_wait and the
// gang's start, run and report), for checking its logic on the CPU under
// many interleavings.  Each worker thread plays one workgroup; a host thread
// posts ring entries (one workgroup, or a gang of `need`), reads completions,
// posts a request again for one workgroup when its gang could not form, and
// finally sets the stop word.  Random yields and sleeps between the steps
// widen the interleavings.
//
// Checked: every request runs exactly once; a gang runs with exactly `need`
// distinct members, ranks 0..need-1; a request handed back by its leader did
// not run; no worker waits forever (every wait is bounded, as on the device);
// the workers all leave after the stop word.  Prints "ok" and exits 0, or
// prints the first violation and exits 1.
//
// usage: resident_model <seed> <workers> <requests> <ring> <max_need> <form_us>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

uint32_t g_ring = 64;
uint64_t g_form_us = 2000;
const uint64_t IDLE_US = 5000000;     // the kernel's own idle exit (never reached here)
const uint64_t DEADLINE_S = 60;       // the whole model must finish within this

enum { EXIT = 0, SINGLE = 1, LEAD = 2, JOIN = 3 };
constexpr int32_t ST_OK = 0, ST_PENDING = 1;

struct Entry {                         // host memory
    std::atomic<uint64_t> seq{0};
    uint32_t need = 1;
    uint64_t req = 0;                  // which request it carries
};
struct Result {                        // host memory
    std::atomic<uint64_t> done{0};
    std::atomic<int32_t> status{0};
};
struct Ctl {                           // device memory
    std::atomic<uint64_t> head{0}, avail{0}, gang{0};
    std::atomic<uint32_t> poll_owner{0}, gang_left{0}, exitf{0};
    std::vector<std::atomic<uint32_t>> need;
    explicit Ctl(uint32_t ring) : need(ring) {}
};

std::vector<Entry> *g_entries;
std::vector<Result> *g_results;
Ctl *g_ctl;
std::atomic<uint32_t> g_stop{0};

// what the checks look at
std::mutex g_mu;
std::vector<int> g_runs;                          // by request: times it ran
std::vector<std::set<uint32_t>> g_members;        // by entry: member ranks that started
std::atomic<int> g_fail{0};

void fail(const char *what, uint64_t a, uint64_t b)
{
    if (g_fail.exchange(1) == 0)
        std::printf("violation: %s (%llu, %llu)\n", what, (unsigned long long)a,
                    (unsigned long long)b);
}

uint64_t us_since(Clock::time_point t0)
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::microseconds>(Clock::now() - t0)
        .count();
}

void jitter(std::mt19937_64 &rng)
{
    const uint32_t r = (uint32_t)(rng() % 16);
    if (r < 10)
        return;
    if (r < 14)
        std::this_thread::yield();
    else
        std::this_thread::sleep_for(std::chrono::microseconds(rng() % 50));
}

bool cas(std::atomic<uint64_t> &a, uint64_t expect, uint64_t v)
{
    return a.compare_exchange_strong(expect, v);
}

// res_next: what this worker does next.
int next(std::mt19937_64 &rng, uint64_t *entry, uint32_t *rank)
{
    Ctl &c = *g_ctl;
    const uint32_t mask = g_ring - 1;
    auto t_last = Clock::now();
    for (;;) {
        jitter(rng);
        const uint64_t W = c.gang.load();
        if (W != 0) {
            const uint32_t joined = (uint32_t)W & 0xFFFu;
            const uint32_t need = (uint32_t)(W >> 12) & 0xFFFu;
            if (joined != 0 && joined < need) {
                if (cas(c.gang, W, W + 1)) {
                    *entry = (W >> 24) - 1;
                    *rank = joined;
                    return JOIN;
                }
                continue;
            }
            if (us_since(t_last) > IDLE_US) {
                c.exitf.store(1);
                return EXIT;
            }
            std::this_thread::yield();
            continue;
        }
        if (c.exitf.load() != 0)
            return EXIT;
        const uint64_t h = c.head.load();
        const uint64_t a = c.avail.load();
        if (h < a) {
            const uint32_t nd = c.need[h & mask].load();
            jitter(rng);
            if (nd <= 1) {
                if (cas(c.head, h, h + 1)) {
                    *entry = h;
                    *rank = 0;
                    return SINGLE;
                }
                continue;
            }
            const uint64_t Wl = ((h + 1) << 24) | ((uint64_t)nd << 12);
            if (cas(c.gang, 0, Wl)) {
                jitter(rng);
                if (cas(c.head, h, h + 1)) {
                    *entry = h;
                    *rank = 0;
                    return LEAD;
                }
                c.gang.exchange(0);   // h was stale; nobody joined a locked gang
            }
            continue;
        }
        if (c.poll_owner.load() == 0 && c.poll_owner.exchange(1) == 0) {
            uint64_t aa = a;
            while (aa - h < g_ring) {
                Entry &e = (*g_entries)[aa & mask];
                if (e.seq.load() != aa + 1)
                    break;
                c.need[aa & mask].store(e.need);
                aa++;
            }
            if (aa > a) {
                uint64_t cur = c.avail.load();
                while (cur < aa && !c.avail.compare_exchange_weak(cur, aa)) {
                }
            }
            const bool stop = g_stop.load() != 0;
            if (stop)
                c.exitf.store(1);
            c.poll_owner.exchange(0);
            if (aa > a) {
                t_last = Clock::now();
                continue;
            }
            if (stop)
                return EXIT;
        }
        if (us_since(t_last) > IDLE_US) {
            c.exitf.store(1);
            return EXIT;
        }
        std::this_thread::yield();
    }
}

// res_gang_wait
bool gang_wait(std::mt19937_64 &rng, uint64_t e, uint32_t need, bool leader)
{
    Ctl &c = *g_ctl;
    const uint64_t id = ((e + 1) << 12) | need;
    const auto t0 = Clock::now();
    for (;;) {
        jitter(rng);
        const uint64_t W = c.gang.load();
        if ((W >> 12) != id)
            return false;
        if ((uint32_t)(W & 0xFFFu) == need) {
            if (c.gang_left.fetch_add(1) + 1 == need) {
                c.gang_left.exchange(0);
                c.gang.exchange(0);
            }
            return true;
        }
        if (leader && us_since(t0) > g_form_us && cas(c.gang, W, 0))
            return false;
        std::this_thread::yield();
    }
}

void publish(uint64_t entry, int32_t status)
{
    Result &r = (*g_results)[entry & (g_ring - 1)];
    r.status.store(status);
    r.done.store(entry + 1);
}

void worker(uint64_t seed)
{
    std::mt19937_64 rng(seed);
    const uint32_t mask = g_ring - 1;
    for (;;) {
        uint64_t e = 0;
        uint32_t rank = 0;
        const int cmd = next(rng, &e, &rank);
        if (cmd == EXIT)
            return;
        const Entry &en = (*g_entries)[e & mask];
        if (en.seq.load() != e + 1)
            fail("claimed an entry that is not posted", e, en.seq.load());
        const uint64_t req = en.req;
        if (cmd == SINGLE) {
            {
                std::lock_guard<std::mutex> lk(g_mu);
                g_runs[req]++;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
            publish(e, ST_OK);
            continue;
        }
        const uint32_t G = en.need;
        if (cmd == LEAD) {
            jitter(rng);
            g_ctl->gang.exchange(((e + 1) << 24) | ((uint64_t)G << 12) | 1u);
        }
        const bool go = gang_wait(rng, e, G, cmd == LEAD);
        if (!go) {
            if (cmd == LEAD)
                publish(e, ST_PENDING);
            continue;
        }
        // the gang's run: every member starts, a bounded barrier, the leader
        // records the run and reports
        {
            std::lock_guard<std::mutex> lk(g_mu);
            if (!g_members[e].insert(rank).second)
                fail("two members with one rank", e, rank);
            if (rank >= G)
                fail("rank beyond the gang", e, rank);
        }
        bool all = false;
        const auto t0 = Clock::now();
        while (!all) {
            {
                std::lock_guard<std::mutex> lk(g_mu);
                all = g_members[e].size() == G;
            }
            if (us_since(t0) > 5000000) {
                fail("a gang member never started", e, rank);
                return;
            }
            std::this_thread::yield();
        }
        std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
        if (rank == 0) {
            {
                std::lock_guard<std::mutex> lk(g_mu);
                g_runs[req]++;
            }
            publish(e, ST_OK);
        }
    }
}

}  // namespace

int main(int argc, char **argv)
{
    if (argc < 7) {
        std::fprintf(stderr, "usage: %s seed workers requests ring max_need form_us\n", argv[0]);
        return 2;
    }
    const uint64_t seed = std::strtoull(argv[1], nullptr, 10);
    const uint32_t workers = (uint32_t)std::atoi(argv[2]);
    const uint32_t nreq = (uint32_t)std::atoi(argv[3]);
    g_ring = (uint32_t)std::atoi(argv[4]);
    const uint32_t max_need = (uint32_t)std::atoi(argv[5]);
    g_form_us = (uint64_t)std::atoll(argv[6]);
    if ((g_ring & (g_ring - 1)) != 0 || max_need > workers) {
        std::fprintf(stderr, "ring must be a power of two and max_need <= workers\n");
        return 2;
    }
    std::mt19937_64 rng(seed);
    std::vector<Entry> entries(g_ring);
    std::vector<Result> results(g_ring);
    Ctl ctl(g_ring);
    g_entries = &entries;
    g_results = &results;
    g_ctl = &ctl;
    g_runs.assign(nreq, 0);
    g_members.resize((size_t)nreq * 4 + g_ring);

    std::vector<std::thread> th;
    for (uint32_t w = 0; w < workers; w++)
        th.emplace_back(worker, seed * 1000 + w);

    // the host: post requests in order, reap, post a handed-back gang again
    // for one workgroup
    const auto t_start = Clock::now();
    std::vector<uint64_t> slot_entry(g_ring, UINT64_MAX);   // entry in each slot
    std::vector<uint64_t> todo;                             // requests to post, in order
    std::vector<uint32_t> want(nreq);
    for (uint32_t r = 0; r < nreq; r++) {
        todo.push_back(r);
        want[r] = (rng() % 3 == 0) ? 1 + (uint32_t)(rng() % max_need) : 1;
    }
    uint64_t posted = 0, next_todo = 0, finished = 0, handed_back = 0;
    std::vector<char> single(nreq, 0);
    while (finished < nreq && !g_fail.load()) {
        if (us_since(t_start) > DEADLINE_S * 1000000) {
            fail("the model did not finish", finished, nreq);
            break;
        }
        // reap
        for (uint32_t s = 0; s < g_ring; s++) {
            const uint64_t e = slot_entry[s];
            if (e == UINT64_MAX || results[s].done.load() != e + 1)
                continue;
            const uint64_t req = entries[s].req;
            slot_entry[s] = UINT64_MAX;
            if (results[s].status.load() == ST_PENDING) {
                std::lock_guard<std::mutex> lk(g_mu);
                if (g_runs[req] != 0)
                    fail("a handed-back request had run", req, g_runs[req]);
                single[req] = 1;
                todo.push_back(req);
                handed_back++;
            } else {
                finished++;
            }
        }
        // post, in order, while the next slot is free
        while (next_todo < todo.size()) {
            const uint32_t s = (uint32_t)(posted & (g_ring - 1));
            if (slot_entry[s] != UINT64_MAX)
                break;
            const uint64_t req = todo[next_todo++];
            entries[s].need = single[req] ? 1 : want[req];
            entries[s].req = req;
            entries[s].seq.store(posted + 1);
            slot_entry[s] = posted;
            posted++;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(rng() % 100));
    }
    g_stop.store(1);
    for (auto &t : th)
        t.join();
    if (!g_fail.load()) {
        for (uint32_t r = 0; r < nreq; r++)
            if (g_runs[r] != 1) {
                fail("a request did not run exactly once", r, g_runs[r]);
                break;
            }
    }
    if (g_fail.load())
        return 1;
    std::printf("ok: %u requests, %llu entries posted, %llu gangs handed back\n", nreq,
                (unsigned long long)posted, (unsigned long long)handed_back);
    return 0;
}
