// Serving form of librp: a request loop on one device.
//
// A server owns one device arena of a fixed budget (the in-place theme of the
// paper -- Section 1, Section 7.6 -- applied to a stream of requests: memory,
// not compute, decides how many requests can be in the system).  Requests are
// admitted strictly in arrival order while their arrays fit in the arena's
// free space, filled on the device, and run:
//   * batched mode: every admitted request of a size class goes out in the
//     next batched launch (rp_batch_submit) on a free stream of that class;
//     launches on different streams overlap on the device, and inside a launch
//     each request owns a workgroup or a wave, so a request that arrives while
//     others run starts as soon as a stream is free and finishes on its own
//     completion flag, not with its launch.  Large requests (n >= 2^large_log2)
//     have their own streams so that small ones never queue behind them;
//   * resident mode: one kernel stays on the device while there is work and
//     takes each admitted request from a ring in host memory as it arrives
//     (rp_resident.h): a small request starts on the next free workgroup, a
//     large one on a gang of idle workgroups, without waiting for a launch;
//   * plain mode: one rp_shuffle_inplace per request, in admission order, on
//     one stream (the per-request path the batched mode is measured against).
// One dispatcher thread does all device work; the C entry points only exchange
// bookkeeping with it under a mutex, so submit never waits for the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <cstddef>
#include <cstdlib>
#include <thread>
#include <vector>

#include "rp.h"
#include "rp_arena.h"
#include "rp_resident.h"

namespace rpint {
// rp.hip: workgroups rp_shuffle_group gives one shuffle (0: not groupable).
int group_grid(uint64_t n, uint32_t elem_bytes, double eps, int device, uint64_t *grid);
}

namespace {

constexpr int N_SMALL_STREAMS = 2;
constexpr int N_LARGE_STREAMS = 2;
constexpr int N_STREAMS = N_SMALL_STREAMS + N_LARGE_STREAMS;
constexpr uint32_t PLAIN_AHEAD = 64;   // plain mode: requests enqueued ahead
constexpr size_t ALONE_QUEUE = 16;     // large_alone: batch beyond this many waiting
constexpr size_t GROUP_MAX = 16;       // shuffles one rp_shuffle_group call takes
// Resident mode: the kernel is stopped after this long without work (and
// launched again when work arrives); on its own it leaves after 30 s with
// nothing to claim; a gang that has not formed within 1 s is given back and
// its request runs on one workgroup instead.
constexpr uint64_t RES_IDLE_STOP_NS = 20000000;
constexpr uint64_t RES_IDLE_TICKS = 3000000000ull;   // 100 MHz ticks
constexpr uint64_t RES_FORM_TICKS = 100000000ull;

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ------------------------------------------------------------- fill kernel

struct FillDesc {
    unsigned char *A;
    uint64_t start;   // first element of this request in the flattened space
    uint64_t n;
    uint32_t eb;
    uint32_t pad;
};

// A[i] = i for every request of a launch.  The requests' elements form one
// flattened index space; each workgroup takes chunks of it and finds the
// request of a chunk by binary search over the start offsets.
constexpr uint32_t FILL_CHUNK = 4096;

__global__ __launch_bounds__(256) void rp_fill_identity_kernel(const FillDesc *d, uint32_t count,
                                                               uint64_t total)
{
    for (uint64_t c0 = (uint64_t)blockIdx.x * FILL_CHUNK; c0 < total;
         c0 += (uint64_t)gridDim.x * FILL_CHUNK) {
        uint32_t lo = 0, hi = count - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            if (d[mid].start <= c0)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint64_t c1 = min(c0 + FILL_CHUNK, total);
        uint32_t q = lo;
        uint64_t qend = d[q].start + d[q].n;
        for (uint64_t g = c0 + threadIdx.x; g < c1; g += blockDim.x) {
            while (g >= qend) {
                q++;
                qend = d[q].start + d[q].n;
            }
            const FillDesc f = d[q];
            const uint64_t i = g - f.start;
            if (f.eb == 4) {
                reinterpret_cast<uint32_t *>(f.A)[i] = (uint32_t)i;
            } else if (f.eb == 8) {
                reinterpret_cast<uint64_t *>(f.A)[i] = i;
            } else {
                uint32_t *rec = reinterpret_cast<uint32_t *>(f.A + i * f.eb);
                rec[0] = (uint32_t)i;
                for (uint32_t w = 1; w < f.eb / 4; w++)
                    rec[w] = 0u;
            }
        }
    }
}

// One request, descriptor passed by value (no host buffer to keep alive).
__global__ __launch_bounds__(256) void rp_fill_identity_one_kernel(FillDesc f)
{
    const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f.n; i += nth) {
        if (f.eb == 4) {
            reinterpret_cast<uint32_t *>(f.A)[i] = (uint32_t)i;
        } else if (f.eb == 8) {
            reinterpret_cast<uint64_t *>(f.A)[i] = i;
        } else {
            uint32_t *rec = reinterpret_cast<uint32_t *>(f.A + i * f.eb);
            rec[0] = (uint32_t)i;
            for (uint32_t w = 1; w < f.eb / 4; w++)
                rec[w] = 0u;
        }
    }
}

// ------------------------------------------------------------------ server

struct Req {
    rp_server_request q{};
    int32_t state = RP_REQ_QUEUED;
    int32_t status = RP_OK;
    uint64_t t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
    uint64_t off = 0, bytes = 0;
    bool has_mem = false;
    uint64_t rounds = 0;
    uint32_t aux_words = 0;
    bool large = false;
    // resident mode
    bool gang_ok = false;       // n >= 2^large_log2: may run on a gang
    bool force_single = false;  // its gang could not form: one workgroup
    uint64_t entry = 0;         // ring entry while posted
    uint32_t gang = 1;
    uint64_t aux_off = 0, aux_bytes = 0;
    bool has_aux = false;
};

struct Resident {
    rpres::Entry *ring = nullptr;       // pinned host memory
    rpres::Result *res = nullptr;       // pinned host memory
    uint32_t *stop = nullptr;           // pinned host memory
    void *ctl = nullptr;                // device memory
    hipStream_t stream = nullptr;       // this server's own
    hipEvent_t ev = nullptr;            // recorded after each launch
    bool running = false;
    bool stop_sent = false;
    uint32_t grid = 0;
    uint64_t posted = 0;                // entries posted so far
    uint64_t floor = 0;                 // oldest posted entry not reaped yet (or posted)
    std::vector<uint64_t> slot_ticket;  // ticket in each ring slot (0: free)
    uint32_t busy_slots = 0;
    uint32_t wgs_out = 0;               // workgroups of the posted entries not done yet
    uint64_t idle_since = 0;
    uint64_t form_ticks = RES_FORM_TICKS;
    uint32_t gang_cap = 0;              // largest gang (0: a quarter of the grid)
};

struct Launch {
    int stream = 0;
    uint64_t batch_id = 0;              // batched mode
    std::vector<uint64_t> tickets;
    std::vector<char> seen;             // batched mode: completion recorded
    uint32_t n_seen = 0;
    hipEvent_t done_ev = nullptr;       // plain mode: after the request
};

struct StreamBufs {                     // reused fill descriptors per stream
    FillDesc *host = nullptr;           // pinned
    FillDesc *dev = nullptr;
    uint32_t cap = 0;
};

struct Server {
    rp_server_config cfg{};
    int device = 0;
    uint32_t cus = 1;                   // compute units of the device
    unsigned char *base = nullptr;
    rpserve::Arena arena;
    hipStream_t streams[N_STREAMS] = {};
    bool busy[N_STREAMS] = {};
    StreamBufs bufs[N_STREAMS];

    std::mutex mu;
    std::condition_variable cv;
    bool stopping = false;
    uint64_t next_ticket = 1;
    std::map<uint64_t, Req> reqs;
    std::deque<uint64_t> queue;         // waiting for arena space, FIFO
    std::deque<uint64_t> admitted[2];   // [0] small, [1] large
    std::deque<uint64_t> completed;
    rp_server_stats stats{};

    std::vector<Launch> inflight;       // dispatcher thread only
    Resident res;                       // resident mode
    std::thread thread;
    int thread_error = RP_OK;
};

std::mutex g_smu;
std::map<uint64_t, Server *> g_servers;
uint64_t g_next_server = 1;
uint64_t g_default_budget = 64ull << 30;   // guarded by g_smu

Server *find_server(uint64_t id)
{
    std::lock_guard<std::mutex> lk(g_smu);
    auto it = g_servers.find(id);
    return it == g_servers.end() ? nullptr : it->second;
}

bool valid_server_request(const rp_server_request &q)
{
    if (q.n == 0 || q.n >= (1ull << 32))
        return false;
    if (q.elem_bytes == 0 || (q.elem_bytes & 3u) || q.elem_bytes > 256)
        return false;
    if (!(q.eps > 0.0 && q.eps < 1.0))
        return false;
    if (q.init != RP_INIT_IDENTITY && q.init != RP_INIT_COPY)
        return false;
    if (q.init == RP_INIT_COPY && q.src == nullptr)
        return false;
    return true;
}

// Free a request's array (caller holds mu).
void drop_memory(Server &s, Req &r)
{
    if (r.has_mem) {
        s.arena.free(r.off, r.bytes);
        r.has_mem = false;
    }
    s.stats.bytes_in_use = s.arena.in_use();
}

bool ensure_bufs(StreamBufs &b, uint32_t count)
{
    if (b.cap >= count)
        return true;
    if (b.host)
        (void)hipHostFree(b.host);
    if (b.dev)
        (void)hipFree(b.dev);
    b = StreamBufs{};
    const uint32_t cap = std::max(count, 4096u);   // growing frees, which waits for the device
    if (hipHostMalloc(reinterpret_cast<void **>(&b.host), sizeof(FillDesc) * cap) != hipSuccess)
        return false;
    if (hipMalloc(reinterpret_cast<void **>(&b.dev), sizeof(FillDesc) * cap) != hipSuccess) {
        (void)hipHostFree(b.host);
        b.host = nullptr;
        return false;
    }
    b.cap = cap;
    return true;
}

// Fill the arrays of one launch on stream `si`.  Identity fills run as one
// kernel over all of them; copies are stream-ordered memcpys.
int fill_arrays(Server &s, int si, const std::vector<Req *> &rs)
{
    hipStream_t st = s.streams[si];
    std::vector<FillDesc> ident;
    uint64_t total = 0;
    for (Req *r : rs) {
        unsigned char *A = s.base + r->off;
        if (r->q.init == RP_INIT_COPY) {
            if (hipMemcpyAsync(A, r->q.src, r->q.n * r->q.elem_bytes, hipMemcpyDefault, st) !=
                hipSuccess)
                return RP_EDEVICE;
        } else {
            ident.push_back(FillDesc{A, total, r->q.n, r->q.elem_bytes, 0});
            total += r->q.n;
        }
    }
    if (ident.empty())
        return RP_OK;
    if (ident.size() == 1) {
        const uint64_t blocks = (ident[0].n + 255) / 256;
        const uint32_t grid = (uint32_t)std::min<uint64_t>(blocks, 4096);
        hipLaunchKernelGGL(rp_fill_identity_one_kernel, dim3(grid), dim3(256), 0, st, ident[0]);
        return hipGetLastError() == hipSuccess ? RP_OK : RP_EDEVICE;
    }
    // Several requests: descriptors through this stream's buffers.  Only the
    // batched mode gets here, and it launches on a stream only after the
    // stream's previous launch has finished, so the buffers are free.
    StreamBufs &b = s.bufs[si];
    if (!ensure_bufs(b, (uint32_t)ident.size()))
        return RP_ENOMEM;
    std::memcpy(b.host, ident.data(), sizeof(FillDesc) * ident.size());
    if (hipMemcpyAsync(b.dev, b.host, sizeof(FillDesc) * ident.size(), hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return RP_EDEVICE;
    const uint64_t chunks = (total + FILL_CHUNK - 1) / FILL_CHUNK;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(chunks, 4096);
    hipLaunchKernelGGL(rp_fill_identity_kernel, dim3(grid), dim3(256), 0, st, b.dev,
                       (uint32_t)ident.size(), total);
    return hipGetLastError() == hipSuccess ? RP_OK : RP_EDEVICE;
}

void mark_done(Server &s, uint64_t ticket, int32_t status)
{
    auto it = s.reqs.find(ticket);
    if (it == s.reqs.end())
        return;
    Req &r = it->second;
    r.state = RP_REQ_DONE;
    r.status = status;
    r.t_done = now_ns();
    s.stats.done++;
    s.stats.elements_done += r.q.n;
    s.completed.push_back(ticket);
    if (s.cfg.auto_release)
        drop_memory(s, r);
}

// One dispatcher pass over the running launches; returns true if anything
// finished.
bool reap(Server &s)
{
    bool progress = false;
    for (size_t li = 0; li < s.inflight.size();) {
        Launch &L = s.inflight[li];
        bool finished = false;
        if (L.done_ev) {   // rp_shuffle_inplace (plain mode, alone) or rp_shuffle_group
            const hipError_t e = hipEventQuery(L.done_ev);
            if (e == hipSuccess || e != hipErrorNotReady) {
                std::lock_guard<std::mutex> lk(s.mu);
                for (uint64_t t : L.tickets)
                    mark_done(s, t, e == hipSuccess ? RP_OK : RP_EDEVICE);
                finished = true;
            }
        } else {
            uint32_t nd = 0;
            const int rc = rp_batch_poll(L.batch_id, &nd);
            if (nd > L.n_seen || rc == RP_OK) {
                std::vector<uint64_t> now_done;
                for (size_t i = 0; i < L.tickets.size(); i++)
                    if (!L.seen[i] && rp_batch_request_done(L.batch_id, (uint32_t)i) == RP_OK) {
                        L.seen[i] = 1;
                        L.n_seen++;
                        now_done.push_back(L.tickets[i]);
                    }
                std::vector<rp_batch_result> res;
                if (L.n_seen == L.tickets.size()) {
                    res.resize(L.tickets.size());
                    if (rp_batch_results(L.batch_id, res.data()) != RP_OK)
                        res.clear();
                    (void)rp_batch_release(L.batch_id);
                    finished = true;
                }
                std::lock_guard<std::mutex> lk(s.mu);
                for (uint64_t t : now_done)
                    mark_done(s, t, RP_OK);
                for (size_t i = 0; i < res.size(); i++) {
                    auto it = s.reqs.find(L.tickets[i]);
                    if (it == s.reqs.end())
                        continue;
                    it->second.rounds = res[i].rounds;
                    it->second.aux_words = res[i].aux_words;
                    it->second.status = res[i].status;
                }
            }
        }
        if (finished) {
            if (L.done_ev)
                (void)hipEventDestroy(L.done_ev);
            s.busy[L.stream] = false;
            s.inflight.erase(s.inflight.begin() + (long)li);
            progress = true;
        } else {
            li++;
        }
    }
    return progress;
}

// Admit queued requests in order while the arena has room (caller holds mu).
bool admit(Server &s)
{
    bool progress = false;
    while (!s.queue.empty()) {
        Req &r = s.reqs[s.queue.front()];
        uint64_t off = 0;
        if (!s.arena.alloc(r.bytes, &off))
            break;
        r.off = off;
        r.has_mem = true;
        r.state = RP_REQ_ADMITTED;
        r.t_admit = now_ns();
        s.admitted[r.large ? 1 : 0].push_back(s.queue.front());
        s.queue.pop_front();
        s.stats.admitted++;
        s.stats.bytes_in_use = s.arena.in_use();
        s.stats.peak_bytes = s.arena.peak();
        progress = true;
    }
    return progress;
}

// Move up to `lim` admitted tickets of class `cls` (0 small, 1 large, -1
// whichever was admitted first) to the running state.
std::vector<uint64_t> take_admitted(Server &s, int cls, size_t lim, std::vector<Req *> *rs)
{
    std::vector<uint64_t> tickets;
    std::lock_guard<std::mutex> lk(s.mu);
    while (tickets.size() < lim) {
        int c = cls;
        if (c < 0) {
            auto &a = s.admitted[0], &b = s.admitted[1];
            if (a.empty() && b.empty())
                break;
            c = (!a.empty() && (b.empty() || s.reqs[a.front()].t_admit <= s.reqs[b.front()].t_admit))
                    ? 0 : 1;
        }
        auto &dq = s.admitted[c];
        if (dq.empty())
            break;
        if (cls >= 0) {
            // One launch holds one record size: take the oldest request's
            // size and every later one of the same size, keeping the order
            // of the others.
            const uint32_t eb = s.reqs[dq.front()].q.elem_bytes;
            for (auto it = dq.begin(); it != dq.end() && tickets.size() < lim;) {
                if (s.reqs[*it].q.elem_bytes == eb) {
                    tickets.push_back(*it);
                    it = dq.erase(it);
                } else {
                    ++it;
                }
            }
            break;
        }
        tickets.push_back(dq.front());
        dq.pop_front();
    }
    const uint64_t t = now_ns();
    for (uint64_t tk : tickets) {
        Req &r = s.reqs[tk];
        r.state = RP_REQ_RUNNING;
        r.t_launch = t;
        rs->push_back(&r);   // map nodes are stable; running requests are never erased
    }
    if (!tickets.empty())
        s.stats.launches++;
    return tickets;
}

void fail_tickets(Server &s, const std::vector<uint64_t> &tickets, int rc)
{
    std::lock_guard<std::mutex> lk(s.mu);
    for (uint64_t t : tickets)
        mark_done(s, t, rc);
}

int free_stream(const Server &s, int cls)
{
    const int first = cls == 0 ? 0 : N_SMALL_STREAMS;
    const int count = cls == 0 ? N_SMALL_STREAMS : N_LARGE_STREAMS;
    for (int i = first; i < first + count; i++)
        if (!s.busy[i])
            return i;
    return -1;
}

// The oldest admitted large requests on stream `si`, each with the
// workgroups a call of its own gets (its rounds grid-wide among them)
// instead of one workgroup: as many of them (of the oldest one's record size,
// at most GROUP_MAX) as fit one cooperative launch side by side -- their
// planned grids together within rp_group_capacity, so that the launch is
// always accepted -- in one rp_shuffle_group call, or one alone through
// rp_shuffle_inplace.  Completion is an event recorded after the call.
int launch_alone(Server &s, int si)
{
    size_t lim = 0;
    {
        std::lock_guard<std::mutex> lk(s.mu);
        const std::deque<uint64_t> &dq = s.admitted[1];
        if (dq.empty())
            return RP_PENDING;
        const uint32_t eb = s.reqs[dq.front()].q.elem_bytes;
        uint64_t cap = s.cus;   // one workgroup per unit always fits
        (void)rp_group_capacity(eb, s.device, &cap);
        uint64_t grid = 0;
        for (uint64_t tk : dq) {
            const rp_server_request &q = s.reqs[tk].q;
            if (q.elem_bytes != eb)
                continue;
            uint64_t g = cap;   // unknown or more than one slot per lane: alone
            uint64_t gg = 0;
            if (rpint::group_grid(q.n, q.elem_bytes, q.eps, s.device, &gg) == RP_OK && gg)
                g = gg;
            if (lim > 0 && (grid + g > cap || lim == GROUP_MAX))
                break;
            grid += g;
            lim++;
            if (grid >= cap)
                break;
        }
    }
    std::vector<Req *> rs;
    const std::vector<uint64_t> tickets = take_admitted(s, 1, std::max<size_t>(lim, 1), &rs);
    if (tickets.empty())
        return RP_PENDING;
    hipStream_t st = s.streams[si];
    Launch P;
    P.stream = si;
    P.tickets = tickets;
    int rc = fill_arrays(s, si, rs);
    if (rc == RP_OK && rs.size() == 1) {
        rc = rp_shuffle_inplace(s.base + rs[0]->off, rs[0]->q.n, rs[0]->q.elem_bytes, nullptr,
                                rs[0]->q.seed, rs[0]->q.eps, st, nullptr);
    } else if (rc == RP_OK) {
        std::vector<rp_batch_request> br(rs.size());
        for (size_t i = 0; i < rs.size(); i++) {
            br[i].A = s.base + rs[i]->off;
            br[i].n = rs[i]->q.n;
            br[i].elem_bytes = rs[i]->q.elem_bytes;
            br[i].reserved = 0;
            br[i].H = nullptr;
            br[i].seed = rs[i]->q.seed;
            br[i].eps = rs[i]->q.eps;
        }
        rc = rp_shuffle_group(br.data(), (uint32_t)br.size(), st, nullptr);
    }
    if (rc == RP_OK && (hipEventCreateWithFlags(&P.done_ev, hipEventDisableTiming) != hipSuccess ||
                        hipEventRecord(P.done_ev, st) != hipSuccess))
        rc = RP_EDEVICE;
    if (rc != RP_OK) {
        if (P.done_ev)
            (void)hipEventDestroy(P.done_ev);
        fail_tickets(s, tickets, rc);
        return rc;
    }
    s.busy[si] = true;
    s.inflight.push_back(P);
    return RP_OK;
}

// Batched mode: every admitted request of class `cls` in one launch on a
// free stream of that class (or, with large_alone, a single large request
// that arrives while no other large one runs goes out alone).
int launch_batched(Server &s, int cls)
{
    const int si = free_stream(s, cls);
    if (si < 0)
        return RP_PENDING;
    if (cls == 1 && s.cfg.large_alone) {
        // Large requests run alone (or a few side by side in one group
        // launch), one launch after another in arrival order, as long as few
        // of them wait; a longer queue (overload) goes out as one batched
        // launch so that they all progress.
        bool alone_running = false;
        for (const Launch &L : s.inflight)
            alone_running = alone_running || (L.done_ev && L.stream >= N_SMALL_STREAMS);
        size_t waiting;
        {
            std::lock_guard<std::mutex> lk(s.mu);
            waiting = s.admitted[1].size();
        }
        if (waiting <= ALONE_QUEUE)
            return alone_running ? RP_PENDING : launch_alone(s, si);
    }
    std::vector<Req *> rs;
    const std::vector<uint64_t> tickets =
        take_admitted(s, cls, s.cfg.max_batch ? s.cfg.max_batch : SIZE_MAX, &rs);
    if (tickets.empty())
        return RP_OK;
    int rc = fill_arrays(s, si, rs);
    Launch L;
    L.stream = si;
    L.tickets = tickets;
    L.seen.assign(tickets.size(), 0);
    if (rc == RP_OK) {
        std::vector<rp_batch_request> br(tickets.size());
        for (size_t i = 0; i < rs.size(); i++) {
            br[i].A = s.base + rs[i]->off;
            br[i].n = rs[i]->q.n;
            br[i].elem_bytes = rs[i]->q.elem_bytes;
            br[i].reserved = 0;
            br[i].H = nullptr;
            br[i].seed = rs[i]->q.seed;
            br[i].eps = rs[i]->q.eps;
        }
        const rp_batch_schedule &sc = s.cfg.schedule;
        const bool have_sched = sc.wave_cutoff || sc.table_ratio_x16 || sc.workgroups_per_cu;
        // Large requests: one 1024-lane workgroup each (four times the active
        // swaps of a 256-lane one, so a quarter of the rounds).
        rp_batch_schedule large{};
        large.wave_cutoff = 0;
        large.table_ratio_x16 = have_sched && sc.table_ratio_x16 ? sc.table_ratio_x16 : 24;
        large.workgroups_per_cu = 2;
        large.workgroup_lanes = 1024;
        // Small requests without a configured schedule: 1024-lane
        // workgroups, two per compute unit.  A launch lasts as long as its
        // largest request, and requests arriving meanwhile wait for a free
        // stream, so the shortest launches (the most lanes per request) give
        // the lowest latency under load.
        rp_batch_schedule small{};
        small.wave_cutoff = 1u << 14;
        small.table_ratio_x16 = 16;
        small.workgroups_per_cu = 2;
        small.workgroup_lanes = 1024;
        const rp_batch_schedule *use = cls == 1 ? &large : (have_sched ? &sc : &small);
        rc = rp_batch_submit(br.data(), (uint32_t)br.size(), use, s.streams[si], &L.batch_id);
    }
    if (rc != RP_OK) {
        fail_tickets(s, tickets, rc);
        return rc;
    }
    s.busy[si] = true;
    s.inflight.push_back(std::move(L));
    return RP_OK;
}

// Plain mode: the oldest admitted request as one rp_shuffle_inplace call,
// stream-ordered behind the ones already enqueued.
int launch_plain_one(Server &s)
{
    std::vector<Req *> rs;
    const std::vector<uint64_t> tickets = take_admitted(s, -1, 1, &rs);
    if (tickets.empty())
        return RP_PENDING;
    const int si = 0;
    hipStream_t st = s.streams[si];
    Launch P;
    P.stream = si;
    P.tickets = tickets;
    int rc = fill_arrays(s, si, rs);
    if (rc == RP_OK)
        rc = rp_shuffle_inplace(s.base + rs[0]->off, rs[0]->q.n, rs[0]->q.elem_bytes, nullptr,
                                rs[0]->q.seed, rs[0]->q.eps, st, nullptr);
    if (rc == RP_OK && (hipEventCreateWithFlags(&P.done_ev, hipEventDisableTiming) != hipSuccess ||
                        hipEventRecord(P.done_ev, st) != hipSuccess))
        rc = RP_EDEVICE;
    if (rc != RP_OK) {
        if (P.done_ev)
            (void)hipEventDestroy(P.done_ev);
        fail_tickets(s, tickets, rc);
        return rc;
    }
    s.inflight.push_back(P);
    return RP_OK;
}

// ------------------------------------------------------------ resident mode

// Entries [floor, posted) hold every unfinished one: each ring slot belongs to
// at most one of them (an entry is posted only into a free slot).  Advance
// floor past the reaped ones.
void res_advance_floor(Resident &R)
{
    while (R.floor < R.posted && R.slot_ticket[R.floor & (rpres::RING - 1)] == 0)
        R.floor++;
}

// Fail every posted entry (the kernel or a device call failed); caller holds mu.
void res_fail_posted(Server &s, int rc)
{
    Resident &R = s.res;
    for (uint64_t e = R.floor; e < R.posted; e++) {
        const uint32_t slot = (uint32_t)(e & (rpres::RING - 1));
        const uint64_t t = R.slot_ticket[slot];
        if (t == 0)
            continue;
        Req &r = s.reqs[t];
        if (r.has_aux) {
            s.arena.free(r.aux_off, r.aux_bytes);
            r.has_aux = false;
        }
        R.slot_ticket[slot] = 0;
        R.busy_slots--;
        mark_done(s, t, rc);
    }
    R.floor = R.posted;
    R.wgs_out = 0;
    s.thread_error = rc;
}

// The end of the kernel, and the results of finished ring entries.  An entry
// whose gang could not form did not run: it is posted again, for one
// workgroup.
bool res_reap(Server &s)
{
    Resident &R = s.res;
    bool progress = false;
    if (R.running) {
        const hipError_t e = hipEventQuery(R.ev);
        if (e == hipSuccess) {
            R.running = false;
            R.stop_sent = false;
            progress = true;
        } else if (e != hipErrorNotReady) {
            R.running = false;
            std::lock_guard<std::mutex> lk(s.mu);
            res_fail_posted(s, RP_EDEVICE);
            return true;
        }
    }
    if (R.busy_slots == 0)
        return progress;
    std::lock_guard<std::mutex> lk(s.mu);
    for (uint64_t e = R.floor; e < R.posted; e++) {
        const uint32_t slot = (uint32_t)(e & (rpres::RING - 1));
        const uint64_t t = R.slot_ticket[slot];
        if (t == 0)
            continue;
        Req &r = s.reqs[t];
        if (__atomic_load_n(&R.res[slot].done, __ATOMIC_ACQUIRE) != r.entry + 1)
            continue;
        const int32_t status = R.res[slot].status;
        R.slot_ticket[slot] = 0;
        R.busy_slots--;
        R.wgs_out -= std::min(R.wgs_out, r.gang);
        if (r.has_aux) {
            s.arena.free(r.aux_off, r.aux_bytes);
            r.has_aux = false;
        }
        progress = true;
        if (status == RP_PENDING) {
            r.force_single = true;
            r.state = RP_REQ_ADMITTED;
            s.admitted[0].push_front(t);
            continue;
        }
        r.rounds = R.res[slot].rounds;
        mark_done(s, t, status);
    }
    res_advance_floor(R);
    s.stats.bytes_in_use = s.arena.in_use();
    return progress;
}

// Post admitted requests, in admission order, to the ring.  A request of at
// least 2^large_log2 elements runs on a gang when one can be planned: up to a
// quarter of the kernel's workgroups and half of those the posted requests do
// not hold, at least 8 (under load gangs shrink: a small gang's rounds cost
// more workgroup time per swap than a large one's, but far less than one
// workgroup's), and when the arena holds its tables; otherwise on one
// workgroup.
bool res_post(Server &s)
{
    Resident &R = s.res;
    bool progress = false;
    std::lock_guard<std::mutex> lk(s.mu);
    while (!s.admitted[0].empty()) {
        const uint32_t slot = (uint32_t)(R.posted & (rpres::RING - 1));
        if (R.slot_ticket[slot] != 0)
            break;   // the ring is full up to the oldest unfinished entry
        const uint64_t t = s.admitted[0].front();
        Req &r = s.reqs[t];
        const uint32_t free_wgs = R.grid - std::min(R.grid, R.wgs_out);
        const uint32_t max_gang = std::min(free_wgs / 2, R.gang_cap ? R.gang_cap : R.grid / 4);
        const bool allow = r.gang_ok && !r.force_single && max_gang >= 8;
        rpres::Entry e;
        uint64_t auxb = 0;
        int rc = rpint::resident_plan(r.q.n, r.q.elem_bytes, r.q.eps, max_gang, s.device, allow,
                                      &e, &auxb);
        if (rc == RP_OK && e.gang > 1) {
            uint64_t off = 0;
            if (s.arena.alloc(auxb, &off)) {
                r.aux_off = off;
                r.aux_bytes = auxb;
                r.has_aux = true;
            } else {
                rc = rpint::resident_plan(r.q.n, r.q.elem_bytes, r.q.eps, 0, s.device, false, &e,
                                          &auxb);
            }
        }
        s.admitted[0].pop_front();
        progress = true;
        if (rc != RP_OK) {
            mark_done(s, t, rc);
            continue;
        }
        e.A = s.base + r.off;
        e.aux = r.has_aux ? s.base + r.aux_off : nullptr;
        e.seed = r.q.seed;
        e.fill = r.q.init == RP_INIT_COPY ? rpres::FILL_COPY : rpres::FILL_IDENTITY;
        e.src = r.q.src;
        // the entry, then its sequence number
        rpres::Entry *dst = &R.ring[slot];
        std::memcpy(static_cast<void *>(dst), &e, offsetof(rpres::Entry, seq));
        __atomic_store_n(&dst->seq, R.posted + 1, __ATOMIC_RELEASE);
        r.entry = R.posted++;
        r.gang = e.gang;
        r.aux_words = e.aux_words;
        r.state = RP_REQ_RUNNING;
        r.t_launch = now_ns();
        R.slot_ticket[slot] = t;
        R.busy_slots++;
        R.wgs_out += e.gang;
    }
    s.stats.bytes_in_use = s.arena.in_use();
    s.stats.peak_bytes = s.arena.peak();
    return progress;
}

// Launch the kernel when entries wait and it is not running (it starts at the
// oldest unfinished entry: everything a previous launch claimed has
// finished); stop it after RES_IDLE_STOP_NS without work, or at once when
// the server is being destroyed and nothing is left.
bool res_manage(Server &s, bool stopping)
{
    Resident &R = s.res;
    bool work;
    uint64_t first = UINT64_MAX;
    {
        std::lock_guard<std::mutex> lk(s.mu);
        work = R.busy_slots > 0 || !s.admitted[0].empty();
        if (R.busy_slots > 0 && !R.running)
            first = R.floor;   // the oldest unfinished entry
    }
    if (first != UINT64_MAX) {
        __atomic_store_n(R.stop, 0u, __ATOMIC_RELEASE);
        const rpres::Launch L{R.ring, R.res, R.stop, R.ctl, first, RES_IDLE_TICKS,
                              R.form_ticks, R.grid};
        int rc = rpint::resident_launch(L, R.stream);
        if (rc == RP_OK && hipEventRecord(R.ev, R.stream) != hipSuccess)
            rc = RP_EDEVICE;
        std::lock_guard<std::mutex> lk(s.mu);
        if (rc != RP_OK) {
            res_fail_posted(s, rc);
            return true;
        }
        R.running = true;
        R.stop_sent = false;
        R.idle_since = 0;
        s.stats.launches++;
        return true;
    }
    if (R.running && !R.stop_sent) {
        if (work) {
            R.idle_since = 0;
        } else {
            const uint64_t t = now_ns();
            if (R.idle_since == 0)
                R.idle_since = t;
            if (stopping || t - R.idle_since > RES_IDLE_STOP_NS) {
                __atomic_store_n(R.stop, 1u, __ATOMIC_RELEASE);
                R.stop_sent = true;
            }
        }
    }
    return false;
}

int res_create(Server &s)
{
    Resident &R = s.res;
    R.slot_ticket.assign(rpres::RING, 0);
    // RP_RES_FORM_US (environment) shortens the time a gang has to form, so
    // that tests can make leaders give their requests back.
    const char *fu = getenv("RP_RES_FORM_US");
    if (fu && *fu)
        R.form_ticks = (uint64_t)std::max(0, atoi(fu)) * 100;
    // RP_RES_MAX_GANG (environment) replaces the largest gang, a quarter of
    // the grid (a tuning override; below 8 every request runs on one
    // workgroup).
    const char *mg = getenv("RP_RES_MAX_GANG");
    if (mg && *mg)
        R.gang_cap = (uint32_t)std::max(1, atoi(mg));
    if (rpint::resident_grid(s.device, &R.grid) != RP_OK)
        return RP_EDEVICE;
    if (hipHostMalloc(reinterpret_cast<void **>(&R.ring), sizeof(rpres::Entry) * rpres::RING,
                      hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&R.res), sizeof(rpres::Result) * rpres::RING,
                      hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&R.stop), 64, hipHostMallocCoherent) != hipSuccess)
        return RP_ENOMEM;
    std::memset(static_cast<void *>(R.ring), 0, sizeof(rpres::Entry) * rpres::RING);
    std::memset(static_cast<void *>(R.res), 0, sizeof(rpres::Result) * rpres::RING);
    *R.stop = 0;
    if (hipMalloc(&R.ctl, rpint::resident_ctl_bytes()) != hipSuccess)
        return RP_ENOMEM;
    if (hipStreamCreateWithFlags(&R.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&R.ev, hipEventDisableTiming) != hipSuccess)
        return RP_EDEVICE;
    return RP_OK;
}

void res_destroy(Server &s)
{
    Resident &R = s.res;
    if (R.stream) {
        if (R.stop)
            __atomic_store_n(R.stop, 1u, __ATOMIC_RELEASE);
        (void)hipStreamSynchronize(R.stream);
        (void)hipStreamDestroy(R.stream);
    }
    if (R.ev)
        (void)hipEventDestroy(R.ev);
    if (R.ctl)
        (void)hipFree(R.ctl);
    if (R.ring)
        (void)hipHostFree(R.ring);
    if (R.res)
        (void)hipHostFree(R.res);
    if (R.stop)
        (void)hipHostFree(R.stop);
    R = Resident{};
}

void dispatcher(Server *sp)
{
    Server &s = *sp;
    (void)hipSetDevice(s.device);
    const auto tick = std::chrono::microseconds(s.cfg.tick_us ? s.cfg.tick_us : 50);
    const bool resident = s.cfg.mode == RP_SERVE_RESIDENT;
    for (;;) {
        bool progress = reap(s);
        if (resident)
            progress = res_reap(s) || progress;
        {
            std::lock_guard<std::mutex> lk(s.mu);
            progress = admit(s) || progress;
        }
        if (resident) {
            progress = res_post(s) || progress;
            bool stopping;
            {
                std::lock_guard<std::mutex> lk(s.mu);
                stopping = s.stopping;
            }
            progress = res_manage(s, stopping) || progress;
        } else if (s.cfg.mode == RP_SERVE_PLAIN) {
            // keep up to PLAIN_AHEAD requests enqueued on the single stream
            while (s.inflight.size() < PLAIN_AHEAD) {
                const int rc = launch_plain_one(s);
                if (rc == RP_PENDING)
                    break;
                progress = true;
                if (rc != RP_OK) {
                    std::lock_guard<std::mutex> lk(s.mu);
                    s.thread_error = rc;
                    break;
                }
            }
        } else {
            for (int cls = 0; cls < 2; cls++) {
                bool any;
                {
                    std::lock_guard<std::mutex> lk(s.mu);
                    any = !s.admitted[cls].empty();
                }
                if (!any)
                    continue;
                const int rc = launch_batched(s, cls);
                if (rc == RP_OK) {
                    progress = true;
                } else if (rc != RP_PENDING) {
                    progress = true;
                    std::lock_guard<std::mutex> lk(s.mu);
                    s.thread_error = rc;
                }
            }
        }
        std::unique_lock<std::mutex> lk(s.mu);
        if (s.stopping) {
            // Requests that were not launched are cancelled; running ones finish.
            for (uint64_t t : s.queue)
                mark_done(s, t, RP_ECANCELED);
            s.queue.clear();
            for (int c = 0; c < 2; c++) {
                for (uint64_t t : s.admitted[c])
                    mark_done(s, t, RP_ECANCELED);
                s.admitted[c].clear();
            }
            if (s.inflight.empty() && s.res.busy_slots == 0 && !s.res.running)
                break;
        }
        if (s.thread_error != RP_OK && s.inflight.empty()) {
            // A device call failed: fail whatever is still waiting.
            for (uint64_t t : s.queue)
                mark_done(s, t, s.thread_error);
            for (int c = 0; c < 2; c++) {
                for (uint64_t t : s.admitted[c])
                    mark_done(s, t, s.thread_error);
                s.admitted[c].clear();
            }
            s.queue.clear();
            if (s.stopping && !s.res.running)
                break;
        }
        if (!progress)
            s.cv.wait_for(lk, tick);
    }
}

// The servers' streams, created once per device and process and shared by
// every server on that device: the runtime spreads a process's streams over
// a few hardware queues in creation order, so a fresh set per server could
// leave a small-request stream on the same hardware queue as a large-request
// one (small launches then wait behind large ones), depending on how many
// streams the process created before.
std::mutex g_stream_mu;
std::map<int, std::vector<hipStream_t>> g_streams;

int server_streams(int device, hipStream_t *out)
{
    std::lock_guard<std::mutex> lk(g_stream_mu);
    auto it = g_streams.find(device);
    if (it == g_streams.end()) {
        std::vector<hipStream_t> v(N_STREAMS, nullptr);
        for (int i = 0; i < N_STREAMS; i++)
            if (hipStreamCreateWithFlags(&v[i], hipStreamNonBlocking) != hipSuccess) {
                for (int j = 0; j < i; j++)
                    (void)hipStreamDestroy(v[j]);
                return RP_EDEVICE;
            }
        it = g_streams.emplace(device, std::move(v)).first;
    }
    for (int i = 0; i < N_STREAMS; i++)
        out[i] = it->second[i];
    return RP_OK;
}

void destroy_server(Server *s)
{
    res_destroy(*s);
    for (int i = 0; i < N_STREAMS; i++) {
        if (s->streams[i])
            (void)hipStreamSynchronize(s->streams[i]);   // shared: not destroyed
        if (s->bufs[i].host)
            (void)hipHostFree(s->bufs[i].host);
        if (s->bufs[i].dev)
            (void)hipFree(s->bufs[i].dev);
    }
    if (s->base)
        (void)hipFree(s->base);
    delete s;
}

}  // namespace

extern "C" {

int rp_set_mem_budget(uint64_t bytes)
{
    if (bytes == 0)
        return RP_EINVAL;
    std::lock_guard<std::mutex> lk(g_smu);
    g_default_budget = bytes;
    return RP_OK;
}

int rp_server_create(const rp_server_config *cfg, uint64_t *server)
{
    if (cfg == nullptr || server == nullptr ||
        (cfg->mode != RP_SERVE_BATCHED && cfg->mode != RP_SERVE_PLAIN &&
         cfg->mode != RP_SERVE_RESIDENT) ||
        cfg->large_log2 > 40)
        return RP_EINVAL;
    Server *s = new Server;
    s->cfg = *cfg;
    if (s->cfg.mem_budget_bytes == 0) {
        std::lock_guard<std::mutex> lk(g_smu);
        s->cfg.mem_budget_bytes = g_default_budget;
    }
    // Default large threshold: 2^22; resident mode 2^20 (a gang beats one
    // 512-lane workgroup from there on: a lone 2^22 request took 16.5 ms on a
    // gang of 54 against 51.5 ms on one workgroup).
    if (s->cfg.large_log2 == 0)
        s->cfg.large_log2 = s->cfg.mode == RP_SERVE_RESIDENT ? 20 : 22;
    int cus = 0;
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device) !=
            hipSuccess) {
        delete s;
        return RP_EDEVICE;
    }
    s->cus = (uint32_t)std::max(cus, 1);
    if (hipMalloc(reinterpret_cast<void **>(&s->base), s->cfg.mem_budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        s->base = nullptr;
        destroy_server(s);
        return RP_ENOMEM;
    }
    s->arena.reset(s->cfg.mem_budget_bytes / rpserve::ALIGN * rpserve::ALIGN);
    if (server_streams(s->device, s->streams) != RP_OK) {
        destroy_server(s);
        return RP_EDEVICE;
    }
    if (s->cfg.mode == RP_SERVE_RESIDENT) {
        const int rc = res_create(*s);
        if (rc != RP_OK) {
            destroy_server(s);
            return rc;
        }
    }
    s->thread = std::thread(dispatcher, s);
    std::lock_guard<std::mutex> lk(g_smu);
    *server = g_next_server++;
    g_servers[*server] = s;
    return RP_OK;
}

int rp_server_submit(uint64_t server, const rp_server_request *req, uint64_t *ticket)
{
    Server *s = find_server(server);
    if (s == nullptr || req == nullptr || ticket == nullptr || !valid_server_request(*req))
        return RP_EINVAL;
    const uint64_t bytes = req->n * req->elem_bytes;
    if (rpserve::Arena::rounded(bytes) > s->arena.size())
        return RP_EINVAL;
    if (s->cfg.mode == RP_SERVE_RESIDENT && req->init == RP_INIT_COPY) {
        // The kernel reads the source itself: it must be device memory or
        // pinned host memory.
        hipPointerAttribute_t at;
        if (hipPointerGetAttributes(&at, req->src) != hipSuccess) {
            (void)hipGetLastError();
            return RP_EINVAL;
        }
        if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeHost &&
            at.type != hipMemoryTypeManaged)
            return RP_EINVAL;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping)
            return RP_EINVAL;
        const uint64_t t = s->next_ticket++;
        Req &r = s->reqs[t];
        r.q = *req;
        r.bytes = bytes;
        r.gang_ok = req->n >= (1ull << s->cfg.large_log2);
        r.large = r.gang_ok && s->cfg.mode != RP_SERVE_RESIDENT;
        r.t_submit = now_ns();
        s->queue.push_back(t);
        s->stats.submitted++;
        *ticket = t;
    }
    s->cv.notify_one();
    return RP_OK;
}

int rp_server_info(uint64_t server, uint64_t ticket, rp_server_ticket_info *info)
{
    Server *s = find_server(server);
    if (s == nullptr || info == nullptr)
        return RP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return RP_EINVAL;
    const Req &r = it->second;
    std::memset(info, 0, sizeof(*info));
    info->state = r.state;
    info->status = r.status;
    info->t_submit_ns = r.t_submit;
    info->t_admit_ns = r.t_admit;
    info->t_launch_ns = r.t_launch;
    info->t_done_ns = r.t_done;
    info->A = r.has_mem ? static_cast<void *>(s->base + r.off) : nullptr;
    info->rounds = r.rounds;
    info->aux_words = r.aux_words;
    info->workgroups = s->cfg.mode == RP_SERVE_RESIDENT ? r.gang : 0;
    return RP_OK;
}

int rp_server_completed(uint64_t server, uint64_t *tickets, uint32_t max, uint32_t *count)
{
    Server *s = find_server(server);
    if (s == nullptr || count == nullptr || (tickets == nullptr && max > 0))
        return RP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    uint32_t c = 0;
    while (c < max && !s->completed.empty()) {
        tickets[c++] = s->completed.front();
        s->completed.pop_front();
    }
    *count = c;
    return RP_OK;
}

int rp_server_copy_out(uint64_t server, uint64_t ticket, void *dst, void *stream)
{
    Server *s = find_server(server);
    if (s == nullptr || dst == nullptr)
        return RP_EINVAL;
    void *A;
    uint64_t bytes;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end())
            return RP_EINVAL;
        const Req &r = it->second;
        if (r.state != RP_REQ_DONE)
            return RP_PENDING;
        if (!r.has_mem)
            return RP_EINVAL;
        A = s->base + r.off;
        bytes = r.q.n * r.q.elem_bytes;
    }
    // The request finished (its completion was observed), so its array is
    // final; the memory stays allocated until the caller releases the ticket.
    return hipMemcpyAsync(dst, A, bytes, hipMemcpyDefault, reinterpret_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? RP_OK
               : RP_EDEVICE;
}

int rp_server_release(uint64_t server, uint64_t ticket)
{
    Server *s = find_server(server);
    if (s == nullptr)
        return RP_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end())
            return RP_EINVAL;
        if (it->second.state != RP_REQ_DONE)
            return RP_PENDING;
        drop_memory(*s, it->second);
        s->reqs.erase(it);
    }
    s->cv.notify_one();   // freed space may admit queued requests
    return RP_OK;
}

int rp_server_stats_get(uint64_t server, rp_server_stats *out)
{
    Server *s = find_server(server);
    if (s == nullptr || out == nullptr)
        return RP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->bytes_in_use = s->arena.in_use();
    out->peak_bytes = s->arena.peak();
    return RP_OK;
}

int rp_server_destroy(uint64_t server)
{
    Server *s;
    {
        std::lock_guard<std::mutex> lk(g_smu);
        auto it = g_servers.find(server);
        if (it == g_servers.end())
            return RP_EINVAL;
        s = it->second;
        g_servers.erase(it);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv.notify_one();
    if (s->thread.joinable())
        s->thread.join();
    const int err = s->thread_error;
    destroy_server(s);
    return err;
}

}  // extern "C"
