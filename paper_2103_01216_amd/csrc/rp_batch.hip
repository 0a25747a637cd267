// Batched form of librp: many independent in-place shuffles in one persistent
// launch.
//
// Every request is the Knuth shuffle of Section 4.1 (Gu, Obeya, Shun,
// "Parallel In-Place Algorithms: Theory and Practice") on its own array, run
// with the same round structure as rp.hip (relaxed-PIP rounds over the first
// k unfinished swaps, RP-Final single reservation with a dense window for the
// round's consecutive keys), but every request is owned by one group of
// lanes and never synchronises with another group:
//   * workgroup mode: the whole workgroup runs one request; the hashed
//     reservation array and the dense window live in the workgroup's LDS and
//     rounds are separated by workgroup barriers;
//   * wave mode: one wave runs one small request in its own quarter of the
//     LDS; a wave executes in order, so rounds need no barrier at all.
// Requests are sorted by size, largest first; the largest ones are claimed by
// workgroups from one counter, the rest by single waves from another (longest
// job first keeps the tail short).  The size that separates the two modes, the
// table ratio and the number of resident workgroups form the schedule, chosen
// by rp_batch_autotune from timed trial runs on scratch copies of a sample of
// the batch.
//
// Auxiliary space per request: the LDS words its round state uses (slots and
// both dense-window parities), at most floor(n^(1-eps)) 8-byte words.
// Completion is signalled per request through host-visible memory, so the
// caller can poll without blocking.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <set>
#include <sstream>
#include <string>
#include <mutex>
#include <numeric>
#include <vector>

#include <sys/stat.h>

#include "rp.h"
#include "rp_device.h"
#include "rp_wg.h"

namespace {

using namespace rpdev;
using namespace rpwg;

struct BatchParams {
    BatchReq *reqs;
    uint32_t count;
    uint32_t n_wg;          // reqs[0 .. n_wg) run in workgroup mode
    uint32_t *claims;       // [0]: next workgroup request, [1]: next wave request
    rp_batch_result *res;   // indexed by the caller's order
    uint32_t *done_flags;   // host-visible: per request (caller's order)
    uint32_t late;          // 1: records read after the decision
};

__device__ __forceinline__ void publish(const BatchParams &bp, const BatchReq &r,
                                        uint64_t rounds, uint64_t attempts,
                                        uint32_t status)
{
    rp_batch_result out;
    out.rounds = rounds;
    out.attempts = attempts;
    out.status = r.invalid ? RP_EINVAL : status ? -(int32_t)status : RP_OK;
    out.aux_words = (uint32_t)(((uint64_t)(r.T + 2 * r.bmw) * 4 + 7) / 8);
    bp.res[r.orig] = out;
    // Make the request's records and result visible beyond the device, then
    // raise its completion flag.  Host memory is only ever written with
    // stores (no read-modify-write atomics across the host link).
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __hip_atomic_store(&bp.done_flags[r.orig], 1u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int EB, int WGL>
__global__ __launch_bounds__(WGL) void rp_batch_kernel(BatchParams bp)
{
    using S = Shape<WGL>;
    __shared__ uint32_t lds[S::LDS_WORDS];
    __shared__ uint32_t sh_scan[S::WAVES];
    __shared__ uint64_t sh_red[S::WAVES];
    __shared__ uint32_t sh_claim;

    // Every value that steers these loops is wave-uniform (held in scalar
    // registers), and the single-lane claim and publish steps are closed by
    // a barrier before the loop's back edge.  Otherwise the compiler may merge
    // the publish of one iteration with the claim of the next into a region
    // that parks the claiming lane outside the loop while the other lanes
    // keep re-running the previous request.

    // Workgroup mode: the largest requests, one per workgroup.
    WGGroup<WGL> wg{lds, sh_scan};
    for (;;) {
        if (threadIdx.x == 0)
            sh_claim = __hip_atomic_fetch_add(&bp.claims[0], 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t idx = __builtin_amdgcn_readfirstlane(sh_claim);
        __syncthreads();
        if (idx >= bp.n_wg)
            break;
        const BatchReq r = bp.reqs[idx];
        uint64_t rounds = 0, attempts = 0;
        uint32_t status = 0;
        if (r.n > 1 && !r.invalid)
            run_request<EB>(wg, r, (uint64_t)r.n + 64, bp.late != 0, &rounds, &attempts, &status);
        attempts = sum_over_group_wg<S::WAVES>(attempts, sh_red);
        rounds = sum_over_group_wg<S::WAVES>(r.T == 0 ? rounds : (threadIdx.x == 0 ? rounds : 0),
                                             sh_red);
        if (threadIdx.x == 0)
            publish(bp, r, rounds, attempts, status);
        __syncthreads();
    }
    // Wave mode: the rest, one per wave, each in its share of the LDS.
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    WaveGroup wv{lds + wave * S::WAVE_WORDS};
    for (;;) {
        // Every lane adds (1 on lane 0, 0 elsewhere); lane 0's old value is
        // the claim.  No lane-divergent branch around the claim.
        const uint32_t got = __hip_atomic_fetch_add(&bp.claims[1], lane == 0 ? 1u : 0u,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t idx = bp.n_wg + __builtin_amdgcn_readlane(got, 0);
        if (idx >= bp.count)
            break;
        const BatchReq r = bp.reqs[idx];
        uint64_t rounds = 0, attempts = 0;
        uint32_t status = 0;
        if (r.n > 1 && !r.invalid)
            run_request<EB>(wv, r, (uint64_t)r.n + 64, bp.late != 0, &rounds, &attempts, &status);
        attempts = wave_sum64(attempts);
        rounds = wave_sum64(lane == 0 ? rounds : 0);
        if (lane == 0)
            publish(bp, r, rounds, attempts, status);
        __builtin_amdgcn_wave_barrier();
    }
}

// Before the batch: reset the claim counters, and mark every explicit-target
// request with some H[i] > i as invalid (it is then skipped and its array is
// left untouched).  One workgroup per request.
__global__ void rp_batch_prepare_kernel(BatchReq *reqs, uint32_t count, uint32_t *claims)
{
    // The claim counters are later advanced by atomic adds: reset them with an
    // atomic too (a plain store and RMW atomics on one word are not ordered).
    if (blockIdx.x == 0 && threadIdx.x < 16)
        (void)__hip_atomic_exchange(&claims[threadIdx.x], 0u, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t q = blockIdx.x; q < count; q += gridDim.x) {
        const BatchReq &r = reqs[q];
        if (r.H == nullptr)
            continue;
        bool bad = false;
        for (uint32_t i = threadIdx.x; i < r.n; i += blockDim.x)
            bad = bad || (r.H[i] > i);
        if (bad)
            __hip_atomic_store(&reqs[q].invalid, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------------- host

int env_or(const char *name, int dflt)
{
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

// Pinned host buffers of one batch.  Allocating pinned memory costs far more
// than a small batch's kernel, so released buffers go back to a pool.
struct HostBufs {
    BatchReq *staging = nullptr;    // pinned copy of the descriptors
    rp_batch_result *res = nullptr; // host-visible results
    uint32_t *done = nullptr;       // coherent: [1..cap] completion flags
    uint32_t cap = 0;
};

std::mutex g_pool_mu;
std::vector<HostBufs> g_pool;
constexpr size_t POOL_MAX = 16;

void free_host(HostBufs &h)
{
    if (h.staging)
        (void)hipHostFree(h.staging);
    if (h.res)
        (void)hipHostFree(h.res);
    if (h.done)
        (void)hipHostFree(h.done);
    h = HostBufs{};
}

bool acquire_host(uint32_t count, HostBufs *out)
{
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        size_t best = g_pool.size();
        for (size_t i = 0; i < g_pool.size(); i++)
            if (g_pool[i].cap >= count && (best == g_pool.size() || g_pool[i].cap < g_pool[best].cap))
                best = i;
        if (best < g_pool.size()) {
            *out = g_pool[best];
            g_pool.erase(g_pool.begin() + (long)best);
            return true;
        }
    }
    HostBufs h;
    h.cap = std::max(count, 64u);
    if (hipHostMalloc(reinterpret_cast<void **>(&h.staging), sizeof(BatchReq) * h.cap) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&h.res), sizeof(rp_batch_result) * h.cap) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&h.done), sizeof(uint32_t) * (h.cap + 1),
                      hipHostMallocCoherent) != hipSuccess) {
        free_host(h);
        return false;
    }
    *out = h;
    return true;
}

// Only after the stream has passed every use of the buffers.
void return_host(HostBufs &h)
{
    if (!h.staging)
        return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (g_pool.size() < POOL_MAX) {
        g_pool.push_back(h);
        h = HostBufs{};
    } else {
        free_host(h);
    }
}

struct Batch {
    hipStream_t stream = nullptr;
    uint32_t count = 0;
    void *dev = nullptr;            // reqs | claims
    HostBufs host;
    rp_batch_result *res = nullptr; // = host.res
    uint32_t *done = nullptr;       // = host.done
    BatchReq *staging = nullptr;    // = host.staging
};

std::mutex g_bmu;
std::map<uint64_t, Batch> g_batches;
uint64_t g_next_id = 1;


bool valid_request(const rp_batch_request &q)
{
    if (!(q.eps > 0.0 && q.eps < 1.0))
        return false;
    if (q.elem_bytes == 0 || (q.elem_bytes & 3u) || q.elem_bytes > 256)
        return false;
    if (q.n >= BATCH_MAX_N)
        return false;
    if (q.A == nullptr && q.n > 1)
        return false;
    if (q.n > 1 && (reinterpret_cast<uintptr_t>(q.A) & (record_alignment(q.elem_bytes) - 1u)) != 0)
        return false;
    if (q.H != nullptr && (reinterpret_cast<uintptr_t>(q.H) & 7u) != 0)
        return false;
    return true;
}

rp_batch_schedule default_schedule()
{
    rp_batch_schedule s{};
    s.wave_cutoff = (uint32_t)env_or("RP_BATCH_CUTOFF", 1 << 14);
    s.table_ratio_x16 = (uint32_t)env_or("RP_BATCH_RATIO16", 16);
    s.workgroups_per_cu = (uint32_t)env_or("RP_BATCH_WPC", 4);
    s.workgroup_lanes = (uint32_t)env_or("RP_BATCH_LANES", 256);
    s.late_loads = (uint32_t)env_or("RP_BATCH_LATE", 0);
    return s;
}

std::mutex g_tmu;
bool g_tuned = false;
rp_batch_schedule g_tuned_sched{};

using BatchKernelFn = void (*)(BatchParams);

uint32_t lanes_of(const rp_batch_schedule &s)
{
    return s.workgroup_lanes == 1024 ? 1024u : 256u;
}

BatchKernelFn pick_batch_kernel(uint32_t eb, uint32_t lanes)
{
    if (lanes == 1024) {
        if (eb == 4) return rp_batch_kernel<4, 1024>;
        if (eb == 8) return rp_batch_kernel<8, 1024>;
        return rp_batch_kernel<0, 1024>;
    }
    if (eb == 4) return rp_batch_kernel<4, 256>;
    if (eb == 8) return rp_batch_kernel<8, 256>;
    return rp_batch_kernel<0, 256>;
}

int launch_batch(const rp_batch_request *reqs, uint32_t count,
                 const rp_batch_schedule &sched, hipStream_t stream, Batch *b)
{
    b->stream = stream;
    b->count = count;
    const double ratio = std::max(1u, sched.table_ratio_x16) / 16.0;
    const uint32_t lanes = lanes_of(sched);
    uint32_t eb = 0;
    for (uint32_t i = 0; i < count; i++) {
        if (!valid_request(reqs[i]))
            return RP_EINVAL;
        if (eb == 0)
            eb = reqs[i].elem_bytes;
        else if (eb != reqs[i].elem_bytes)
            return RP_EINVAL;  // one record size per batch
    }
    // Order: largest first; workgroup mode for n >= cutoff.
    std::vector<uint32_t> order(count);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t c) { return reqs[a].n > reqs[c].n; });
    if (!acquire_host(count, &b->host))
        return RP_ENOMEM;
    b->staging = b->host.staging;
    b->res = b->host.res;
    b->done = b->host.done;
    std::memset(b->done, 0, sizeof(uint32_t) * (count + 1));
    std::memset(b->res, 0, sizeof(rp_batch_result) * std::max(1u, count));
    uint32_t n_wg = 0;
    for (uint32_t i = 0; i < count; i++) {
        const rp_batch_request &q = reqs[order[i]];
        const bool wgm = q.n >= sched.wave_cutoff;
        n_wg += wgm ? 1u : 0u;
        BatchReq &r = b->staging[i];
        r.A = static_cast<unsigned char *>(q.A);
        r.H = q.H;
        r.seed = q.seed;
        r.n = (uint32_t)q.n;
        r.eb = q.elem_bytes;
        plan_request(q.n, q.eps, ratio, wgm ? lanes : 64,
                     wgm ? (lanes == 1024 ? Shape<1024>::LDS_WORDS : Shape<256>::LDS_WORDS)
                         : (lanes == 1024 ? Shape<1024>::WAVE_WORDS : Shape<256>::WAVE_WORDS),
                     &r.k, &r.T, &r.bmw);
        r.wg_mode = wgm ? 1u : 0u;
        r.orig = order[i];
        r.invalid = 0;
    }
    // Sorted order puts every workgroup-mode request first.
    const size_t bytes = sizeof(BatchReq) * std::max(1u, count) + 64;
    if (hipMallocAsync(&b->dev, bytes, stream) != hipSuccess) {
        (void)hipGetLastError();
        return RP_ENOMEM;
    }
    BatchReq *dreqs = static_cast<BatchReq *>(b->dev);
    uint32_t *claims = reinterpret_cast<uint32_t *>(
        static_cast<unsigned char *>(b->dev) + sizeof(BatchReq) * std::max(1u, count));
    if (count > 0 && hipMemcpyAsync(dreqs, b->staging, sizeof(BatchReq) * count,
                                    hipMemcpyHostToDevice, stream) != hipSuccess)
        return RP_EDEVICE;
    rp_batch_prepare_kernel<<<std::max(1u, std::min(count, 4096u)), 256, 0, stream>>>(
        dreqs, count, claims);
    if (hipGetLastError() != hipSuccess)
        return RP_EDEVICE;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
    }
    const BatchKernelFn fn = pick_batch_kernel(eb, lanes);
    int occ = 1;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, reinterpret_cast<const void *>(fn), (int)lanes, 0);
    const uint32_t wpc = std::max(1u, std::min<uint32_t>(sched.workgroups_per_cu,
                                                         (uint32_t)std::max(occ, 1)));
    uint32_t grid = (uint32_t)cus * wpc;
    BatchParams bp{};
    bp.reqs = dreqs;
    bp.count = count;
    bp.n_wg = n_wg;
    bp.claims = claims;
    bp.res = b->res;
    bp.done_flags = b->done + 1;
    bp.late = sched.late_loads ? 1u : 0u;
    if (count > 0) {
        hipLaunchKernelGGL(fn, dim3(grid), dim3(lanes), 0, stream, bp);
        if (hipGetLastError() != hipSuccess)
            return RP_EDEVICE;
    }
    return RP_OK;
}

// ---------------------------------------------------- remembered schedules
//
// rp_batch_autotune keeps its choice in a text file, one line per tuned batch:
//   <device key> <size mix> <wave_cutoff> <ratio16> <per_cu> <lanes> <late> <tuned_us>
// The device key names the architecture, the compute units, the record size
// and the batch's eps values; the size mix is the share of the sample's
// requests in each octave of n, in thousandths ("octave:share,...").  A later
// batch takes the line with its device key whose size mix is closest to its
// own, if the two cumulative shares over the octaves differ by at most
// MIX_MATCH anywhere (a Kolmogorov-Smirnov distance: batches of a few hundred
// requests drawn from one distribution stay well within it, a mix shifted by
// an octave in six does not).

constexpr double MIX_MATCH = 0.15;

std::string tune_cache_path()
{
    const char *v = getenv("RP_TUNE_CACHE");
    if (v != nullptr)
        return std::string(v);   // empty: no cache
    const char *home = getenv("HOME");
    if (home == nullptr || *home == '\0')
        return std::string();
    return std::string(home) + "/.cache/librp/batch_schedules.txt";
}

struct TuneShape {
    std::string key;        // device, record size, eps values
    double mix[33] = {};    // share of requests per octave of n
};

TuneShape tune_shape(int dev, const std::vector<rp_batch_request> &sample)
{
    TuneShape t;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    arch = arch.substr(0, arch.find(':'));
    std::set<long> epss;
    for (const rp_batch_request &q : sample) {
        uint32_t b = 0;
        while (b < 32 && (q.n >> (b + 1)) != 0)
            b++;
        t.mix[b] += 1.0 / (double)sample.size();
        epss.insert(std::lround(q.eps * 1000.0));
    }
    std::ostringstream k;
    k << arch << ":cu" << cus << ":eb" << sample[0].elem_bytes << ":eps";
    for (long e : epss)
        k << "." << e;
    t.key = k.str();
    return t;
}

std::string mix_text(const double *mix)
{
    std::ostringstream m;
    bool first = true;
    for (int b = 0; b < 33; b++) {
        const long sh = std::lround(mix[b] * 1000.0);
        if (sh > 0) {
            m << (first ? "" : ",") << b << ":" << sh;
            first = false;
        }
    }
    return first ? std::string("0:0") : m.str();
}

bool parse_mix(const std::string &text, double *mix)
{
    std::istringstream in(text);
    std::string item;
    while (std::getline(in, item, ',')) {
        const size_t c = item.find(':');
        if (c == std::string::npos)
            return false;
        const int b = std::atoi(item.substr(0, c).c_str());
        if (b < 0 || b > 32)
            return false;
        mix[b] = std::atoi(item.substr(c + 1).c_str()) / 1000.0;
    }
    return true;
}

bool tune_lookup(const std::string &path, const TuneShape &shape, rp_batch_schedule *out)
{
    if (path.empty())
        return false;
    std::ifstream f(path);
    std::string line;
    double best = MIX_MATCH + 1e-9;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string k, m;
        rp_batch_schedule s{};
        if (!(in >> k >> m >> s.wave_cutoff >> s.table_ratio_x16 >> s.workgroups_per_cu >>
              s.workgroup_lanes >> s.late_loads >> s.tuned_ms_x1000) ||
            k != shape.key || s.table_ratio_x16 == 0 || s.workgroups_per_cu == 0 ||
            (s.workgroup_lanes != 256 && s.workgroup_lanes != 1024) || s.late_loads > 1)
            continue;
        double mix[33] = {};
        if (!parse_mix(m, mix))
            continue;
        double ks = 0.0, ca = 0.0, cb = 0.0;
        for (int b = 0; b < 33; b++) {
            ca += mix[b];
            cb += shape.mix[b];
            ks = std::max(ks, std::fabs(ca - cb));
        }
        if (ks <= best) {   // the closest; among equals the later line
            best = ks;
            *out = s;
            found = true;
        }
    }
    return found;
}

void tune_store(const std::string &path, const TuneShape &shape, const rp_batch_schedule &s)
{
    if (path.empty())
        return;
    // Create the directories on the way (a failure shows as a failed open).
    for (size_t i = path.find('/', 1); i != std::string::npos; i = path.find('/', i + 1))
        (void)mkdir(path.substr(0, i).c_str(), 0755);
    std::ofstream f(path, std::ios::app);
    if (f)
        f << shape.key << ' ' << mix_text(shape.mix) << ' ' << s.wave_cutoff << ' '
          << s.table_ratio_x16 << ' ' << s.workgroups_per_cu << ' ' << s.workgroup_lanes << ' '
          << s.late_loads << ' ' << s.tuned_ms_x1000 << '\n';
}

void release_batch(Batch &b)
{
    if (b.dev)
        (void)hipFreeAsync(b.dev, b.stream);
    if (b.host.staging) {
        // The descriptors' copy and the kernel's result writes must be done
        // before the buffers serve another batch.
        if (hipStreamSynchronize(b.stream) == hipSuccess)
            return_host(b.host);
        else
            free_host(b.host);
    }
    b = Batch{};
}

}  // namespace

extern "C" {

int rp_batch_submit(const rp_batch_request *reqs, uint32_t count,
                    const rp_batch_schedule *sched, void *stream_,
                    uint64_t *batch_id)
{
    if (batch_id == nullptr || (reqs == nullptr && count > 0))
        return RP_EINVAL;
    rp_batch_schedule s;
    if (sched) {
        s = *sched;
    } else {
        std::lock_guard<std::mutex> lk(g_tmu);
        s = g_tuned ? g_tuned_sched : default_schedule();
    }
    Batch b;
    const int rc = launch_batch(reqs, count, s, reinterpret_cast<hipStream_t>(stream_), &b);
    if (rc != RP_OK) {
        release_batch(b);
        return rc;
    }
    std::lock_guard<std::mutex> lk(g_bmu);
    *batch_id = g_next_id++;
    g_batches[*batch_id] = b;
    return RP_OK;
}

int rp_batch_poll(uint64_t batch_id, uint32_t *n_done)
{
    std::lock_guard<std::mutex> lk(g_bmu);
    auto it = g_batches.find(batch_id);
    if (it == g_batches.end())
        return RP_EINVAL;
    const Batch &b = it->second;
    uint32_t d = 0;
    for (uint32_t i = 0; i < b.count; i++)
        d += __atomic_load_n(b.done + 1 + i, __ATOMIC_ACQUIRE) ? 1u : 0u;
    if (n_done)
        *n_done = d;
    return d >= b.count ? RP_OK : RP_PENDING;
}

int rp_batch_request_done(uint64_t batch_id, uint32_t index)
{
    std::lock_guard<std::mutex> lk(g_bmu);
    auto it = g_batches.find(batch_id);
    if (it == g_batches.end() || index >= it->second.count)
        return RP_EINVAL;
    return __atomic_load_n(it->second.done + 1 + index, __ATOMIC_ACQUIRE) ? RP_OK
                                                                           : RP_PENDING;
}

int rp_batch_results(uint64_t batch_id, rp_batch_result *out)
{
    Batch b;
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        auto it = g_batches.find(batch_id);
        if (it == g_batches.end())
            return RP_EINVAL;
        b = it->second;
    }
    if (hipStreamSynchronize(b.stream) != hipSuccess)
        return RP_EDEVICE;
    if (out)
        std::memcpy(out, b.res, sizeof(rp_batch_result) * b.count);
    return RP_OK;
}

int rp_batch_release(uint64_t batch_id)
{
    Batch b;
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        auto it = g_batches.find(batch_id);
        if (it == g_batches.end())
            return RP_EINVAL;
        b = it->second;
        g_batches.erase(it);
    }
    release_batch(b);
    return RP_OK;
}

int rp_batch_autotune(const rp_batch_request *reqs, uint32_t count, void *stream_,
                      rp_batch_schedule *out)
{
    if (reqs == nullptr || count == 0)
        return RP_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    for (uint32_t i = 0; i < count; i++)
        if (!valid_request(reqs[i]))
            return RP_EINVAL;
    // Sample: every request when the batch is small, else an evenly spaced
    // subset of the size-sorted batch (the same size mix), on scratch arrays
    // in seed mode so that the caller's arrays are never touched.
    std::vector<uint32_t> order(count);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t c) { return reqs[a].n > reqs[c].n; });
    const uint32_t want = std::min<uint32_t>(count, (uint32_t)env_or("RP_TUNE_SAMPLE", 512));
    std::vector<rp_batch_request> sample;
    uint64_t elems = 0;
    for (uint32_t i = 0; i < want; i++) {
        rp_batch_request q = reqs[order[(uint64_t)i * count / want]];
        q.H = nullptr;
        elems += q.n;
        sample.push_back(q);
    }
    const uint32_t eb = sample[0].elem_bytes;
    // A batch of this shape on this device was tuned before: take that.
    int dev = 0;
    (void)hipGetDevice(&dev);
    const std::string cache = tune_cache_path();
    const TuneShape shape = tune_shape(dev, sample);
    rp_batch_schedule known{};
    if (tune_lookup(cache, shape, &known)) {
        std::lock_guard<std::mutex> lk(g_tmu);
        g_tuned = true;
        g_tuned_sched = known;
        if (out)
            *out = known;
        return RP_OK;
    }
    void *scratch = nullptr;
    if (hipMalloc(&scratch, std::max<uint64_t>(elems * eb, 64)) != hipSuccess)
        return RP_ENOMEM;
    if (hipMemsetAsync(scratch, 0, std::max<uint64_t>(elems * eb, 64), stream) != hipSuccess) {
        (void)hipFree(scratch);
        return RP_EDEVICE;
    }
    uint64_t off = 0;
    for (auto &q : sample) {
        q.A = static_cast<unsigned char *>(scratch) + off * eb;
        off += q.n;
    }
    const uint32_t cutoffs[] = {1u << 10, 1u << 12, 1u << 14, 1u << 16, 1u << 18, 0xFFFFFFFFu};
    const uint32_t ratios[] = {12, 16, 24};
    struct Shape_ { uint32_t lanes, wpc; };
    const Shape_ shapes[] = {{256, 2}, {256, 4}, {256, 8}, {1024, 1}, {1024, 2}};
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best_ms = 1e30f;
    rp_batch_schedule best = default_schedule();
    for (uint32_t c : cutoffs)
        for (uint32_t r16 : ratios)
            for (const Shape_ &sh : shapes)
              for (uint32_t late = 0; late < 2; late++) {
                rp_batch_schedule s{};
                s.wave_cutoff = c;
                s.table_ratio_x16 = r16;
                s.workgroups_per_cu = sh.wpc;
                s.workgroup_lanes = sh.lanes;
                s.late_loads = late;
                float tot = 0.f;
                bool ok = true;
                for (int rep = 0; rep < 2 && ok; rep++) {
                    Batch b;
                    (void)hipEventRecord(e0, stream);
                    ok = launch_batch(sample.data(), (uint32_t)sample.size(), s, stream, &b) == RP_OK;
                    (void)hipEventRecord(e1, stream);
                    (void)hipEventSynchronize(e1);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (rep == 1)
                        tot = ms;  // the first run is a warm-up
                    release_batch(b);
                }
                if (ok && tot < best_ms) {
                    best_ms = tot;
                    best = s;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    best.tuned_ms_x1000 = (uint32_t)std::min<double>(4e9, best_ms * 1000.0);
    tune_store(cache, shape, best);
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        g_tuned = true;
        g_tuned_sched = best;
    }
    if (out)
        *out = best;
    return RP_OK;
}

}  // extern "C"
