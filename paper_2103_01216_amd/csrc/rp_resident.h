// rp_resident.h -- the resident serving kernel's request ring, as seen by the
// server (rp_serve.hip) that posts requests and by the kernel (rp.hip) that
// claims them.  Internal to the library; not part of the ABI.
//
// The host writes each request into the next entry of a ring in host memory
// and stores the entry's sequence number last; workgroups of the resident
// kernel claim entries in ring order.  A request runs either on one
// workgroup, with its round state in LDS, or on a gang of workgroups formed
// from idle ones, with its tables in device memory the server allocated with
// the request.  Completion is reported per ring slot in host memory.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rpres {

constexpr uint32_t RING = 4096;      // ring entries (a power of two)
constexpr uint32_t MAX_GANG = 4095;  // largest gang (12-bit fields)

constexpr uint32_t FILL_NONE = 0;      // the array already holds the input
constexpr uint32_t FILL_IDENTITY = 1;  // A[i] = i first (word 0 of a wider record)
constexpr uint32_t FILL_COPY = 2;      // copy n * eb bytes from src first

// One request as the host posts it (host memory; 128 bytes).
struct Entry {
    unsigned char *A;           // records, n * eb bytes (device memory)
    unsigned char *aux;         // gang: its round tables (device memory); else nullptr
    const void *src;            // FILL_COPY: the input (device or pinned host memory)
    uint64_t seed;              // H[i] = splitmix64(seed ^ i) mod (i + 1)
    uint64_t max_rounds;
    uint32_t n, eb;
    uint32_t k, T, bmw;         // one workgroup: its LDS plan; a gang: its table plan
    uint32_t gang;              // workgroups: 1, or the gang size
    uint32_t chunk_log2;        // gang: fresh indices are dealt in chunks of 2^this
    uint32_t rank_cap;          // gang: the refill throttle's rank limit
    uint32_t fill;              // FILL_*
    uint32_t aux_words;         // round-state words, reported back
    uint32_t pad[10];
    uint64_t seq;               // entry index + 1, stored last
};
static_assert(sizeof(Entry) == 128, "ring entry layout");

// What the device reports per ring slot (host memory; 64 bytes).
struct Result {
    uint64_t rounds, attempts;
    int32_t status;             // RP_OK, RP_ETIMEOUT, or RP_PENDING: the gang
                                // could not form in time and the request did
                                // not run (the array is untouched): post again
    uint32_t pad0;
    uint64_t started;           // seq of the entry once a workgroup claimed it
    uint64_t done;              // seq of the entry once the result is final
    uint64_t pad[3];
};
static_assert(sizeof(Result) == 64, "ring result layout");

// One launch of the resident kernel.
struct Launch {
    const Entry *ring;          // host memory, RING entries
    Result *res;                // host memory, RING results
    const uint32_t *stop;       // host memory: nonzero = leave once idle
    void *ctl;                  // device memory, rpint::resident_ctl_bytes()
    uint64_t first;             // the first entry index this launch serves
    uint64_t idle_ticks;        // leave after this long with nothing to claim (100 MHz)
    uint64_t form_ticks;        // a gang not formed by then is given back (RP_PENDING)
    uint32_t grid;              // workgroups
};

}  // namespace rpres

namespace rpint {

// Device bytes of the kernel's control block.
uint64_t resident_ctl_bytes();

// Workgroups of the resident kernel on `device`: one per compute unit.
int resident_grid(int device, uint32_t *grid);

// Plan one request into e (n, eb, k, T, bmw, gang, chunk_log2, rank_cap,
// max_rounds, aux_words): a gang of at most max_gang workgroups when
// allow_gang and the bound leaves room for its tables, else one workgroup.
// *aux_bytes: device bytes of the gang's tables (0 for one workgroup).
int resident_plan(uint64_t n, uint32_t eb, double eps, uint32_t max_gang, int device,
                  bool allow_gang, rpres::Entry *e, uint64_t *aux_bytes);

// Reset the control block and launch the kernel on `stream`.
int resident_launch(const rpres::Launch &L, hipStream_t stream);

}  // namespace rpint
