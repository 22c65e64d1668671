// The scratch array of pi_execute_batch_noalloc: the batch step for callers
// that cannot allocate device memory (graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// Every per-batch buffer of the multi-kernel path (ordering, descent
// results, ownership scan, new-node staging) is carved from one file-scope
// device array instead of the index's own workspaces.  The array exists once
// per GPU for the life of the process; host code never uses its name as an
// address, only the pointer hipGetSymbolAddress returns for the current
// device, taken once per device when an index is created there.
#include <mutex>

#include "index.h"

namespace pi {
namespace {

constexpr size_t SCRATCH_BYTES = size_t(8) << 20;  // 8 MiB per GPU
constexpr uint64_t MAX_BATCH = 1u << 16;            // queries per call
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

std::mutex g_mu;
uint8_t *g_ptr[MAX_DEVICES] = {};

}  // namespace

// Bytes the workspaces of a MAX_BATCH-query batch take from an arena (a
// counting arena: nothing is allocated or written).
static size_t workspace_bytes() {
    Arena count{nullptr, ~size_t(0), 0};
    ArenaScope scope(&count);
    SortWorkspace sw;
    MsdWorkspace mw;
    ScanWorkspace cw;
    BatchWorkspace bw;
    sw.ensure(MAX_BATCH);
    mw.ensure(MAX_BATCH);
    cw.ensure(MAX_BATCH);
    bw.ensure(MAX_BATCH);
    return count.used;
}

void noalloc_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) throw Error{PI_ERR_INVALID_ARG, "device ordinal out of range"};
    std::lock_guard<std::mutex> g(g_mu);
    if (g_ptr[device]) return;
    // the largest batch must fit (256 bytes at the start hold the insert count)
    if (workspace_bytes() + 256 > SCRATCH_BYTES) throw Error{PI_ERR_DEVICE, "internal error: scratch too small"};
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        throw Error{PI_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    }
    g_ptr[device] = static_cast<uint8_t *>(p);
}

uint8_t *noalloc_scratch(int device) {
    std::lock_guard<std::mutex> g(g_mu);
    uint8_t *p = device >= 0 && device < MAX_DEVICES ? g_ptr[device] : nullptr;
    if (!p) throw Error{PI_ERR_STATE, "no scratch address for this device (no index was created on it)"};
    return p;
}

uint64_t noalloc_max_batch() { return MAX_BATCH; }
size_t noalloc_scratch_bytes() { return SCRATCH_BYTES; }

}  // namespace pi
