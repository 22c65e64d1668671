// Internal definitions shared by the HIP translation units of libpi.
// gfx950 only: wave64, 160 KB LDS per CU, 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pi.h"

namespace pi {

constexpr uint64_t KEY_MAX = ~0ull;  // +infinity pad; never a valid query key
constexpr uint32_t HEAD_SLOT = 0;    // virtual head of the storage list (key -infinity)
constexpr int MAX_LEVELS = 33;       // level numbers 0..32 (levels 2..32 used)
constexpr uint32_t LEVEL_PAD = 16;   // +infinity entries after the last key of a level
constexpr uint64_t STORAGE_SLACK = 16;  // allocated storage slots beyond the capacity

// storage node flag bits (one byte per node)
constexpr uint8_t META_DEL = 1;   // F_del of Algorithm 4
constexpr uint8_t META_LINK = 2;  // successor is snext[] (else the next slot)

// ---------------------------------------------------------------------------
// Index-layer descriptor, passed to kernels by value.  Level l (2..top) has
// n[l] keys stored at entries off[l]+1 .. off[l]+n[l] of the level arena;
// entry off[l] is the head (its key is never compared; its down pointer is
// the head of the level below) and LEVEL_PAD +infinity entries follow.
struct IndexDesc {
    uint64_t off[MAX_LEVELS];
    uint32_t n[MAX_LEVELS];
    uint32_t lds_off[MAX_LEVELS];  // entry offset inside the LDS copy
    int32_t top;                   // highest non-empty level (1 = none)
    int32_t lds_from;              // levels >= lds_from are staged in LDS
    uint32_t lds_entries;          // entries staged (0 = none)
    uint32_t pad_;
};

// Device-resident counters.  Written only by kernels; the host reads a copy.
struct DevState {
    unsigned long long nused;    // first free storage slot
    unsigned long long n_live;   // live keys
    unsigned long long changes;  // new nodes + live->deleted since rebuild
    unsigned int has_links;      // some node has META_LINK set
    unsigned int has_dead;       // some node has META_DEL set
    // cumulative
    unsigned long long batches, queries, hits, invalid, new_nodes, deletes, revives;
    // current batch
    unsigned int b_writers;      // nonzero: the batch has INSERT/DELETE queries
    unsigned int b_new, b_deletes, b_revives, b_hits, b_invalid;
    unsigned int b_n;
    unsigned int b_pad;          // padding queries of a graph replay (not counted)
    unsigned int errors;         // ERR_* bits of internal consistency failures (must stay 0)
    unsigned int bar;            // grid barrier of the fused post-descent step (cleared per batch)
    unsigned int b_first;        // first storage slot of the batch's new nodes (fused step)
    // fused post-descent step, cleared per batch: blocks that joined (bit 31
    // once the window closed), their number once fixed (bit 31 = set), next
    // tile of the first phase
    unsigned int join, parts, tile_next;
};

// DevState::errors bits
constexpr unsigned int ERR_WALK = 1;      // a storage walk passed its bound (the list is malformed)
constexpr unsigned int ERR_CAPACITY = 2;  // new nodes would have passed the storage capacity (none written)
constexpr unsigned int ERR_WRITERS = 4;   // a storage node had two writers in one phase of a batch (checked mode)
constexpr unsigned int ERR_BARRIER = 8;   // a grid barrier outwaited its bound (blocks not co-resident)
constexpr unsigned int ERR_LIVE = 16;     // a rebuild's live flags disagree with the live counter

// Host message for DevState::errors (empty when 0).
inline std::string device_error_text(unsigned int e) {
    std::string m;
    if (e & ERR_WALK) m += "internal error: storage walk exceeded its bound";
    if (e & ERR_CAPACITY) m += std::string(m.empty() ? "" : "; ") +
                               "internal error: new nodes would pass the storage capacity (not written)";
    if (e & ERR_WRITERS) m += std::string(m.empty() ? "" : "; ") +
                              "internal error: a storage node had two writers in one phase of a batch";
    if (e & ERR_BARRIER) m += std::string(m.empty() ? "" : "; ") +
                              "internal error: a grid barrier did not complete";
    if (e & ERR_LIVE) m += std::string(m.empty() ? "" : "; ") +
                           "internal error: live flags disagree with the live counter";
    return m;
}

// Checked mode of the single-writer invariant (Section 3.2.4: after the
// hand-over every storage node that changes has exactly one writer).  Every
// storage write of a batch also records its writer in a shadow word per node:
// tag = (unit << 2) | phase, writer = the owning query's sorted position (the
// apply phase) or the new node's rank (the link phase).  A second, different
// writer of one node under one tag sets ERR_WRITERS.  The phases of a batch
// run one after the other (separate kernels, or separated by a workgroup
// barrier), so only writers within one phase could race.
struct WriterCheck {
    unsigned long long *owner;  // u64 per storage slot, null when the check is off
    uint32_t unit;              // batch (or workgroup chunk) number, < 2^30
    enum : uint32_t { APPLY = 1, LINK = 2 };
    __device__ __forceinline__ void note(uint32_t node, uint32_t phase, uint32_t who, unsigned int *errors) const {
        if (!owner) return;
        const uint32_t tag = (unit << 2) | phase;
        const unsigned long long want = ((unsigned long long)tag << 32) | who;
        unsigned long long old = owner[node];
        for (int i = 0; i < 64; i++) {  // a legal pattern needs one or two rounds
            if ((uint32_t)(old >> 32) == tag) {
                if ((uint32_t)old != who) atomicOr(errors, ERR_WRITERS);
                return;
            }
            const unsigned long long prev = atomicCAS(&owner[node], old, want);
            if (prev == old) return;
            old = prev;
        }
        atomicOr(errors, ERR_WRITERS);
    }
};

// ---------------------------------------------------------------------------
// wave64 helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t mask_rank(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Block-wide exclusive scan of one u32 per thread; NT threads (multiple of
// 64).  s_tmp must hold NT/64 + 1 words.  Returns the exclusive prefix and
// writes the block total to *total.  Contains __syncthreads().
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t x, uint32_t *s_tmp, uint32_t *total) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    uint32_t inc = wave_incl_scan_u32(x);
    if (lane_id() == 63) s_tmp[w] = inc;
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int i = 0; i < NW; i++) {
            uint32_t t = s_tmp[i];
            s_tmp[i] = run;
            run += t;
        }
        s_tmp[NW] = run;
    }
    __syncthreads();
    uint32_t r = s_tmp[w] + inc - x;
    *total = s_tmp[NW];
    __syncthreads();
    return r;
}

// XCD-aware mapping of a persistent block id to a contiguous chunk: blocks
// are dispatched round-robin over the 8 XCDs, so consecutive chunks (adjacent
// key ranges, which share index lines) go to blocks of the same XCD and its
// L2.  grid must be a multiple of 8 (or smaller than 8).
__device__ __forceinline__ uint32_t xcd_chunk(uint32_t b, uint32_t grid) {
    if (grid < 8 || (grid & 7)) return b;
    const uint32_t per = grid >> 3;
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// Height rule: z = key ^ seed; splitmix64 output finalizer (Steele, Lea,
// Flood, OOPSLA 2014); height = 1 + min(ctz(z) / log2_inv_p, max_height-1),
// with ctz(0) = 64.  P(height >= h) = p^(h-1), the geometric law of the
// paper's tower heights (Section 3.2), but a pure function of the key.
__device__ __forceinline__ uint32_t tower_height(uint64_t key, uint64_t seed, uint32_t log2_inv_p,
                                                 uint32_t max_height) {
    uint64_t z = key ^ seed;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    uint32_t tz = z ? (uint32_t)__builtin_ctzll(z) : 64u;
    uint32_t extra = tz / log2_inv_p;
    if (extra > max_height - 1) extra = max_height - 1;
    return 1 + extra;
}

// Key -> position of `bits` bits (24 or 32, or 16 for a batch ordered only
// for locality) inside the batch's key span [lo, ...]: the top significant
// bits of key - lo (keys below lo map to 0, above the span to the largest
// position).  Monotone in the key, so ordering by it, then by key among equal
// positions, orders by key.
struct RangeMap {
    uint64_t lo;
    uint32_t shift;
    uint32_t top;  // largest position, 2^bits - 1
};

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
    const uint32_t lo = __shfl_xor((uint32_t)x, m, 64), hi = __shfl_xor((uint32_t)(x >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Map of the span [lo, hi] of a batch's valid keys (lo > hi: no valid key)
// onto positions of `bits` bits.
__device__ __forceinline__ RangeMap span_map(uint64_t lo, uint64_t hi, uint32_t bits) {
    if (lo > hi) lo = hi = 0;
    const uint64_t span = hi - lo;
    uint32_t sbits = 0;
    while (sbits < 64 && (span >> sbits) != 0) sbits++;
    RangeMap m;
    m.lo = lo;
    m.shift = sbits > bits ? sbits - bits : 0;
    m.top = (uint32_t)((1ull << bits) - 1);
    return m;
}

__device__ __forceinline__ uint32_t range_pos(uint64_t k, const RangeMap &m) {
    if (k <= m.lo) return 0;
    const uint64_t r = (k - m.lo) >> m.shift;
    return r > m.top ? m.top : (uint32_t)r;
}

// ---------------------------------------------------------------------------
// host-side helpers

struct Error {
    pi_status code;
    std::string msg;
};

#define PI_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::pi::Error{PI_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define PI_LAUNCH_CHECK() PI_HIP(hipGetLastError())

// Memory a DevBuf takes its bytes from instead of hipMalloc while an
// ArenaScope is active on the calling thread (the call that allocates
// nothing): bump allocation from a fixed range, never freed.  With base
// null it only counts the bytes asked for.
struct Arena {
    uint8_t *base;
    size_t cap;
    size_t used;
};
extern thread_local Arena *t_arena;
struct ArenaScope {
    Arena *prev;
    explicit ArenaScope(Arena *a) : prev(t_arena) { t_arena = a; }
    ~ArenaScope() { t_arena = prev; }
};

// While a DeferFrees is active on the calling thread, the device buffers
// that DevBufs release (a regrow, a release) go to its list instead of
// hipFree, which waits for the whole device: its owner frees them once the
// work that may still read them has completed.
extern thread_local std::vector<void *> *t_defer;
struct DeferFrees {
    std::vector<void *> *prev;
    explicit DeferFrees(std::vector<void *> *l) : prev(t_defer) { t_defer = l; }
    ~DeferFrees() { t_defer = prev; }
};

// A device buffer that only grows.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void ensure(size_t need);
    void release();
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

// ---- sort (sort.hip) ------------------------------------------------------
struct SortWorkspace {
    DevBuf keys[2], idx[2], tile_hist, digit_tot;
    void ensure(uint64_t n);
    void release();
};
// Stable LSD radix sort of keys (payload = input position).  When ops is not
// null, keys whose op is > 2 sort as KEY_MAX, and *writers (when not null) is
// set nonzero when there is a valid INSERT/DELETE query.  Returns pointers
// into the workspace.
void sort_keys_with_index(SortWorkspace &ws, const uint64_t *keys, const uint8_t *ops, uint64_t n,
                          unsigned int *writers, hipStream_t s, const uint64_t **out_keys,
                          const uint32_t **out_idx);
// Same, with an explicit u32 payload.
void sort_pairs(SortWorkspace &ws, const uint64_t *keys, const uint32_t *payload, uint64_t n,
                hipStream_t s, const uint64_t **out_keys, const uint32_t **out_payload);

// Ordering of a query batch: partition by key range, then order inside each
// range (msd.hip).  Same contract as sort_keys_with_index.  With batch set,
// the workspace's writers flag (MsdWorkspace::wflag) is cleared and then set
// when there is a valid INSERT/DELETE query, and a batch without any stops at
// the grouping by range position (its order only serves locality).  Touches
// nothing of the index, so that it may run beside another batch's steps.
struct MsdWorkspace {
    DevBuf partials, map, big, nbig, dirty, wflag;
    void ensure(uint64_t n);
    void release();
};
// pos_bits (16, 24 or 32; 0: 24 up to 2^20 keys, else 32): the width of the
// range position, one radix pass per byte.  16 orders by key only to 1/65536
// of the span before the in-group fix-up, which is all a batch without
// INSERT/DELETE needs (its order serves locality; the descent then sorts each
// wave's queries itself).  The wider the position, the fewer keys share one
// and the less the fix-up has to sort.
void sort_batch_by_range(SortWorkspace &ws, MsdWorkspace &mw, const uint64_t *keys, const uint8_t *ops, uint64_t n,
                         bool batch, hipStream_t s, const uint64_t **out_keys, const uint32_t **out_idx,
                         uint32_t pos_bits = 0);

// One stable 8-bit LSD pass (hist, column scan, scatter).  The digit is
// (key >> shift) & 255, or, when map is not null, (range_pos(key) >> shift)
// & 255.  idx_in null = input positions; ops not null = keys whose op is
// invalid count as KEY_MAX, and *writers (when not null) is set when there is
// an INSERT/DELETE query.
void radix_pass(SortWorkspace &ws, const uint64_t *kin, const uint32_t *iin, const uint8_t *ops, uint32_t n,
                uint32_t shift, const RangeMap *map, unsigned int *writers, uint64_t *kout, uint32_t *iout,
                hipStream_t s);

// Exclusive scan of each of ncols columns of length len stored back to back
// (column c at cols + c*len); totals[c] receives the column sum.
void column_scan(uint32_t *cols, uint32_t ncols, uint32_t len, uint32_t *totals, hipStream_t s);

// ---- scan (scan.hip) ------------------------------------------------------
struct ScanWorkspace {
    DevBuf tiles;
    void ensure(uint64_t n);
    void release();
};
// out[i] = sum of in[0..i) ; *d_total = sum of all (device u32).  When
// d_enable is not null and *d_enable == 0 the kernels do nothing.
void exclusive_scan_u32(ScanWorkspace &ws, const uint32_t *in, uint32_t *out, uint64_t n,
                        uint32_t *d_total, const unsigned int *d_enable, hipStream_t s);
// Same over the live flags of the base region: out[i] (i = 0 .. nbase) =
// number of slots 1 .. i that are not flagged deleted, from the node flags of
// slot 1 onwards; *d_total = the live count.
void exclusive_scan_live(ScanWorkspace &ws, const uint8_t *meta_slot1, uint64_t nbase, uint32_t *out,
                         uint32_t *d_total, hipStream_t s);

}  // namespace pi
