// Host-side state of one index and the operations of the library.
#pragma once

#include <algorithm>
#include <functional>
#include <vector>

#include "pi_internal.h"
#include "trace.h"

namespace pi {

// Storage layer (Definition 1, Section 4.1) as structure-of-arrays in HBM:
//   slot 0            head (key -infinity; never compared)
//   slots 1..nbase    base region, strictly increasing keys, successor of
//                     slot i is i+1 unless META_LINK is set
//   slot nbase+1      tail (key +infinity)
//   slots > nbase+1   nodes created by inserts since the last rebuild, one
//                     key-sorted run per batch, successor always in snext
struct Storage {
    uint64_t cap = 0;
    DevBuf all;                   // the one allocation
    DevBuf key, val, next, meta;  // views into it (never grown or freed on their own)
    // capacity of at least cap slots (exactly cap when exact)
    void alloc(uint64_t cap, bool exact);
    void release();
};

struct BatchWorkspace {
    DevBuf res_val, res_flags, loc, locnext, newflag, newpos, gw, agg;
    DevBuf part;       // per apply tile: hits, deletes, revives, new nodes (summed at the batch's end)
    DevBuf dpart;      // per descent block: hits, invalid queries (summed at the batch's end)
    static constexpr uint32_t DPART = 8192;  // count slots of the descent (its grid is at most this)
    DevBuf nk, nv, npred, npnext;
    DevBuf sop, svin;  // op and inserted value of each sorted query (batches with updates)
    uint64_t n = 0;
    void ensure(uint64_t n);
    void release();
};

// Stage timing with HIP events on the caller's stream (pi_config.profile).
struct Profiler {
    bool on = false;
    struct Rec {
        hipEvent_t e[5];
        int n;  // 5 = batch (begin, sorted, descended, owned, end); 2 = rebuild
    };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> pending;
    pi_profile acc{};
    hipEvent_t take();
    void drain(bool wait);  // folds completed records into acc
    void release();
};

// Sliced layout of the lower index levels (rebuild policy SLICES): slices of
// SL_B consecutive base slots; on levels 2..ls slice j owns entries
// [1 + j*cap[l], 1 + (j+1)*cap[l]) of the level (its keys, then a gap).
constexpr uint32_t SL_LOG = 12;
constexpr uint32_t SL_B = 1u << SL_LOG;
struct SliceLayout {
    uint32_t S;                  // slices
    int32_t ls;                  // highest sliced level
    uint32_t cap[MAX_LEVELS];    // entries per segment on level l <= ls
};

struct Index {
    pi_config cfg{};
    int device = 0;
    bool failed = false;
    std::string err;

    Storage st;
    Storage spare;                 // the previous storage, reused by the next rebuild
    uint64_t nbase = 0;        // base-region nodes
    uint64_t used_upper = 2;   // host upper bound of DevState::nused
    uint64_t batch_peak = 0;   // largest batch taken (queries), for the room a rebuild leaves
    // Queries enqueued on this index so far, by any path (single batches,
    // group calls, serving).  Every counter copy records the value at the
    // time it was enqueued, so nused in the copy plus the queries enqueued
    // since then (each adds at most one node) bounds nused now, whichever
    // path the later batches took.
    uint64_t enq_queries = 0;
    uint64_t live_at_rebuild = 0;
    uint64_t repairs = 0;

    DevBuf arena_key, arena_down;  // index levels
    IndexDesc desc{};

    DevState *dstate = nullptr;    // device
    DevState *hstate = nullptr;    // pinned host copy (blocking reads)
    // Counters after each of the last STATE_RING batches, copied to pinned
    // host memory behind an event: the threshold rebuild is decided from the
    // newest copy that has landed, and the host never runs more than
    // STATE_RING batches ahead of that decision.
    static constexpr int STATE_RING = 4;
    DevState *hring = nullptr;
    hipEvent_t ev_ring[STATE_RING] = {};
    uint64_t ring_enq[STATE_RING] = {};  // enq_queries when each copy was enqueued
    uint64_t ring_head = 0;        // copies enqueued
    bool recent_writers = false;   // the newest copy consumed was of a batch with INSERT/DELETE
    uint64_t ring_seen = 0;        // copies consumed (or dropped)

    SortWorkspace sortws;
    MsdWorkspace msdws;
    ScanWorkspace scanws;
    BatchWorkspace bws;
    // Serving with micro-batches in flight: the ordering of a micro-batch
    // runs on a side stream, beside the descent and updates of the one
    // before it on the caller's stream.  Two sets of batch buffers take
    // turns; `ordered` hands a set from the side stream to the caller's
    // stream, `done` hands it back.  Made on first use, kept until destroy.
    struct ServePipe {
        hipStream_t side = nullptr;
        hipEvent_t inputs = nullptr;  // the caller's stream at the start of a serve call
        struct Set {
            SortWorkspace sort;
            MsdWorkspace msd;
            ScanWorkspace scan;
            BatchWorkspace bws;
            hipEvent_t ordered = nullptr, done = nullptr;
            bool used = false;
        } set[2];
        int next = 0;
    } pipe;
    DevBuf tmp[10];                // rebuild / export scratch
    DevBuf rng[4];                 // range search: first node, end slot, counts, scan tiles
    // Bumped by every call that may change the storage or reuse the ordering
    // workspace.  rcache names the ranges whose order and interceptions the
    // workspaces hold (set by every range location); a range collect of the
    // same arrays in the same epoch reuses them.
    uint64_t epoch = 0;
    struct RangeCache {
        const uint64_t *lo = nullptr, *hi = nullptr;
        uint64_t n = 0, epoch = ~0ull;
        const uint64_t *slo = nullptr;
        const uint32_t *sperm = nullptr;
    } rcache;
    // captured hot path per batch-size class 2^c (queries padded with invalid
    // ones), valid while the buffers and launch parameters it was captured
    // with are unchanged
    struct Graph {
        hipGraphExec_t exec = nullptr;
        std::vector<uint64_t> fp;
    };
    Graph graphs[23];
    // background index rebuild (rebuild policy BACKGROUND)
    struct Background {
        int phase = 0;                 // 0 idle, 1 counting the new nodes, 2 building the levels
        hipStream_t side = nullptr;    // default priority, like every stream here
        hipEvent_t ev_main = nullptr, ev_side = nullptr;
        uint64_t first = 0, snap = 0;  // new nodes taken: storage slots [first, snap)
        uint64_t changes_at = 0, live_at = 0;
        SortWorkspace sortws;
        MsdWorkspace msdws;
        ScanWorkspace scanws;
        DevBuf okeys, flags, pos, cnt, b2key, b2slot, o2key, o2slot, m2key, m2slot, tcnt, ttot;
        DevBuf akey, adown;            // the levels being built; after the switch, the spare
        const uint64_t *sk = nullptr;  // the new keys in key order (in the side stream's sort workspace)
        const uint32_t *si = nullptr;  // ... and their positions in [first, snap)
        uint32_t *h_cnt = nullptr;     // pinned: new-node counts per level
        IndexDesc desc{};
        uint64_t done = 0;
    } bg;
    uint32_t base_level_n[MAX_LEVELS] = {};  // level sizes of the base region alone
    // slice repair (rebuild policy SLICES)
    struct Slices {
        bool on = false;
        SliceLayout lay{};
        DevBuf cnt;      // u32 [MAX_LEVELS][S]: keys of each segment
        DevBuf first;    // u64 [S]: first key of each slice (slice 0: 0)
        DevBuf dirty;    // u32 [S]: rewritten by the last round
        DevBuf offs, offs2, misc, ukey, upos, okeys, tcnt, ttot;
        SortWorkspace sortws;
        MsdWorkspace msdws;
        uint64_t round_first = 0;  // new nodes from this slot on are not indexed yet
        uint64_t rounds = 0, repaired = 0;
        uint64_t arena_used = 0;
        uint64_t real_n[MAX_LEVELS] = {};  // keys per level (without gaps)
    } slc;
    uint64_t changes_base = 0;     // DevState::changes when the index layer was last rebuilt
    DevBuf stage[5];               // graph inputs/outputs: ops, keys, values, answer values, answer status
    DevBuf owner;                  // writer-check shadow: u64 per storage slot (check_writers)
    uint32_t writer_unit = 0;      // writer-check units handed out
    hipStream_t cap_stream = nullptr;
    uint64_t *hcounts = nullptr;   // pinned: level totals etc.
    int num_cus = 256;
    Profiler prof;
};

}  // namespace pi

// The opaque handle of the C ABI.
struct pi_index {
    pi::Index ix;
};

namespace pi {

// Changes since the last rebuild that trigger the next one: the fraction of
// the live keys at the last rebuild (Section 4.3.5), at least rebuild_min.
inline double rebuild_threshold(const Index &ix) {
    const double frac = (double)ix.cfg.rebuild_fraction * (double)ix.live_at_rebuild;
    return std::max(std::max(1.0, frac), (double)ix.cfg.rebuild_min);
}

// build.hip
void init_empty(Index &ix, hipStream_t s);
void bulk_load(Index &ix, const uint64_t *keys, const uint64_t *vals, uint64_t n, hipStream_t s);
// merge + drop deleted + rebuild levels; known: the index's counters when the
// caller holds an exact copy (else they are read, a wait for the stream)
void rebuild(Index &ix, hipStream_t s, const DevState *known = nullptr);
uint64_t export_live(Index &ix, uint64_t *okeys, uint64_t *ovals, uint64_t cap, hipStream_t s);
void read_state(Index &ix, hipStream_t s, DevState *out);  // synchronises s
// Storage of at least need slots (the slots in use plus a batch), sized want
// when it has to be allocated; synchronises s.
void grow_storage(Index &ix, uint64_t need, uint64_t want, hipStream_t s);

// batch.hip
// The per-batch buffers of the multi-kernel path (the index's own, or ones
// taken from the no-allocation scratch).
struct BatchBuffers {
    SortWorkspace &sort;
    MsdWorkspace &msd;
    ScanWorkspace &scan;
    BatchWorkspace &bws;
};
void execute_batch(Index &ix, const uint8_t *ops, const uint64_t *keys, const uint64_t *vals, uint64_t n,
                   uint64_t *out_vals, uint8_t *out_status, hipStream_t s);
void execute_batch(Index &ix, const BatchBuffers &buf, const uint8_t *ops, const uint64_t *keys,
                   const uint64_t *vals, uint64_t n, uint64_t *out_vals, uint8_t *out_status, hipStream_t s);
// The two halves of execute_batch.  The ordering reads only the batch and
// writes only buf.sort / buf.msd, so it may run on another stream beside the
// steps of an earlier batch; finish_batch (the descent and everything after
// it, on s) must come after it.  prec: profiler record to complete, or null.
// pos_bits: the width of the ordering's range position (order_bits), which
// finish_batch must be told too (16: the descent sorts each wave's queries).
void order_batch(const BatchBuffers &buf, const uint8_t *ops, const uint64_t *keys, uint64_t n, hipStream_t so,
                 const uint64_t **sk, const uint32_t **sidx, uint32_t pos_bits);
void finish_batch(Index &ix, const BatchBuffers &buf, const uint64_t *sk, const uint32_t *sidx, const uint8_t *ops,
                  const uint64_t *vals, uint64_t n, uint64_t *out_vals, uint8_t *out_status, hipStream_t s,
                  Profiler::Rec *prec, uint32_t pos_bits);
// Width of the range position of a batch of n queries: pi_config::order_bits,
// or 16 after a batch without INSERT/DELETE (such a batch is ordered only for
// locality), and after one with them 24, or 32 above 2^20 queries (a full
// order is what the fix-up completes: about n^2 / 2^(bits+1) pairs of
// queries share a position, which costs more than a fourth radix pass once
// n passes 2^20).
uint32_t order_bits(const Index &ix, uint64_t n);
// Same result through a captured graph of the hot path for the smallest
// power-of-two class >= n (padding with invalid queries).
void execute_batch_graph(Index &ix, const uint8_t *ops, const uint64_t *keys, const uint64_t *vals, uint64_t n,
                         uint64_t *out_vals, uint8_t *out_status, hipStream_t s);
void release_graphs(Index &ix);

// The writer check of the next `units` batch units (an off check when
// check_writers is 0); sizes and clears the shadow when the storage grew.
WriterCheck writer_check(Index &ix, uint32_t units);
// Runs the check's detection on a private two-word shadow: error bits of one
// writer recording twice, and of two writers of one node (synchronises s).
bool writer_selftest(Index &ix, hipStream_t s, uint32_t *same_writer_err, uint32_t *two_writer_err);

// small.hip: the whole batch (n <= 4096) in one workgroup, one launch
void execute_batch_small(Index &ix, const uint8_t *ops, const uint64_t *keys, const uint64_t *vals, uint64_t n,
                         uint64_t *out_vals, uint8_t *out_status, hipStream_t s);
uint32_t small_batch_lds_bytes();
void debug_interceptions(Index &ix, const uint64_t *keys, uint64_t n, uint64_t *icpt_keys, uint8_t *is_head,
                         hipStream_t s);
// Number of valid INSERT queries of a batch (synchronises s); the counter is
// cnt (device, one word) when given, else index scratch.
uint64_t count_inserts(Index &ix, const uint8_t *ops, const uint64_t *keys, uint64_t n, hipStream_t s,
                       unsigned int *cnt = nullptr);

// noalloc.hip: the scratch array of the call that allocates nothing
void noalloc_init(int device);  // once per device, with that device current
uint8_t *noalloc_scratch(int device);
uint64_t noalloc_max_batch();
size_t noalloc_scratch_bytes();

// serve.hip
struct ServePlan {
    double deadline_us = 100.0;
    uint64_t max_batch = 1u << 22;
    uint32_t max_inflight = 4;
};
// Largest micro-batch that free device memory allows (at most 2^22).
uint64_t serve_batch_limit(uint32_t inflight);
// Replays the arrival schedule; launch(b, e) enqueues queries [b, e) on s.
// nb receives the number of micro-batches enqueued (their end indices in
// batch_end); when launch throws, the micro-batches before it have been
// waited for and stamped, nb counts them, and the error passes on.
void serve_loop(const double *arrival_us, uint64_t n, const ServePlan &plan, hipStream_t s,
                const std::function<void(uint64_t, uint64_t)> &launch, double *done_us, uint64_t *batch_end,
                uint64_t &nb);
// The side stream and events of Index::pipe (default priority), made once;
// the side stream then waits for what the caller's stream s holds so far.
void pipe_open(Index &ix, hipStream_t s);
void pipe_release(Index &ix);

// build.hip: level descriptor from sizes; level arrays from sorted keys
IndexDesc make_desc(const Index &ix, const uint32_t *level_n, uint64_t *arena_entries);
void select_lds_levels(const Index &ix, IndexDesc &d);
// Writes keys[0 .. n) into the levels first_level.. their towers reach; the
// down pointer on first_level is slots[i] (or 1 + i when slots is null).
void scatter_levels(const Index &ix, const uint64_t *keys, const uint32_t *slots, uint64_t n, const IndexDesc &d,
                    DevBuf &cnt, DevBuf &tot, DevBuf &akey, DevBuf &adown, hipStream_t s, uint32_t first_level = 2);
// Keys per level (height >= l) of keys[0 .. n) into level_n (synchronises).
void level_totals(Index &ix, const uint64_t *keys, uint64_t n, DevBuf &cnt, DevBuf &tot, uint32_t *level_n,
                  hipStream_t s);
// Head entries and +infinity pads of every level of d.
void pad_levels(Index &ix, const IndexDesc &d, hipStream_t s);

// slices.hip: slice repair (rebuild policy SLICES)
void slice_build(Index &ix, hipStream_t s);                 // full build of the sliced layout (synchronises)
bool slice_round(Index &ix, uint64_t snap, hipStream_t s);  // repair round; false: a segment would overflow
uint64_t slice_export_level(Index &ix, int l, uint64_t *okey, uint32_t *odown, uint64_t cap, hipStream_t s);
void slice_release(Index &ix);

// bgrebuild.hip: background index rebuild (rebuild policy BACKGROUND)
void bg_start(Index &ix, const DevState &latest, hipStream_t s);  // enqueues the counting step
void bg_advance(Index &ix);                                       // moves on when the side stream is done
void bg_quiesce(Index &ix);                                       // waits and drops a rebuild in flight
void bg_release(Index &ix);
// Sizes every buffer of the background rebuild for the storage capacity, so
// that none is reallocated (a device-wide wait) inside a batch call.
void bg_reserve(Index &ix);
uint64_t storage_room(const Index &ix, uint64_t live);
uint64_t arena_entries_for(uint64_t cap);
void scatter_reserve(DevBuf &cnt, DevBuf &tot, uint64_t n);

// range.hip
void range_count(Index &ix, const uint64_t *lo, const uint64_t *hi, uint64_t n, uint64_t *offsets, hipStream_t s);
void range_collect(Index &ix, const uint64_t *lo, const uint64_t *hi, uint64_t n, const uint64_t *offsets,
                   uint64_t *keys, uint64_t *vals, hipStream_t s);

}  // namespace pi
