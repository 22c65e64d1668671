/*
 * pi.h -- C ABI of the MI355X (gfx950) batched skip-list index.
 *
 * The index is the structure of "PI: a Parallel in-memory skip list based
 * Index" (Xie, Cai, Jagadish, Ooi, Wong): a storage layer (a key-ordered list
 * of data nodes, Definition 1) under an index layer (levels >= 2, each a
 * contiguous sorted key array, Section 3.1 and Section 4.1).  A batch of
 * search / insert / delete queries (Definition 2) is answered by the steps of
 * Algorithm 1: order the batch by key (Definition 3), descend the index layer
 * level by level for every query (Algorithm 2) to its interception
 * (Definition 4), give every storage node that will change exactly one owner
 * (the purpose of Algorithm 3), apply the changes without latches
 * (Algorithm 4, Section 3.2.4), and rebuild the index layer once enough
 * updates have accumulated (Section 4.1 and Section 4.3.5).
 *
 * Results are exactly those of applying the batch's queries one by one in
 * arrival order:
 *   SEARCH k    -> (PI_R_PRESENT, value of k) if k is present, else (PI_R_ABSENT, 0)
 *   INSERT k v  -> the same answer, then k maps to v
 *   DELETE k    -> the same answer, then k is absent
 *   op not in {0,1,2} or k == UINT64_MAX -> (PI_R_INVALID, 0), no effect
 * (the answers of INSERT and DELETE -- previous value if the key was live --
 * are this library's reading; the paper returns 1/null for delete.)
 *
 * Memory and streams.  Every pointer named d_* is DEVICE memory on the
 * index's device, owned by the caller; it must stay valid until the work
 * enqueued on the given stream has completed.  Inputs are only read.  All
 * device work is enqueued on the stream argument (a hipStream_t; NULL is the
 * null stream); calls that return host values synchronise that stream and say
 * so.  The library owns, allocates (hipMalloc) and frees its own device
 * memory.  A handle is not thread-safe: calls on one handle must be ordered by
 * the caller.
 *
 * Errors.  Every entry point returns a pi_status.  Argument and capacity
 * errors are detected on the host before anything is enqueued and leave the
 * index unchanged.  A failing HIP call marks the handle failed: every later
 * call returns PI_ERR_DEVICE.  pi_last_error() describes the last error.
 */
#ifndef PI_H
#define PI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pi_index pi_index; /* opaque; owns all device state */
typedef int32_t pi_status;
typedef void *pi_stream; /* a hipStream_t */

enum {
    PI_OK = 0,
    PI_ERR_INVALID_ARG = -1,
    PI_ERR_OUT_OF_MEMORY = -2,
    PI_ERR_STATE = -3,
    PI_ERR_DEVICE = -4,
    PI_ERR_CAPACITY = -5
};

/* query type t of Definition 2 */
enum { PI_OP_SEARCH = 0, PI_OP_INSERT = 1, PI_OP_DELETE = 2 };

/* per-query answer status */
enum { PI_R_ABSENT = 0, PI_R_PRESENT = 1, PI_R_INVALID = 255 };

/* Rebuild policies for the index layer (Section 4.3.5: rebuilt once the
 * number of insertions and deletions passes a threshold). */
enum {
    PI_REBUILD_THRESHOLD = 0, /* rebuild when changes >= fraction * live nodes */
    PI_REBUILD_NEVER = 1,     /* only pi_repair() rebuilds */
    PI_REBUILD_ALWAYS = 2,    /* rebuild after every batch that changed the structure */
    PI_REBUILD_BACKGROUND = 3, /* when changes >= fraction * live nodes, rebuild the index layer over the
                                 storage as it stands (new nodes included) on a second stream while
                                 batches go on, and switch to it at a batch boundary (Section 4.3.5);
                                 merge the storage itself (a full rebuild) only when the new and
                                 deleted nodes reach compact_percent of the base region.  Batch calls
                                 neither allocate nor free device memory under this policy (freeing
                                 waits for the whole device): the storage keeps room for new nodes
                                 up to that merge point, and the buffers of the background rebuild
                                 (about 88 bytes per storage slot) are reserved when the storage is
                                 loaded, merged or grown */
    PI_REBUILD_SLICES = 4     /* finer-grained repair (Section 7): the lower index levels are kept in
                                 per-key-range segments (slices of 4096 base slots) with room to grow;
                                 when changes >= fraction * live nodes, only the slices that received
                                 new nodes since the last round are rewritten in place (their keys
                                 merged with the new ones), and the small upper levels are rebuilt;
                                 a segment that would overflow, or new and deleted nodes reaching
                                 compact_percent of the base region, triggers a full rebuild that also
                                 merges the storage.  Runs on the caller's stream between batches */
};

typedef struct {
    uint32_t struct_size;     /* sizeof(pi_config) */
    int32_t device;           /* HIP device ordinal */
    uint32_t max_height;      /* cap on tower heights, 2..32 (default 24) */
    uint32_t log2_inv_p;      /* promotion probability p = 2^-log2_inv_p, 1..8 (default 1) */
    uint64_t height_seed;     /* seed of the height rule (default 0x9E3779B97F4A7C15) */
    float rebuild_fraction;   /* threshold as a fraction of live nodes (default 0.15) */
    uint32_t rebuild_policy;  /* PI_REBUILD_* (default PI_REBUILD_THRESHOLD) */
    uint64_t capacity_hint;   /* fixed storage capacity in nodes, counting the head and tail
                                 sentinels; 0 = grow on demand */
    uint32_t lds_levels;      /* index levels kept in LDS by the descent: 0 = auto */
    uint32_t profile;         /* 1 = time every stage with HIP events (pi_get_profile) */
    uint32_t queries_per_lane;/* descent: queries carried by one lane, 1, 2 or 4 (0 = 1) */
    uint32_t blocks_per_cu;   /* descent: cap on resident blocks per CU (0 = occupancy limit) */
    uint32_t lds_budget;      /* descent: index entries staged in LDS per block, <= 13000 (0 = 12000) */
    uint32_t descent_block;   /* descent: threads per block, 256, 512 or 1024 (0 = 1024) */
    uint32_t graph_max_log2;  /* batches of up to 2^graph_max_log2 queries replay a captured HIP graph of the
                                 hot path instead of ~26 launches; 12..22, 0 = never (default) */
    uint32_t small_batch_log2; /* batches of at most 2^small_batch_log2 queries run in one workgroup, one
                                 launch (0 = 10, i.e. 1024; 1..12; 255 = never) */
    uint32_t compact_percent; /* PI_REBUILD_BACKGROUND: full rebuild when new + deleted nodes reach this
                                 percentage of the base region (0 = 100, at most 1000); the storage
                                 keeps room for that many new nodes */
    uint64_t rebuild_min;     /* a threshold rebuild also needs at least this many changes (default 4096):
                                 an index of a few thousand keys is cheaper to walk than to rebuild */
    uint32_t check_writers;   /* 1 = checked mode of the single-writer invariant (Section 3.2.4): every
                                 storage write of a batch records its writer in a shadow word per node
                                 (8 bytes per storage slot); a node written by two different writers in
                                 one phase of a batch fails the handle with PI_ERR_DEVICE.  0 = off
                                 (default).  Not available with pi_execute_batch_noalloc */
    uint32_t post_form;       /* form of the steps after the descent (ownership hand-off of Algorithm 3's
                                 purpose, the updates of Algorithm 4): 0 = chosen per batch from the
                                 index's latest counters that reached the host (one launch after a batch
                                 without INSERT/DELETE, separate kernels after one with them; default),
                                 1 = always one launch, 2 = always separate kernels.  Results are the same
                                 in every form; under graph capture the kernels are always separate */
    uint32_t order_bits;      /* width of the position inside the batch's key span that the ordering sorts
                                 by (Definition 3's order, then fixed up by key inside equal positions):
                                 24, or 32 (one radix pass more, few equal positions left to fix up), or
                                 16 (one radix pass fewer; the descent then sorts each wave's 64 queries
                                 itself, which is all a batch without INSERT/DELETE needs for locality),
                                 or 0 = chosen per batch like post_form (16 after a batch without
                                 INSERT/DELETE, 24 after one with them; default).  Results are the same */
} pi_config;

/* Accumulated device time per stage of pi_execute_batch (profile = 1). */
typedef struct {
    uint64_t batches;         /* batches timed since the last reset */
    uint64_t rebuilds;        /* rebuilds timed since the last reset */
    double sort_ms;           /* ordering of the batch by key */
    double descend_ms;        /* index descent + storage walk (answers of read-only batches) */
    double own_ms;            /* ownership scan, answers, in-place updates */
    double link_ms;           /* allocation and linking of new nodes, counters */
    double rebuild_ms;        /* index-layer rebuilds */
} pi_profile;

typedef struct {
    uint64_t batches;         /* batches executed */
    uint64_t queries;         /* queries executed */
    uint64_t hits;            /* answers with status PRESENT */
    uint64_t invalid;         /* answers with status INVALID */
    uint64_t new_nodes;       /* storage nodes created by inserts */
    uint64_t deletes;         /* live -> deleted transitions */
    uint64_t revives;         /* deleted -> live transitions (insert on a flagged node) */
    uint64_t changes;         /* new nodes + live->deleted since the last rebuild */
    uint64_t repairs;         /* index-layer rebuilds */
    uint64_t live_nodes;      /* keys currently present */
    uint64_t base_nodes;      /* nodes in the sorted base region */
    uint64_t overflow_nodes;  /* nodes appended since the last rebuild */
    uint64_t capacity;        /* storage node capacity */
    uint32_t n_levels;        /* highest non-empty level (1 = no index levels) */
    uint32_t lds_from;        /* lowest level kept in LDS by the descent */
    uint64_t level_size[33];  /* keys on level l, l = 2..32 */
    uint64_t index_rebuilds;  /* background index-layer rebuilds switched in */
    uint64_t slice_rounds;    /* slice repair rounds (PI_REBUILD_SLICES) */
    uint64_t slices_repaired; /* slices rewritten over all rounds */
    uint64_t slices;          /* slices of the current layout (0: not sliced) */
} pi_stats;

/* Fills *cfg with the defaults listed above. */
pi_status pi_config_default(pi_config *cfg);

/* Creates an empty index on cfg->device (cfg NULL = defaults).  On success
 * *out receives the handle.  Errors: PI_ERR_INVALID_ARG (bad field or NULL
 * out), PI_ERR_DEVICE, PI_ERR_OUT_OF_MEMORY. */
pi_status pi_create(const pi_config *cfg, pi_index **out);

/* Frees every resource of the index (synchronises its device).  NULL is a
 * no-op. */
pi_status pi_destroy(pi_index *idx);

/* Bottom-up construction of an EMPTY index (Section 3.1: one scan of the
 * ordered data fills every index level).  d_keys/d_values: n pairs in device
 * memory, any order; a duplicated key keeps its LAST value (as if the pairs
 * were inserted in order); pairs whose key is UINT64_MAX are skipped.
 * Synchronises the stream.  Errors: PI_ERR_STATE if the index is not empty,
 * PI_ERR_INVALID_ARG (NULL with n > 0, n >= 2^31), PI_ERR_OUT_OF_MEMORY. */
pi_status pi_bulk_load(pi_index *idx, const uint64_t *d_keys, const uint64_t *d_values,
                       uint64_t n, pi_stream stream);

/* Answers a batch of n queries (Algorithm 1) and applies its updates.
 * d_ops u8[n] (PI_OP_*), d_keys u64[n], d_values u64[n] (read only for
 * INSERT queries, but always required), arrival order.
 * d_out_values u64[n], d_out_status u8[n] receive one answer per query in
 * arrival order.  Work is enqueued on the stream; the call does not wait for
 * it except when the storage must grow or the index layer is rebuilt (then it
 * synchronises).  n = 0 is a no-op.  Errors: PI_ERR_INVALID_ARG (NULL
 * pointers with n > 0, n >= 2^31), PI_ERR_CAPACITY (capacity_hint fixed and
 * too small for the worst case of this batch; nothing enqueued),
 * PI_ERR_OUT_OF_MEMORY, PI_ERR_DEVICE. */
pi_status pi_execute_batch(pi_index *idx, const uint8_t *d_ops, const uint64_t *d_keys,
                           const uint64_t *d_values, uint64_t n, uint64_t *d_out_values,
                           uint8_t *d_out_status, pi_stream stream);

/* pi_execute_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, answers and effect as pi_execute_batch, but
 * the call never allocates or frees memory: every per-batch buffer of the hot
 * path lives in one scratch array of 8 MiB that the library keeps per GPU for
 * the life of the process (its address is taken when the first index is
 * created on that GPU).  Limits: n <= 65536 (2^16) queries, else
 * PI_ERR_INVALID_ARG; the storage is never grown, so a batch whose new nodes
 * may not fit the free slots gets PI_ERR_CAPACITY with nothing enqueued; no
 * index rebuild runs inside this call (one that is due runs at the next
 * pi_execute_batch).  The scratch keeps the last call's contents and is
 * shared by every index of the GPU: calls of this function that overlap on
 * one GPU (other streams, other host threads) race and must be ordered by the
 * caller.  n = 0 is a no-op. */
pi_status pi_execute_batch_noalloc(pi_index *idx, const uint8_t *d_ops, const uint64_t *d_keys,
                                   const uint64_t *d_values, uint64_t n, uint64_t *d_out_values,
                                   uint8_t *d_out_status, pi_stream stream);

/* Rebuilds the storage base region and every index level now, whatever the
 * policy (Section 4.1: rebuild from the storage layer, bottom-up, drop
 * deleted nodes).  Synchronises the stream. */
pi_status pi_repair(pi_index *idx, pi_stream stream);

/* Writes the live (key, value) pairs in increasing key order into
 * d_keys/d_values (capacity cap pairs) and their number into *n_out (host).
 * Does not change the index.  Synchronises the stream.  Errors:
 * PI_ERR_CAPACITY when cap is too small (*n_out still receives the count). */
pi_status pi_export(pi_index *idx, uint64_t *d_keys, uint64_t *d_values, uint64_t cap,
                    uint64_t *n_out, pi_stream stream);

/* Range search: the range query of Section 3.2.5, for SEARCH.  Range i
 * holds every live (key, value) pair with d_lo[i] <= key <= d_hi[i]
 * (none when d_lo[i] > d_hi[i]), in increasing key order.  Two calls on the
 * same stream, with no batch or repair of this index in between:
 *
 *   pi_range_count   writes d_offsets u64[n + 1]: d_offsets[i] is the number
 *                    of pairs in ranges 0 .. i-1, d_offsets[n] the total.
 *   pi_range_collect writes range i's pairs to d_keys/d_values u64 at
 *                    [d_offsets[i], d_offsets[i+1]).  It never writes past
 *                    d_offsets[i+1]; if the index changed since the count,
 *                    a range may fill fewer entries than reserved.
 *
 * Inputs d_lo, d_hi u64[n] and d_offsets are device memory owned by the
 * caller, and d_lo, d_hi hold the same ranges in both calls; both calls are
 * asynchronous on the stream and do not change the index.  A collect that
 * follows the count of the same arrays with no other call on this index in
 * between reuses the count's ordering of the ranges and their
 * interceptions instead of computing them again.  n = 0 writes d_offsets[0] = 0.  Errors: PI_ERR_INVALID_ARG for
 * NULL pointers or n above 2^31 - 1. */
pi_status pi_range_count(pi_index *idx, const uint64_t *d_lo, const uint64_t *d_hi, uint64_t n,
                         uint64_t *d_offsets, pi_stream stream);
pi_status pi_range_collect(pi_index *idx, const uint64_t *d_lo, const uint64_t *d_hi, uint64_t n,
                           const uint64_t *d_offsets, uint64_t *d_keys, uint64_t *d_values, pi_stream stream);

/* Serving loop: continuous batching of an open-loop arrival schedule.
 *
 * Query i (arrays in arrival order, device memory as for pi_execute_batch)
 * arrives h_arrival_us[i] microseconds after the call starts (host array,
 * non-decreasing).  The loop admits arrived queries into a micro-batch that
 * closes deadline_us after its first query arrived, or as soon as it holds
 * max_batch queries; a closed micro-batch is enqueued as one pi_execute_batch
 * on the stream when fewer than max_inflight micro-batches are still running
 * on the device, and keeps admitting arrivals (up to max_batch) while it
 * waits for a slot; with no micro-batch on the device it is enqueued at once.  Micro-batches are contiguous runs of the arrival order
 * applied in that order, so every answer equals that of applying all n
 * queries one by one in arrival order (the serial semantics of
 * pi_execute_batch); the batching changes only when answers are ready.
 *
 * Outputs: d_out_values/d_out_status as for pi_execute_batch; h_done_us[i]
 * (host) = device completion time of query i's micro-batch, microseconds
 * since the call started; h_batch_end (host, capacity n) = end index of each
 * micro-batch, *n_batches of them.  Returns when every query is answered
 * (synchronises the stream).  Errors: PI_ERR_INVALID_ARG for NULL pointers,
 * a wrong struct_size, max_batch above 2^31 - 1, max_inflight above 64 or
 * decreasing arrival times; PI_ERR_CAPACITY when the index has a fixed
 * capacity_hint and the stream's INSERT queries could need more slots than
 * are free at the start.  These are checked before the first micro-batch and
 * leave the index unchanged.  An error met later (storage growth failing with
 * PI_ERR_OUT_OF_MEMORY, PI_ERR_DEVICE) stops the loop between micro-batches:
 * the micro-batches before it took effect, *n_batches and h_batch_end
 * describe them and their answers and h_done_us are written; no query after
 * them was applied. */
typedef struct {
    uint32_t struct_size;   /* sizeof(pi_serve_config) */
    uint32_t max_inflight;  /* micro-batches on the device at once (0 = 1: the host's ~26 launches per
                               micro-batch, not the device, bound the rate, and queued batches only
                               add latency) */
    double deadline_us;     /* micro-batch deadline after its first arrival (default 100) */
    uint64_t max_batch;     /* queries per micro-batch (0 = as many as free device memory allows, <= 2^22) */
} pi_serve_config;

pi_status pi_serve_config_default(pi_serve_config *cfg);
pi_status pi_serve(pi_index *idx, const pi_serve_config *cfg, const double *h_arrival_us, const uint8_t *d_ops,
                   const uint64_t *d_keys, const uint64_t *d_values, uint64_t n, uint64_t *d_out_values,
                   uint8_t *d_out_status, double *h_done_us, uint64_t *h_batch_end, uint64_t *n_batches,
                   pi_stream stream);

/* ---- many indices, one launch (batching form) ---------------------------
 *
 * A group runs one batch on each of several independent indices of one
 * device.  Batches of at most fused_max queries run in one persistent fused
 * launch: each workgroup takes the next (index, batch) from a work queue,
 * largest first, and runs the whole hot path for it (ordering, descent,
 * ownership, apply) in chunks of 4096 queries; larger batches take the
 * multi-kernel path of pi_execute_batch.  Every index's answers and final
 * state equal those of pi_execute_batch on that index alone.
 *
 * The counters of all indices are copied back once per call; threshold
 * rebuilds and storage growth are decided from that copy at the next call
 * (the host waits for the previous call's copy, so a group lags the device
 * by at most one call). */
typedef struct {
    const uint8_t *d_ops;       /* as for pi_execute_batch; n = 0 skips the index */
    const uint64_t *d_keys;
    const uint64_t *d_values;
    uint64_t n;
    uint64_t *d_out_values;
    uint8_t *d_out_status;
} pi_batch;

typedef struct pi_group pi_group; /* opaque: scratch and tuning of the fused launch */

typedef struct {
    uint32_t struct_size;  /* sizeof(pi_group_config) */
    uint32_t max_indices;  /* most indices per call (0 = 4096) */
    uint64_t fused_max;    /* largest batch run in the fused launch (0 = 4096) */
    uint32_t host_threads; /* host threads that issue the work of the indices
                            * with large batches or a rebuild due, each on a
                            * lane stream of its own (0 = 4, at most 4; 1 =
                            * everything from the calling thread) */
    uint32_t reserved;     /* must be 0 */
} pi_group_config;

pi_status pi_group_config_default(pi_group_config *cfg);
pi_status pi_group_create(const pi_group_config *cfg, pi_group **out);
/* Waits for the group's last call, then frees it (NULL ok). */
pi_status pi_group_destroy(pi_group *g);
/* Runs batches[i] on indices[i] for i < count, asynchronously on the stream:
 * batches of at most fused_max queries in one persistent fused launch on a
 * stream of the group's own, the others on the multi-kernel path spread over
 * four lane streams of the group, issued by host_threads host threads (the
 * calling one and workers that live for the call).  The rebuild policies of
 * the indices of the group's previous call act on its counters at this call:
 * for an index whose batch runs fused (or whose capacity is fixed) before
 * the fused launch; for one with a larger batch on its lane right before
 * that batch; for one without a batch in this call on a lane beside the
 * rest.  All of it is joined back into the caller's stream.  The indices
 * must be distinct, live on one device and not be used by other calls until
 * this one completes (nor, until then, the indices of the group's previous
 * call).  Errors: PI_ERR_INVALID_ARG (NULL pointers, count above
 * max_indices, a repeated index, mixed devices, n above 2^31 - 1),
 * PI_ERR_CAPACITY (an index with a fixed capacity has no room; nothing of
 * this call's batches is enqueued). */
pi_status pi_group_execute(pi_group *g, pi_index *const *indices, const pi_batch *batches, uint32_t count,
                           pi_stream stream);
/* Autotuner: replays the given batches as SEARCH-only (the indices' contents
 * do not change; their query counters do).  First under several fused_max
 * thresholds (the batch size that still runs in the fused launch): keeps the
 * fastest in the group and returns it in *fused_max (host).  Then, when some
 * batch exceeds it, under several descent shapes for the multi-kernel path
 * -- threads per workgroup (256/512/1024: the key range one workgroup's
 * tiles cover) with an LDS staging budget (3000..12000 entries) -- and sets
 * the fastest as descent_block and lds_budget of every given index.
 * Synchronises the stream. */
pi_status pi_group_autotune(pi_group *g, pi_index *const *indices, const pi_batch *batches, uint32_t count,
                            pi_stream stream, uint64_t *fused_max);
/* What the last autotune chose: the fused threshold, and the descent shape it
 * applied to the indices (0, 0 when it tried none).  Host pointers. */
pi_status pi_group_tuning(const pi_group *g, uint64_t *fused_max, uint32_t *descent_block, uint32_t *lds_budget);
/* Message of the last error of the group. */
const char *pi_group_last_error(const pi_group *g);

/* Copies the counters into *out (host).  Synchronises the index's device. */
pi_status pi_get_stats(pi_index *idx, pi_stats *out);

/* Copies the stage times accumulated since the last reset into *out (host)
 * and, when reset is nonzero, clears them.  All zero unless the index was
 * created with profile = 1.  Synchronises the index's device. */
pi_status pi_get_profile(pi_index *idx, pi_profile *out, int32_t reset);

/* Message of the last error on this handle ("" if none).  NULL handle gives
 * the message of the last pi_create failure. */
const char *pi_last_error(const pi_index *idx);

/* ---- inspection entry points used by the parity tests ------------------- */

/* Interception of every key (Definition 4) on the CURRENT index layer: the
 * largest key <= d_keys[i] among the keys of height > 1 that the index layer
 * holds.  d_icpt_keys u64[n] receives that key, d_is_head u8[n] receives 1
 * when there is none (the head of the list) and 0 otherwise. */
pi_status pi_debug_interceptions(pi_index *idx, const uint64_t *d_keys, uint64_t n,
                                 uint64_t *d_icpt_keys, uint8_t *d_is_head, pi_stream stream);

/* Copies level `level` (2..max_height) of the index layer: its keys in order
 * into d_keys (u64) and, for every key, the position of the same key on the
 * level below (level 2: the storage slot) into d_down (u32).  *n_out (host)
 * receives the number of keys.  Synchronises.  PI_ERR_CAPACITY if cap is too
 * small. */
pi_status pi_debug_level(pi_index *idx, uint32_t level, uint64_t *d_keys, uint32_t *d_down,
                         uint64_t cap, uint64_t *n_out, pi_stream stream);

/* Stable sort of n keys by value, as the batch's ordering step does it
 * (Definition 3; equal keys keep input order): d_sorted_keys u64[n] and
 * d_perm u32[n] (input position of each output).  Uses the index's
 * workspace. */
pi_status pi_debug_sort(pi_index *idx, const uint64_t *d_keys, uint64_t n,
                        uint64_t *d_sorted_keys, uint32_t *d_perm, pi_stream stream);

/* Self-test of the checked mode's detection (check_writers), on a private
 * two-word shadow rather than the storage: *same_writer_err receives the error
 * bits raised by one writer recording a node twice (must be 0), and
 * *two_writer_err those raised by two writers of one node in one phase (must
 * be nonzero).  Synchronises the stream.  Host pointers. */
pi_status pi_debug_writer_selftest(pi_index *idx, uint32_t *same_writer_err, uint32_t *two_writer_err,
                                   pi_stream stream);

/* Test hook: sets the host's upper bound on the storage slots in use, the
 * bound that decides whether a batch needs room checked before it is
 * enqueued.  A bound below the truth must never let a batch write past the
 * capacity: the kernels then drop that batch's new nodes, and the next call
 * that reads the counters fails the handle with PI_ERR_DEVICE.  Tests only. */
pi_status pi_debug_set_storage_bound(pi_index *idx, uint64_t used_upper);

#ifdef __cplusplus
}
#endif

#endif /* PI_H */
