// C ABI of libpi (declared in include/pi.h): argument checks, device
// selection, storage capacity, the rebuild policy and error reporting.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "index.h"


namespace pi {

thread_local Arena *t_arena = nullptr;
thread_local std::vector<void *> *t_defer = nullptr;

void DevBuf::ensure(size_t need) {
    if (need <= bytes && p) return;
    if (t_arena) {
        // the caller's fixed range: no device allocation, nothing freed
        const size_t off = (t_arena->used + 255) & ~size_t(255);
        if (off + need > t_arena->cap)
            throw Error{PI_ERR_INVALID_ARG, "scratch of " + std::to_string(t_arena->cap) + " bytes too small"};
        p = reinterpret_cast<void *>(reinterpret_cast<uintptr_t>(t_arena->base) + off);
        bytes = need;
        t_arena->used = off + need;
        return;
    }
    // Buffers up to 16 MiB (batch workspaces, the storage of small indices)
    // take the next power of two, so sizes that vary from call to call
    // reallocate at most once per doubling; a larger buffer is allocated as
    // asked the first time and gets half as much again when it has to grow.
    const bool regrow = p != nullptr;
    if (p) {
        if (t_defer)
            t_defer->push_back(p);
        else
            PI_HIP(hipFree(p));
        p = nullptr;
        bytes = 0;
    }
    constexpr size_t POW2_MAX = size_t(16) << 20;
    size_t b = 256;
    if (need <= POW2_MAX)
        while (b < need) b <<= 1;
    else
        b = regrow ? need + need / 2 : need;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, b);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{PI_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(b) + " bytes failed"};
    }
    p = q;
    bytes = b;
}

void DevBuf::release() {
    if (p && t_defer)
        t_defer->push_back(p);
    else if (p)
        (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

}  // namespace pi

namespace {

std::mutex g_create_err_mu;
std::string g_create_err;

constexpr uint64_t MAX_BATCH = (1ull << 31) - 1;

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) PI_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// keeps_state: the call changes neither the storage nor the ordering
// workspace (a range collect, a counter read), so a cached range location
// stays valid across it.
template <class F>
pi_status guarded(pi_index *h, F &&f, bool keeps_state = false) {
    if (!h) return PI_ERR_INVALID_ARG;
    pi::Index &ix = h->ix;
    if (ix.failed) return PI_ERR_DEVICE;
    if (!keeps_state) ix.epoch++;
    try {
        DeviceGuard g(ix.device);
        pi_status r = f(ix);
        if (r == PI_OK) ix.err.clear();
        return r;
    } catch (const pi::Error &e) {
        ix.err = e.msg;
        if (e.code == PI_ERR_DEVICE) ix.failed = true;
        return e.code;
    } catch (const std::exception &e) {
        ix.err = e.what();
        ix.failed = true;
        return PI_ERR_DEVICE;
    }
}

pi_status fail(pi::Index &ix, pi_status code, const char *msg) {
    ix.err = msg;
    return code;
}

void release_all(pi::Index &ix) {
    ix.st.release();
    ix.spare.release();
    ix.arena_key.release();
    ix.arena_down.release();
    ix.sortws.release();
    ix.msdws.release();
    ix.scanws.release();
    ix.bws.release();
    for (auto &b : ix.tmp) b.release();
    for (auto &b : ix.rng) b.release();
    pi::release_graphs(ix);
    pi::pipe_release(ix);
    pi::bg_release(ix);
    pi::slice_release(ix);
    ix.owner.release();
    if (ix.dstate) (void)hipFree(ix.dstate);
    if (ix.hstate) (void)hipHostFree(ix.hstate);
    if (ix.hcounts) (void)hipHostFree(ix.hcounts);
    if (ix.hring) (void)hipHostFree(ix.hring);
    for (auto &e : ix.ev_ring)
        if (e) (void)hipEventDestroy(e);
    ix.prof.release();
    ix.dstate = nullptr;
    ix.hstate = nullptr;
    ix.hcounts = nullptr;
    ix.hring = nullptr;
    for (auto &e : ix.ev_ring) e = nullptr;
}

// Threshold rebuild (Section 4.3.5, 15 % by default) decided from the newest
// counters that have reached the host.  A copy that has not landed is waited
// for only when STATE_RING batches are queued behind it, so the decision
// lags the device by at most that many batches and the GPU queue never runs
// dry because of it.
void maybe_rebuild(pi::Index &ix, hipStream_t s, bool may_rebuild = true) {
    const uint32_t pol = ix.cfg.rebuild_policy;
    // only the threshold and background policies decide from the counters;
    // the others (and a call that may not allocate, which a rebuild does)
    // read the copies that have landed (device errors, the storage bound)
    // and never wait for one
    const bool decides = may_rebuild && (pol == PI_REBUILD_THRESHOLD || pol == PI_REBUILD_BACKGROUND ||
                                         pol == PI_REBUILD_SLICES);
    if (may_rebuild && pol == PI_REBUILD_BACKGROUND) pi::bg_advance(ix);
    bool have = false;
    pi::DevState latest{};
    uint64_t latest_enq = 0;
    while (ix.ring_seen < ix.ring_head) {
        const int slot = (int)(ix.ring_seen % pi::Index::STATE_RING);
        const bool full = ix.ring_head - ix.ring_seen >= (uint64_t)pi::Index::STATE_RING;
        if (full && decides) {
            PI_HIP(hipEventSynchronize(ix.ev_ring[slot]));
        } else if (hipEventQuery(ix.ev_ring[slot]) != hipSuccess) {
            (void)hipGetLastError();
            if (full) {  // the slot is about to be reused: drop the copy unread
                ix.ring_seen++;
                continue;
            }
            break;
        }
        latest = ix.hring[slot];
        latest_enq = ix.ring_enq[slot];
        have = true;
        ix.ring_seen++;
        ix.recent_writers = latest.b_writers != 0;
        if (latest.errors) throw pi::Error{PI_ERR_DEVICE, pi::device_error_text(latest.errors)};
    }
    if (!have) return;
    // a tighter bound on the storage in use: the counters of the copy plus
    // every query enqueued on the index after it, whatever path took them
    ix.used_upper = std::min<uint64_t>(ix.used_upper, latest.nused + (ix.enq_queries - latest_enq));
    if (!decides) return;
    const double thr = pi::rebuild_threshold(ix);
    if (pol == PI_REBUILD_THRESHOLD) {
        if ((double)latest.changes >= thr) {
            pi::rebuild(ix, s);
            ix.ring_seen = ix.ring_head;  // copies taken before the rebuild are stale
        }
        return;
    }
    // background and slices: merge the storage when new and deleted nodes
    // have piled up, else rebuild the index layer beside the batches, or
    // repair the slices that changed
    const double compact = (ix.cfg.compact_percent ? ix.cfg.compact_percent : 100) / 100.0 *
                           (double)std::max<uint64_t>(ix.nbase, 1);
    if ((double)latest.changes >= std::max(compact, thr)) {
        pi::rebuild(ix, s);
        ix.ring_seen = ix.ring_head;
        return;
    }
    if (latest.changes >= ix.changes_base && (double)(latest.changes - ix.changes_base) >= thr) {
        if (pol == PI_REBUILD_BACKGROUND) {
            pi::bg_start(ix, latest, s);
        } else if (pi::slice_round(ix, latest.nused, s)) {
            ix.changes_base = latest.changes;
        } else {  // a segment would overflow: rebuild everything
            pi::rebuild(ix, s);
            ix.ring_seen = ix.ring_head;
        }
    }
}

// Queues the copy of the counters after a batch.
void push_state(pi::Index &ix, hipStream_t s) {
    const int slot = (int)(ix.ring_head % pi::Index::STATE_RING);
    ix.ring_enq[slot] = ix.enq_queries;
    PI_HIP(hipMemcpyAsync(ix.hring + slot, ix.dstate, sizeof(pi::DevState), hipMemcpyDeviceToHost, s));
    PI_HIP(hipEventRecord(ix.ev_ring[slot], s));
    ix.ring_head++;
}

void ensure_capacity(pi::Index &ix, const uint8_t *ops, const uint64_t *keys, uint64_t n, hipStream_t s) {
    ix.batch_peak = std::max(ix.batch_peak, n);
    if (ix.used_upper + n <= ix.st.cap) return;
    pi::DevState cur;
    pi::read_state(ix, s, &cur);  // refreshes used_upper
    if (cur.nused + n <= ix.st.cap) return;
    if (ix.cfg.capacity_hint) {
        const uint64_t ins = pi::count_inserts(ix, ops, keys, n, s);
        if (cur.nused + ins > ix.st.cap)
            throw pi::Error{PI_ERR_CAPACITY, "batch may need " + std::to_string(ins) + " new nodes; " +
                                                 std::to_string(ix.st.cap - cur.nused) + " slots free"};
        return;
    }
    // room for two batches of this size: batch sizes that vary do not force a
    // counter read (a wait for the stream) on every call
    pi::grow_storage(ix, cur.nused + n, std::max<uint64_t>(cur.nused + 2 * n, ix.st.cap * 2), s);
}

}  // namespace

extern "C" {

pi_status pi_serve_config_default(pi_serve_config *cfg) {
    if (!cfg) return PI_ERR_INVALID_ARG;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->struct_size = sizeof(pi_serve_config);
    cfg->max_inflight = 1;
    cfg->deadline_us = 100.0;
    cfg->max_batch = 0;
    return PI_OK;
}

pi_status pi_config_default(pi_config *cfg) {
    if (!cfg) return PI_ERR_INVALID_ARG;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->struct_size = sizeof(pi_config);
    cfg->device = 0;
    cfg->max_height = 24;
    cfg->log2_inv_p = 1;
    cfg->height_seed = 0x9E3779B97F4A7C15ull;
    cfg->rebuild_fraction = 0.15f;
    cfg->rebuild_min = 4096;
    cfg->rebuild_policy = PI_REBUILD_THRESHOLD;
    cfg->capacity_hint = 0;
    cfg->lds_levels = 0;
    cfg->profile = 0;
    cfg->queries_per_lane = 0;
    cfg->blocks_per_cu = 0;
    cfg->lds_budget = 0;
    cfg->descent_block = 0;
    cfg->graph_max_log2 = 0;
    cfg->small_batch_log2 = 0;
    return PI_OK;
}

pi_status pi_create(const pi_config *cfg_in, pi_index **out) {
    auto set_err = [](const std::string &m) {
        std::lock_guard<std::mutex> g(g_create_err_mu);
        g_create_err = m;
    };
    if (!out) {
        set_err("out is NULL");
        return PI_ERR_INVALID_ARG;
    }
    *out = nullptr;
    pi_config cfg;
    pi_config_default(&cfg);
    if (cfg_in) {
        if (cfg_in->struct_size != sizeof(pi_config)) {
            set_err("pi_config.struct_size mismatch");
            return PI_ERR_INVALID_ARG;
        }
        cfg = *cfg_in;
    }
    if (cfg.max_height < 2 || cfg.max_height > 32 || cfg.log2_inv_p < 1 || cfg.log2_inv_p > 8 ||
        !(cfg.rebuild_fraction >= 0.0f) || cfg.rebuild_policy > PI_REBUILD_SLICES ||
        cfg.capacity_hint > (1ull << 32) - 64 ||
        (cfg.queries_per_lane != 0 && cfg.queries_per_lane != 1 && cfg.queries_per_lane != 2 &&
         cfg.queries_per_lane != 4) ||
        cfg.lds_budget > 13000 ||
        (cfg.descent_block != 0 && cfg.descent_block != 256 && cfg.descent_block != 512 &&
         cfg.descent_block != 1024) ||
        (cfg.graph_max_log2 != 0 && (cfg.graph_max_log2 < 12 || cfg.graph_max_log2 > 22)) ||
        (cfg.small_batch_log2 > 12 && cfg.small_batch_log2 != 255) || cfg.compact_percent > 1000 ||
        cfg.check_writers > 1 || cfg.post_form > 2 ||
        (cfg.order_bits != 0 && cfg.order_bits != 16 && cfg.order_bits != 24 && cfg.order_bits != 32)) {
        set_err("invalid pi_config field");
        return PI_ERR_INVALID_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg.device < 0 || cfg.device >= ndev) {
        (void)hipGetLastError();
        set_err("no such HIP device");
        return PI_ERR_INVALID_ARG;
    }
    pi_index *h = new (std::nothrow) pi_index;
    if (!h) return PI_ERR_OUT_OF_MEMORY;
    pi::Index &ix = h->ix;
    ix.cfg = cfg;
    ix.device = cfg.device;
    ix.prof.on = cfg.profile != 0;
    try {
        DeviceGuard g(ix.device);
        hipDeviceProp_t prop;
        PI_HIP(hipGetDeviceProperties(&prop, ix.device));
        ix.num_cus = prop.multiProcessorCount;
        PI_HIP(hipMalloc(&ix.dstate, sizeof(pi::DevState)));
        PI_HIP(hipHostMalloc(&ix.hstate, sizeof(pi::DevState), hipHostMallocDefault));
        PI_HIP(hipHostMalloc(&ix.hcounts, 256 * sizeof(uint64_t), hipHostMallocDefault));
        PI_HIP(hipHostMalloc(&ix.hring, pi::Index::STATE_RING * sizeof(pi::DevState), hipHostMallocDefault));
        for (auto &e : ix.ev_ring) PI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        std::memset(ix.hstate, 0, sizeof(pi::DevState));
        std::memset(ix.hring, 0, pi::Index::STATE_RING * sizeof(pi::DevState));
        const uint64_t cap = std::max<uint64_t>(cfg.capacity_hint ? cfg.capacity_hint : (1u << 16), 4);
        ix.st.alloc(cap, cfg.capacity_hint != 0);
        pi::noalloc_init(ix.device);
        pi::init_empty(ix, nullptr);
        PI_HIP(hipDeviceSynchronize());
    } catch (const pi::Error &e) {
        set_err(e.msg);
        release_all(ix);
        delete h;
        return e.code;
    }
    *out = h;
    return PI_OK;
}

pi_status pi_destroy(pi_index *h) {
    if (!h) return PI_OK;
    {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(h->ix.device);
        (void)hipDeviceSynchronize();
        release_all(h->ix);
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    delete h;
    return PI_OK;
}

pi_status pi_bulk_load(pi_index *h, const uint64_t *d_keys, const uint64_t *d_values, uint64_t n, pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (n > MAX_BATCH) return fail(ix, PI_ERR_INVALID_ARG, "n too large");
        if (n > 0 && (!d_keys || !d_values)) return fail(ix, PI_ERR_INVALID_ARG, "NULL input");
        hipStream_t s = (hipStream_t)stream;
        pi::DevState cur;
        pi::read_state(ix, s, &cur);
        if (cur.n_live != 0 || cur.nused != ix.nbase + 2 || ix.nbase != 0)
            return fail(ix, PI_ERR_STATE, "bulk load needs an empty index");
        pi::bulk_load(ix, d_keys, d_values, n, s);
        ix.ring_seen = ix.ring_head;
        return PI_OK;
    });
}

// One batch: the rebuild decision, room for the batch's new nodes, the hot
// path, the queued counter copy.
void batch_step(pi::Index &ix, const uint8_t *d_ops, const uint64_t *d_keys, const uint64_t *d_values, uint64_t n,
                uint64_t *d_out_values, uint8_t *d_out_status, hipStream_t s) {
    maybe_rebuild(ix, s);
    ensure_capacity(ix, d_ops, d_keys, n, s);
    const uint32_t slog = ix.cfg.small_batch_log2 ? ix.cfg.small_batch_log2 : 10;
    const uint32_t glog = ix.cfg.graph_max_log2;
    if (slog != 255 && n <= (1ull << slog))
        pi::execute_batch_small(ix, d_ops, d_keys, d_values, n, d_out_values, d_out_status, s);
    else if (glog != 0 && !ix.prof.on && n <= (1ull << glog))
        pi::execute_batch_graph(ix, d_ops, d_keys, d_values, n, d_out_values, d_out_status, s);
    else
        pi::execute_batch(ix, d_ops, d_keys, d_values, n, d_out_values, d_out_status, s);
    ix.used_upper = std::min<uint64_t>(ix.used_upper + n, ~0ull);
    ix.enq_queries += n;
    push_state(ix, s);
    if (ix.cfg.rebuild_policy == PI_REBUILD_ALWAYS) {
        pi::DevState cur;
        pi::read_state(ix, s, &cur);
        if (cur.changes > 0) pi::rebuild(ix, s);
    }
}

// One micro-batch of the serving loop with the ordering on the side stream
// (pi::pipe_open done): the same steps, bookkeeping and results as
// batch_step.  Batches that take the one-workgroup path have no separate
// ordering and run as there.
void serve_step(pi::Index &ix, const uint8_t *d_ops, const uint64_t *d_keys, const uint64_t *d_values, uint64_t n,
                uint64_t *d_out_values, uint8_t *d_out_status, hipStream_t s) {
    const uint32_t slog = ix.cfg.small_batch_log2 ? ix.cfg.small_batch_log2 : 10;
    if (ix.prof.on || ix.cfg.graph_max_log2 != 0 || (slog != 255 && n <= (1ull << slog)) ||
        ix.cfg.rebuild_policy == PI_REBUILD_ALWAYS) {
        batch_step(ix, d_ops, d_keys, d_values, n, d_out_values, d_out_status, s);
        return;
    }
    maybe_rebuild(ix, s);
    ensure_capacity(ix, d_ops, d_keys, n, s);
    pi::Index::ServePipe &p = ix.pipe;
    auto &set = p.set[p.next];
    p.next ^= 1;
    const pi::BatchBuffers buf{set.sort, set.msd, set.scan, set.bws};
    // this set's previous batch is done with its buffers before they are
    // ordered into again
    if (set.used) PI_HIP(hipStreamWaitEvent(p.side, set.done, 0));
    const uint64_t *sk = nullptr;
    const uint32_t *sidx = nullptr;
    const uint32_t bits = pi::order_bits(ix, n);
    pi::order_batch(buf, d_ops, d_keys, n, p.side, &sk, &sidx, bits);
    PI_HIP(hipEventRecord(set.ordered, p.side));
    PI_HIP(hipStreamWaitEvent(s, set.ordered, 0));
    pi::finish_batch(ix, buf, sk, sidx, d_ops, d_values, n, d_out_values, d_out_status, s, nullptr, bits);
    PI_HIP(hipEventRecord(set.done, s));
    set.used = true;
    ix.used_upper = std::min<uint64_t>(ix.used_upper + n, ~0ull);
    ix.enq_queries += n;
    push_state(ix, s);
}

pi_status pi_execute_batch(pi_index *h, const uint8_t *d_ops, const uint64_t *d_keys, const uint64_t *d_values,
                           uint64_t n, uint64_t *d_out_values, uint8_t *d_out_status, pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (n == 0) return PI_OK;
        if (n > MAX_BATCH) return fail(ix, PI_ERR_INVALID_ARG, "n too large");
        if (!d_ops || !d_keys || !d_values || !d_out_values || !d_out_status)
            return fail(ix, PI_ERR_INVALID_ARG, "NULL pointer");
        batch_step(ix, d_ops, d_keys, d_values, n, d_out_values, d_out_status, (hipStream_t)stream);
        return PI_OK;
    });
}

pi_status pi_execute_batch_noalloc(pi_index *h, const uint8_t *d_ops, const uint64_t *d_keys,
                                   const uint64_t *d_values, uint64_t n, uint64_t *d_out_values,
                                   uint8_t *d_out_status, pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (n == 0) return PI_OK;
        if (n > pi::noalloc_max_batch()) return fail(ix, PI_ERR_INVALID_ARG, "n above the scratch limit (2^16)");
        if (ix.cfg.check_writers) return fail(ix, PI_ERR_INVALID_ARG, "the writer check allocates its shadow");
        if (!d_ops || !d_keys || !d_values || !d_out_values || !d_out_status)
            return fail(ix, PI_ERR_INVALID_ARG, "NULL pointer");
        hipStream_t s = (hipStream_t)stream;
        uint8_t *scr = pi::noalloc_scratch(ix.device);
        // counters that have landed: device errors and the storage bound; no
        // rebuild (it allocates): the next allocating call takes it up
        maybe_rebuild(ix, s, false);
        // room for the new nodes, never by growing the storage; the insert
        // count goes to the first word of the scratch
        ix.batch_peak = std::max(ix.batch_peak, n);
        if (ix.used_upper + n > ix.st.cap) {
            pi::DevState cur;
            pi::read_state(ix, s, &cur);
            if (cur.nused + n > ix.st.cap) {
                const uint64_t ins = pi::count_inserts(ix, d_ops, d_keys, n, s, reinterpret_cast<unsigned int *>(scr));
                if (cur.nused + ins > ix.st.cap)
                    return fail(ix, PI_ERR_CAPACITY, "no room for the batch's new nodes (this call never grows "
                                                     "the storage)");
            }
        }
        // every per-batch buffer from the scratch, sized before the first launch
        constexpr size_t RESERVED = 256;  // the insert counter above
        pi::Arena arena{scr + RESERVED, pi::noalloc_scratch_bytes() - RESERVED, 0};
        pi::SortWorkspace sw;
        pi::MsdWorkspace mw;
        pi::ScanWorkspace cw;
        pi::BatchWorkspace bw;
        const bool prof = ix.prof.on;  // stage events are created on demand: off for this call
        ix.prof.on = false;
        try {
            pi::ArenaScope scope(&arena);
            sw.ensure(n);
            mw.ensure(n);
            cw.ensure(n);
            bw.ensure(n);
            pi::execute_batch(ix, pi::BatchBuffers{sw, mw, cw, bw}, d_ops, d_keys, d_values, n, d_out_values,
                              d_out_status, s);
        } catch (...) {
            ix.prof.on = prof;
            throw;
        }
        ix.prof.on = prof;
        ix.used_upper = std::min<uint64_t>(ix.used_upper + n, ~0ull);
        ix.enq_queries += n;
        push_state(ix, s);
        return PI_OK;
    });
}

pi_status pi_serve(pi_index *h, const pi_serve_config *cfg, const double *h_arrival_us, const uint8_t *d_ops,
                   const uint64_t *d_keys, const uint64_t *d_values, uint64_t n, uint64_t *d_out_values,
                   uint8_t *d_out_status, double *h_done_us, uint64_t *h_batch_end, uint64_t *n_batches,
                   pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (!cfg || cfg->struct_size != sizeof(pi_serve_config)) return fail(ix, PI_ERR_INVALID_ARG, "bad config");
        if (!n_batches) return fail(ix, PI_ERR_INVALID_ARG, "n_batches is NULL");
        *n_batches = 0;
        if (n == 0) return PI_OK;
        if (!h_arrival_us || !d_ops || !d_keys || !d_values || !d_out_values || !d_out_status || !h_done_us ||
            !h_batch_end)
            return fail(ix, PI_ERR_INVALID_ARG, "NULL pointer");
        if (!(cfg->deadline_us >= 0.0) || cfg->max_batch > MAX_BATCH || cfg->max_inflight > 64)
            return fail(ix, PI_ERR_INVALID_ARG, "bad config");
        for (uint64_t i = 1; i < n; i++)
            if (!(h_arrival_us[i] >= h_arrival_us[i - 1]))
                return fail(ix, PI_ERR_INVALID_ARG, "arrival times must be non-decreasing");
        hipStream_t s = (hipStream_t)stream;
        if (ix.cfg.capacity_hint) {
            // a fixed capacity must hold every insert of the stream: checked
            // before the first micro-batch, so this error leaves the index
            // unchanged
            pi::DevState cur;
            pi::read_state(ix, s, &cur);
            if (cur.nused + n > ix.st.cap) {
                const uint64_t ins = pi::count_inserts(ix, d_ops, d_keys, n, s);
                if (cur.nused + ins > ix.st.cap)
                    return fail(ix, PI_ERR_CAPACITY, "the stream's inserts do not fit the fixed capacity");
            }
        }
        pi::ServePlan plan;
        plan.deadline_us = cfg->deadline_us;
        plan.max_inflight = cfg->max_inflight ? cfg->max_inflight : 1;
        plan.max_batch = cfg->max_batch ? cfg->max_batch : pi::serve_batch_limit(plan.max_inflight);
        // more than one micro-batch in flight: the next one's ordering runs
        // beside the current one's descent
        const bool overlap = plan.max_inflight > 1;
        if (overlap) pi::pipe_open(ix, s);
        pi::serve_loop(
            h_arrival_us, n, plan, s,
            [&](uint64_t b, uint64_t e) {
                if (overlap)
                    serve_step(ix, d_ops + b, d_keys + b, d_values + b, e - b, d_out_values + b, d_out_status + b, s);
                else
                    batch_step(ix, d_ops + b, d_keys + b, d_values + b, e - b, d_out_values + b, d_out_status + b,
                               s);
            },
            h_done_us, h_batch_end, *n_batches);
        return PI_OK;
    });
}

pi_status pi_repair(pi_index *h, pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        pi::rebuild(ix, (hipStream_t)stream);
        ix.ring_seen = ix.ring_head;
        return PI_OK;
    });
}

pi_status pi_export(pi_index *h, uint64_t *d_keys, uint64_t *d_values, uint64_t cap, uint64_t *n_out,
                    pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (!n_out) return fail(ix, PI_ERR_INVALID_ARG, "n_out is NULL");
        if (cap > 0 && (!d_keys || !d_values)) return fail(ix, PI_ERR_INVALID_ARG, "NULL output");
        pi::DevState cur;
        pi::read_state(ix, (hipStream_t)stream, &cur);
        *n_out = cur.n_live;
        if (cur.n_live > cap) return fail(ix, PI_ERR_CAPACITY, "export capacity too small");
        *n_out = pi::export_live(ix, d_keys, d_values, cap, (hipStream_t)stream);
        return PI_OK;
    });
}

pi_status pi_range_count(pi_index *h, const uint64_t *d_lo, const uint64_t *d_hi, uint64_t n, uint64_t *d_offsets,
                         pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (n > MAX_BATCH) return fail(ix, PI_ERR_INVALID_ARG, "n too large");
        if (!d_offsets || (n > 0 && (!d_lo || !d_hi))) return fail(ix, PI_ERR_INVALID_ARG, "NULL pointer");
        pi::range_count(ix, d_lo, d_hi, n, d_offsets, (hipStream_t)stream);
        return PI_OK;
    });
}

pi_status pi_range_collect(pi_index *h, const uint64_t *d_lo, const uint64_t *d_hi, uint64_t n,
                           const uint64_t *d_offsets, uint64_t *d_keys, uint64_t *d_values, pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (n > MAX_BATCH) return fail(ix, PI_ERR_INVALID_ARG, "n too large");
        if (n > 0 && (!d_lo || !d_hi || !d_offsets || !d_keys || !d_values))
            return fail(ix, PI_ERR_INVALID_ARG, "NULL pointer");
        pi::range_collect(ix, d_lo, d_hi, n, d_offsets, d_keys, d_values, (hipStream_t)stream);
        return PI_OK;
    }, true);
}

pi_status pi_get_stats(pi_index *h, pi_stats *out) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (!out) return fail(ix, PI_ERR_INVALID_ARG, "out is NULL");
        PI_HIP(hipDeviceSynchronize());
        pi::DevState cur;
        pi::read_state(ix, nullptr, &cur);
        std::memset(out, 0, sizeof(*out));
        out->batches = cur.batches;
        out->queries = cur.queries;
        out->hits = cur.hits;
        out->invalid = cur.invalid;
        out->new_nodes = cur.new_nodes;
        out->deletes = cur.deletes;
        out->revives = cur.revives;
        out->changes = cur.changes;
        out->repairs = ix.repairs;
        out->live_nodes = cur.n_live;
        out->base_nodes = ix.nbase;
        out->overflow_nodes = cur.nused - (ix.nbase + 2);
        out->capacity = ix.st.cap;
        out->n_levels = (uint32_t)ix.desc.top;
        out->lds_from = (uint32_t)ix.desc.lds_from;
        for (int l = 2; l <= ix.desc.top && l < 33; l++)
            out->level_size[l] = ix.slc.on ? ix.slc.real_n[l] : ix.desc.n[l];
        out->index_rebuilds = ix.bg.done;
        out->slice_rounds = ix.slc.rounds;
        out->slices_repaired = ix.slc.repaired;
        out->slices = ix.slc.on ? ix.slc.lay.S : 0;
        return PI_OK;
    });
}

pi_status pi_get_profile(pi_index *h, pi_profile *out, int32_t reset) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (!out) return fail(ix, PI_ERR_INVALID_ARG, "out is NULL");
        PI_HIP(hipDeviceSynchronize());
        ix.prof.drain(true);
        *out = ix.prof.acc;
        if (reset) ix.prof.acc = pi_profile{};
        return PI_OK;
    });
}

const char *pi_last_error(const pi_index *h) {
    if (!h) {
        std::lock_guard<std::mutex> g(g_create_err_mu);
        return g_create_err.c_str();
    }
    return h->ix.err.c_str();
}

pi_status pi_debug_interceptions(pi_index *h, const uint64_t *d_keys, uint64_t n, uint64_t *d_icpt_keys,
                                 uint8_t *d_is_head, pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (n == 0) return PI_OK;
        if (n > MAX_BATCH) return fail(ix, PI_ERR_INVALID_ARG, "n too large");
        if (!d_keys || !d_icpt_keys || !d_is_head) return fail(ix, PI_ERR_INVALID_ARG, "NULL pointer");
        pi::debug_interceptions(ix, d_keys, n, d_icpt_keys, d_is_head, (hipStream_t)stream);
        return PI_OK;
    });
}

pi_status pi_debug_level(pi_index *h, uint32_t level, uint64_t *d_keys, uint32_t *d_down, uint64_t cap,
                         uint64_t *n_out, pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (!n_out) return fail(ix, PI_ERR_INVALID_ARG, "n_out is NULL");
        if (level < 2 || level > ix.cfg.max_height) return fail(ix, PI_ERR_INVALID_ARG, "bad level");
        hipStream_t s = (hipStream_t)stream;
        if (ix.slc.on) {
            const uint64_t n = (int)level <= ix.desc.top ? ix.slc.real_n[level] : 0;
            *n_out = n;
            if (n > cap) return fail(ix, PI_ERR_CAPACITY, "level larger than cap");
            if (n > 0 && (!d_keys || !d_down)) return fail(ix, PI_ERR_INVALID_ARG, "NULL output");
            if (n > 0) pi::slice_export_level(ix, (int)level, d_keys, d_down, cap, s);
            return PI_OK;
        }
        const uint64_t n = (int)level <= ix.desc.top ? ix.desc.n[level] : 0;
        *n_out = n;
        if (n > cap) return fail(ix, PI_ERR_CAPACITY, "level larger than cap");
        if (n > 0) {
            if (!d_keys || !d_down) return fail(ix, PI_ERR_INVALID_ARG, "NULL output");
            const uint64_t o = ix.desc.off[level] + 1;
            PI_HIP(hipMemcpyAsync(d_keys, ix.arena_key.as<uint64_t>() + o, n * 8, hipMemcpyDeviceToDevice, s));
            PI_HIP(hipMemcpyAsync(d_down, ix.arena_down.as<uint32_t>() + o, n * 4, hipMemcpyDeviceToDevice, s));
        }
        PI_HIP(hipStreamSynchronize(s));
        return PI_OK;
    });
}

pi_status pi_debug_writer_selftest(pi_index *h, uint32_t *same_writer_err, uint32_t *two_writer_err,
                                   pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (!same_writer_err || !two_writer_err) return fail(ix, PI_ERR_INVALID_ARG, "NULL output");
        pi::writer_selftest(ix, (hipStream_t)stream, same_writer_err, two_writer_err);
        return PI_OK;
    }, true);
}

pi_status pi_debug_set_storage_bound(pi_index *h, uint64_t used_upper) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        ix.used_upper = used_upper;
        return PI_OK;
    }, true);
}

pi_status pi_debug_sort(pi_index *h, const uint64_t *d_keys, uint64_t n, uint64_t *d_sorted_keys, uint32_t *d_perm,
                        pi_stream stream) {
    return guarded(h, [&](pi::Index &ix) -> pi_status {
        if (n == 0) return PI_OK;
        if (n > MAX_BATCH) return fail(ix, PI_ERR_INVALID_ARG, "n too large");
        if (!d_keys || !d_sorted_keys || !d_perm) return fail(ix, PI_ERR_INVALID_ARG, "NULL pointer");
        hipStream_t s = (hipStream_t)stream;
        const uint64_t *sk = nullptr;
        const uint32_t *si = nullptr;
        pi::sort_batch_by_range(ix.sortws, ix.msdws, d_keys, nullptr, n, false, s, &sk, &si);
        PI_HIP(hipMemcpyAsync(d_sorted_keys, sk, n * 8, hipMemcpyDeviceToDevice, s));
        PI_HIP(hipMemcpyAsync(d_perm, si, n * 4, hipMemcpyDeviceToDevice, s));
        return PI_OK;
    });
}

}  // extern "C"
