// Many independent indices, one launch: the batching form of the hot path.
//
// The paper splits one index into per-NUMA-node sub-indices that process
// their own queries independently (Section 4.2); here many independent
// indices of very different sizes share one GPU.  Batches that are small
// enough run in one persistent fused launch: each workgroup pulls the next
// (index, batch) item from a work queue -- items sorted largest first -- and
// runs the whole hot path for it in LDS-sized chunks (the workgroup batch of
// small.h), so one launch serves hundreds of indices and the host cost per
// index is a few bytes of descriptor instead of ~26 launches.  Larger
// batches use the GPU-wide multi-kernel path.  A workgroup is the only
// writer of its index while it runs, which is why an index may appear once
// per call.
//
// The threshold between the two paths is picked by an autotuner that times
// SEARCH-only replays of the caller's batches.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <exception>
#include <cstring>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "small.h"

namespace pi {
namespace {

struct GroupItem {
    IndexView v;
    BatchView b;
};

__global__ __launch_bounds__(SBT) void k_group_batches(const GroupItem *__restrict__ items, uint32_t nitems,
                                                       unsigned int *next) {
    extern __shared__ uint64_t s_raw[];
    __shared__ uint32_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(next, 1u);
        __syncthreads();
        const uint32_t it = s_item;
        __syncthreads();
        if (it >= nitems) break;
        const GroupItem &g = items[it];
        const uint32_t n = g.b.n;
        for (uint32_t c = 0; c < n; c += SB_MAX) {
            BatchView b = g.b;
            b.ops += c;
            b.keys += c;
            b.vals += c;
            b.out_vals += c;
            b.out_status += c;
            b.n = n - c < SB_MAX ? n - c : SB_MAX;
            b.unit = g.b.unit + c / SB_MAX;  // each chunk is a batch of its own for the writer check
            b.first = c == 0;
            block_batch(g.v, b, s_raw);
        }
    }
}

__global__ void k_gather_states(DevState *const *__restrict__ src, uint32_t n, DevState *__restrict__ dst) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = *src[i];
}

__global__ void k_zero_counter(unsigned int *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

}  // namespace
}  // namespace pi

struct pi_group {
    pi_group_config cfg{};
    int device = -1;
    pi::DevBuf d_items, d_ptrs, d_states, d_counter, d_zero_ops;
    pi::GroupItem *h_items = nullptr;
    pi::DevState **h_ptrs = nullptr;
    pi::DevState *h_states = nullptr;
    uint32_t cap_items = 0;
    std::vector<pi_index *> last;  // indices whose counters h_states holds
    std::vector<uint64_t> last_enq;  // their enq_queries when the copy was enqueued
    std::vector<uint64_t> last_epoch;  // their epoch then (unchanged: no call has touched them since)
    hipEvent_t ev = nullptr;
    hipEvent_t ev_start = nullptr, ev_fused = nullptr;  // fork/join of the fused launch
    hipStream_t fstream = nullptr;                      // the fused launch runs beside the large batches
    static constexpr int LANES = 4;                     // streams the large batches are spread over
    hipStream_t lane[LANES] = {};
    hipEvent_t ev_fork = nullptr, ev_lane[LANES] = {};
    hipEvent_t ev_in = nullptr;  // the caller's stream at the start of a call
    // the workspaces of the large batches and of the rebuilds, one set per
    // lane (the lane's stream orders their uses): they grow to the largest
    // batch and index the group has run once, where each index's own would
    // grow with that index (every growth frees a buffer, and a free waits
    // for the whole device)
    struct LaneBuffers {
        pi::SortWorkspace sort;
        pi::MsdWorkspace msd;
        pi::ScanWorkspace scan;
        pi::BatchWorkspace bws;
        pi::DevBuf tmp[10];
    } lbuf[LANES];
    // device buffers released during a call (by the calling thread and by
    // each worker), freed at the next call once this one has completed
    std::vector<void *> graveyard[LANES];
    bool pending = false;
    bool lds_attr = false;
    uint32_t tuned_block = 0, tuned_lds = 0;  // descent shape the autotuner applied (0 = none)
    std::string err;
};

namespace pi {
namespace {

struct GroupError {
    pi_status code;
    std::string msg;
};

void ensure_host(pi_group *g, uint32_t count) {
    if (count <= g->cap_items) return;
    if (g->h_items) (void)hipHostFree(g->h_items);
    if (g->h_ptrs) (void)hipHostFree(g->h_ptrs);
    if (g->h_states) (void)hipHostFree(g->h_states);
    g->h_items = nullptr;
    g->h_ptrs = nullptr;
    g->h_states = nullptr;
    PI_HIP(hipHostMalloc(&g->h_items, count * sizeof(GroupItem), hipHostMallocDefault));
    PI_HIP(hipHostMalloc(&g->h_ptrs, count * sizeof(DevState *), hipHostMallocDefault));
    PI_HIP(hipHostMalloc(&g->h_states, count * sizeof(DevState), hipHostMallocDefault));
    g->cap_items = count;
}

void ensure_lanes(pi_group *g) {
    if (g->ev_fork) return;
    for (int k = 0; k < pi_group::LANES; k++) {
        if (!g->lane[k]) PI_HIP(hipStreamCreateWithFlags(&g->lane[k], hipStreamNonBlocking));
        if (!g->ev_lane[k]) PI_HIP(hipEventCreateWithFlags(&g->ev_lane[k], hipEventDisableTiming));
    }
    if (!g->ev_in) PI_HIP(hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming));
    PI_HIP(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
}

// Runs fn(j, lane) for every job j < njobs, the jobs touching disjoint
// indices, on the group's lane streams (ordered after the work already on s,
// joined back into s).  Up to host_threads host threads take the jobs from a
// shared counter, each issuing on a lane stream of its own: a large batch is
// ~16 launches and a rebuild ~30 plus a wait for its index's counters, and
// one thread issuing all of them for hundreds of indices keeps the device
// waiting.  The first error a job raises stops the taking of new jobs and is
// rethrown once every thread has finished and the lanes are joined.
// after: what the lanes wait for (null: everything on s so far).
template <class F>
void on_lanes(pi_group *g, hipStream_t s, uint32_t njobs, F &&fn, hipEvent_t after = nullptr) {
    if (!njobs) return;
    ensure_lanes(g);
    const int lanes = (int)std::min<uint32_t>(njobs, pi_group::LANES);
    const int threads = std::min<int>(lanes, (int)g->cfg.host_threads);
    if (!after) {
        PI_HIP(hipEventRecord(g->ev_fork, s));
        after = g->ev_fork;
    }
    for (int k = 0; k < lanes; k++) PI_HIP(hipStreamWaitEvent(g->lane[k], after, 0));
    int dev = 0;
    PI_HIP(hipGetDevice(&dev));
    std::atomic<uint32_t> next{0};
    std::atomic<bool> failed{false};
    std::exception_ptr err[pi_group::LANES];
    auto work = [&](int t) {
        DeferFrees defer(&g->graveyard[t]);
        try {
            if (t) PI_HIP(hipSetDevice(dev));
            uint32_t j;
            // one thread (host_threads 1) cycles the lanes as the jobs come
            for (uint32_t m = 0; !failed.load() && (j = next.fetch_add(1)) < njobs; m++)
                fn(j, threads == 1 ? (int)(m % lanes) : t);
        } catch (...) {
            err[t] = std::current_exception();
            failed.store(true);
        }
    };
    std::vector<std::thread> th;
    th.reserve(threads - 1);
    for (int t = 1; t < threads; t++) th.emplace_back(work, t);
    work(0);
    for (std::thread &t : th) t.join();
    for (int k = 0; k < lanes; k++) {
        PI_HIP(hipEventRecord(g->ev_lane[k], g->lane[k]));
        PI_HIP(hipStreamWaitEvent(s, g->ev_lane[k], 0));
    }
    for (int t = 0; t < threads; t++)
        if (err[t]) std::rethrow_exception(err[t]);
}

// Lends a lane's workspaces to an index for the span of its rebuild.
struct LentScratch {
    Index &ix;
    pi_group::LaneBuffers &lb;
    LentScratch(Index &i, pi_group::LaneBuffers &l) : ix(i), lb(l) { swap(); }
    ~LentScratch() { swap(); }
    void swap() {
        std::swap(ix.sortws, lb.sort);
        std::swap(ix.msdws, lb.msd);
        std::swap(ix.scanws, lb.scan);
        static_assert(sizeof(ix.tmp) == sizeof(lb.tmp), "the lent set mirrors the index's scratch");
        for (size_t k = 0; k < sizeof(lb.tmp) / sizeof(lb.tmp[0]); k++) std::swap(ix.tmp[k], lb.tmp[k]);
    }
};

// The index's rebuild policy after a batch whose counters are st (exact:
// nothing has run on the index since, so a rebuild need not read them again).
void apply_policy(Index &ix, const DevState &st, bool exact, hipStream_t s) {
    const DevState *known = exact ? &st : nullptr;
    const uint32_t pol = ix.cfg.rebuild_policy;
    const double thr = rebuild_threshold(ix);
    if (pol == PI_REBUILD_BACKGROUND || pol == PI_REBUILD_SLICES) {
        if (pol == PI_REBUILD_BACKGROUND) bg_advance(ix);
        const double compact = (ix.cfg.compact_percent ? ix.cfg.compact_percent : 100) / 100.0 *
                               (double)std::max<uint64_t>(ix.nbase, 1);
        if ((double)st.changes >= std::max(compact, thr)) {
            rebuild(ix, s, known);
            ix.ring_seen = ix.ring_head;
        } else if (st.changes >= ix.changes_base && (double)(st.changes - ix.changes_base) >= thr) {
            if (pol == PI_REBUILD_BACKGROUND) {
                bg_start(ix, st, s);
            } else if (slice_round(ix, st.nused, s)) {
                ix.changes_base = st.changes;
            } else {  // (after a slice round that gave up: counters read again)
                rebuild(ix, s);
                ix.ring_seen = ix.ring_head;
            }
        }
        return;
    }
    if ((pol == PI_REBUILD_ALWAYS && st.changes > 0) || (double)st.changes >= thr) {
        rebuild(ix, s, known);
        ix.ring_seen = ix.ring_head;
    }
}

// Frees the buffers released during earlier calls, after every stream of
// the group has finished what may still read them (the wait costs nothing
// once the previous call has completed).
void free_deferred(pi_group *g) {
    bool any = false;
    for (const auto &l : g->graveyard) any |= !l.empty();
    if (!any) return;
    if (g->fstream) PI_HIP(hipStreamSynchronize(g->fstream));
    for (hipStream_t l : g->lane)
        if (l) PI_HIP(hipStreamSynchronize(l));
    // every pointer leaves the lists before any free can fail (none freed twice)
    hipError_t first = hipSuccess;
    for (auto &l : g->graveyard) {
        std::vector<void *> ps;
        ps.swap(l);
        for (void *p : ps) {
            const hipError_t e = hipFree(p);
            if (first == hipSuccess) first = e;
        }
    }
    PI_HIP(first);
}

// An index whose rebuild policy may act, and the counters it acts on.
struct Due {
    pi_index *h;
    DevState st;
    bool exact;  // no call has touched the index since the copy: st is its state now
};

// Waits for the previous call and takes up its counters: an index whose
// counters carry a device error fails; the host bounds are refreshed.
// Returns the indices whose rebuild policy may act on those counters.
std::vector<Due> settle_previous(pi_group *g) {
    std::vector<Due> due;
    if (!g->pending) return due;
    PI_HIP(hipEventSynchronize(g->ev));
    g->pending = false;
    free_deferred(g);
    for (size_t k = 0; k < g->last.size(); k++) {
        Index &ix = g->last[k]->ix;
        const DevState &st = g->h_states[k];
        if (st.errors) {
            ix.failed = true;
            ix.err = device_error_text(st.errors);
            throw Error{PI_ERR_DEVICE, ix.err};
        }
        // nused in the copy plus every query enqueued on the index since the
        // copy (group or single calls) bounds the storage in use now
        ix.used_upper = std::min<uint64_t>(ix.used_upper, st.nused + (ix.enq_queries - g->last_enq[k]));
        ix.recent_writers = st.b_writers != 0;  // the form of the next large batch's post-descent steps
        if (ix.cfg.rebuild_policy != PI_REBUILD_NEVER) {
            const bool exact = ix.epoch == g->last_epoch[k];
            // the policy may change the storage: no range search of an
            // earlier call may reuse its ordering and interceptions
            ix.epoch++;
            due.push_back(Due{g->last[k], st, exact});
        }
    }
    g->last.clear();
    g->last_enq.clear();
    g->last_epoch.clear();
    return due;
}

// Room for the batch's new nodes (the host bound first, the device count
// when the bound does not fit).
void group_capacity(Index &ix, const pi_batch &b, hipStream_t s) {
    ix.batch_peak = std::max(ix.batch_peak, b.n);
    if (ix.used_upper + b.n <= ix.st.cap) return;
    DevState cur;
    read_state(ix, s, &cur);
    if (cur.nused + b.n <= ix.st.cap) return;
    if (ix.cfg.capacity_hint) {
        const uint64_t ins = count_inserts(ix, b.d_ops, b.d_keys, b.n, s);
        if (cur.nused + ins > ix.st.cap) throw GroupError{PI_ERR_CAPACITY, "an index of the group has no room"};
        return;
    }
    grow_storage(ix, cur.nused + b.n, std::max<uint64_t>(cur.nused + 2 * b.n, ix.st.cap * 2), s);
}

void run_group_body(pi_group *g, pi_index *const *indices, const pi_batch *batches, uint32_t count, hipStream_t s,
                    uint64_t fused_max, const uint8_t *ops_override);

void run_group(pi_group *g, pi_index *const *indices, const pi_batch *batches, uint32_t count, hipStream_t s,
               uint64_t fused_max, const uint8_t *ops_override) {
    TraceRange tr("pi:group");
    DeferFrees defer(&g->graveyard[0]);
    try {
        run_group_body(g, indices, batches, count, s, fused_max, ops_override);
    } catch (...) {
        // what this call enqueued may still read the released buffers
        (void)hipDeviceSynchronize();
        for (auto &l : g->graveyard) {
            for (void *p : l) (void)hipFree(p);
            l.clear();
        }
        throw;
    }
}

void run_group_body(pi_group *g, pi_index *const *indices, const pi_batch *batches, uint32_t count, hipStream_t s,
                    uint64_t fused_max, const uint8_t *ops_override) {
    const std::vector<Due> due = settle_previous(g);
    for (uint32_t i = 0; i < count; i++) indices[i]->ix.epoch++;
    ensure_lanes(g);
    PI_HIP(hipEventRecord(g->ev_in, s));
    // A policy acts before its index's batch.  Before the fused launch: the
    // indices whose batch it runs, and those of fixed capacity (all such
    // rooms are checked before any batch of the call is enqueued).  The
    // others act on their lane right before their large batch, or, with no
    // batch in this call, beside the rest: neither waits for the fused launch
    // nor holds it up.
    std::unordered_map<const pi_index *, uint32_t> slot;
    slot.reserve(2 * (size_t)count);
    for (uint32_t i = 0; i < count; i++) slot.emplace(indices[i], i);
    auto early = [&](uint32_t i) {
        return batches[i].n && (batches[i].n <= fused_max || indices[i]->ix.cfg.capacity_hint);
    };
    struct Job {
        int32_t batch, due;  // -1: none
    };
    std::vector<uint32_t> first;
    std::vector<int32_t> due_of(count, -1);
    std::vector<Job> jobs;
    for (uint32_t j = 0; j < due.size(); j++) {
        const auto it = slot.find(due[j].h);
        if (it == slot.end() || !batches[it->second].n)
            jobs.push_back(Job{-1, (int32_t)j});
        else if (early(it->second))
            first.push_back(j);
        else
            due_of[it->second] = (int32_t)j;
    }
    on_lanes(g, s, (uint32_t)first.size(), [&](uint32_t j, int k) {
        const Due &d = due[first[j]];
        LentScratch lent(d.h->ix, g->lbuf[k]);
        apply_policy(d.h->ix, d.st, d.exact, g->lane[k]);
    });
    for (uint32_t i = 0; i < count; i++)
        if (early(i)) group_capacity(indices[i]->ix, batches[i], s);
    ensure_host(g, count);
    std::vector<uint32_t> fused;
    for (uint32_t i = 0; i < count; i++) {
        const pi_batch &b = batches[i];
        if (!early(i)) continue;
        if (b.n <= fused_max) fused.push_back(i);
        indices[i]->ix.used_upper = std::min<uint64_t>(indices[i]->ix.used_upper + b.n, ~0ull);
        indices[i]->ix.enq_queries += b.n;
    }
    // small batches: one persistent launch, largest first, on the group's
    // own stream so that it overlaps the large batches below
    if (!fused.empty()) {
        if (!g->fstream) {
            PI_HIP(hipStreamCreateWithFlags(&g->fstream, hipStreamNonBlocking));
            PI_HIP(hipEventCreateWithFlags(&g->ev_start, hipEventDisableTiming));
            PI_HIP(hipEventCreateWithFlags(&g->ev_fused, hipEventDisableTiming));
        }
        PI_HIP(hipEventRecord(g->ev_start, s));
        PI_HIP(hipStreamWaitEvent(g->fstream, g->ev_start, 0));
        std::sort(fused.begin(), fused.end(), [&](uint32_t a, uint32_t b) { return batches[a].n > batches[b].n; });
        const uint32_t nf = (uint32_t)fused.size();
        for (uint32_t k = 0; k < nf; k++) {
            const pi_batch &b = batches[fused[k]];
            GroupItem &it = g->h_items[k];
            Index &fx = indices[fused[k]]->ix;
            const WriterCheck wc = writer_check(fx, (uint32_t)((b.n + SB_MAX - 1) / SB_MAX));
            it.v = index_view(fx);
            it.v.owner = wc.owner;
            it.b = BatchView{ops_override ? ops_override : b.d_ops, b.d_keys, b.d_values, (uint32_t)b.n,
                             b.d_out_values, b.d_out_status, wc.unit, 1};
        }
        g->d_items.ensure((size_t)g->cap_items * sizeof(GroupItem));
        g->d_counter.ensure(64);
        hipStream_t fs = g->fstream;
        PI_HIP(hipMemcpyAsync(g->d_items.p, g->h_items, nf * sizeof(GroupItem), hipMemcpyHostToDevice, fs));
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, fs, g->d_counter.as<unsigned int>());
        const uint32_t lds = SmallLds::bytes();
        if (!g->lds_attr) {
            PI_HIP(hipFuncSetAttribute((const void *)k_group_batches, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds));
            g->lds_attr = true;
        }
        const uint32_t grid = std::min<uint32_t>(nf, (uint32_t)indices[fused[0]]->ix.num_cus);
        hipLaunchKernelGGL(k_group_batches, dim3(grid), dim3(SBT), lds, fs, g->d_items.as<GroupItem>(), nf,
                           g->d_counter.as<unsigned int>());
        PI_LAUNCH_CHECK();
        PI_HIP(hipEventRecord(g->ev_fused, fs));
    }
    // large batches: the GPU-wide path on the group's lane streams (the
    // indices are disjoint, and one batch of a few hundred thousand queries
    // does not fill the GPU), each after its index's policy, beside the fused
    // launch; joined back into the caller's stream
    for (uint32_t i = 0; i < count; i++)
        if (batches[i].n > fused_max) jobs.push_back(Job{(int32_t)i, due_of[i]});
    // the largest batches first; the policies of indices without a batch last
    std::sort(jobs.begin(), jobs.end(), [&](const Job &a, const Job &b) {
        const uint64_t na = a.batch < 0 ? 0 : batches[a.batch].n, nb = b.batch < 0 ? 0 : batches[b.batch].n;
        return na > nb;
    });
    on_lanes(
        g, s, (uint32_t)jobs.size(),
        [&](uint32_t j, int k) {
            const Job &jb = jobs[j];
            hipStream_t ls = g->lane[k];
            pi_group::LaneBuffers &lb = g->lbuf[k];
            if (jb.due >= 0) {
                const Due &d = due[jb.due];
                LentScratch lent(d.h->ix, lb);
                apply_policy(d.h->ix, d.st, d.exact, ls);
            }
            if (jb.batch < 0) return;
            const pi_batch &b = batches[jb.batch];
            Index &ix = indices[jb.batch]->ix;
            if (!ix.cfg.capacity_hint) {  // (a fixed capacity was checked before the fused launch)
                group_capacity(ix, b, ls);
                ix.used_upper = std::min<uint64_t>(ix.used_upper + b.n, ~0ull);
                ix.enq_queries += b.n;
            }
            execute_batch(ix, BatchBuffers{lb.sort, lb.msd, lb.scan, lb.bws}, ops_override ? ops_override : b.d_ops,
                          b.d_keys, b.d_values, b.n, b.d_out_values, b.d_out_status, ls);
        },
        g->ev_in);
    if (!fused.empty()) PI_HIP(hipStreamWaitEvent(s, g->ev_fused, 0));
    // one copy of every index's counters
    uint32_t ns = 0;
    g->last.clear();
    g->last_enq.clear();
    g->last_epoch.clear();
    for (uint32_t i = 0; i < count; i++) {
        if (!batches[i].n) continue;
        g->h_ptrs[ns++] = indices[i]->ix.dstate;
        g->last.push_back(indices[i]);
        g->last_enq.push_back(indices[i]->ix.enq_queries);
        g->last_epoch.push_back(indices[i]->ix.epoch);
    }
    if (ns) {
        g->d_ptrs.ensure((size_t)g->cap_items * sizeof(DevState *));
        g->d_states.ensure((size_t)g->cap_items * sizeof(DevState));
        PI_HIP(hipMemcpyAsync(g->d_ptrs.p, g->h_ptrs, ns * sizeof(DevState *), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_gather_states, dim3((ns + 255) / 256), dim3(256), 0, s,
                           g->d_ptrs.as<DevState *>(), ns, g->d_states.as<DevState>());
        PI_LAUNCH_CHECK();
        PI_HIP(hipMemcpyAsync(g->h_states, g->d_states.p, ns * sizeof(DevState), hipMemcpyDeviceToHost, s));
    }
    PI_HIP(hipEventRecord(g->ev, s));
    g->pending = true;
}

pi_status validate(pi_group *g, pi_index *const *indices, const pi_batch *batches, uint32_t count) {
    if (count == 0) return PI_OK;
    if (!indices || !batches) return PI_ERR_INVALID_ARG;
    if (count > g->cfg.max_indices) return PI_ERR_INVALID_ARG;
    std::unordered_set<const pi_index *> seen;
    int dev = -1;
    for (uint32_t i = 0; i < count; i++) {
        const pi_index *h = indices[i];
        const pi_batch &b = batches[i];
        if (!h || h->ix.failed) return PI_ERR_INVALID_ARG;
        if (!seen.insert(h).second) return PI_ERR_INVALID_ARG;
        if (dev < 0) dev = h->ix.device;
        if (h->ix.device != dev) return PI_ERR_INVALID_ARG;
        if (b.n > (1ull << 31) - 1) return PI_ERR_INVALID_ARG;
        if (b.n && (!b.d_ops || !b.d_keys || !b.d_values || !b.d_out_values || !b.d_out_status))
            return PI_ERR_INVALID_ARG;
    }
    if (g->device >= 0 && g->device != dev) return PI_ERR_INVALID_ARG;
    g->device = dev;
    return PI_OK;
}

template <class F>
pi_status group_guarded(pi_group *g, F &&f) {
    if (!g) return PI_ERR_INVALID_ARG;
    int prev = -1;
    (void)hipGetDevice(&prev);
    pi_status r = PI_OK;
    try {
        r = f();
        if (r == PI_OK) g->err.clear();
    } catch (const GroupError &e) {
        g->err = e.msg;
        r = e.code;
    } catch (const Error &e) {
        g->err = e.msg;
        r = e.code;
    } catch (const std::exception &e) {
        g->err = e.what();
        r = PI_ERR_DEVICE;
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    return r;
}

}  // namespace
}  // namespace pi

extern "C" {

pi_status pi_group_config_default(pi_group_config *cfg) {
    if (!cfg) return PI_ERR_INVALID_ARG;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->struct_size = sizeof(pi_group_config);
    cfg->max_indices = 4096;
    cfg->fused_max = 4096;
    cfg->host_threads = pi_group::LANES;
    return PI_OK;
}

pi_status pi_group_create(const pi_group_config *cfg, pi_group **out) {
    if (!out) return PI_ERR_INVALID_ARG;
    *out = nullptr;
    pi_group_config c;
    pi_group_config_default(&c);
    if (cfg) {
        if (cfg->struct_size != sizeof(pi_group_config)) return PI_ERR_INVALID_ARG;
        c = *cfg;
        if (!c.max_indices) c.max_indices = 4096;
        if (!c.fused_max) c.fused_max = 4096;
        if (!c.host_threads) c.host_threads = pi_group::LANES;
    }
    if (c.fused_max > (1ull << 31) - 1) return PI_ERR_INVALID_ARG;
    if (c.host_threads > (uint32_t)pi_group::LANES || c.reserved) return PI_ERR_INVALID_ARG;
    pi_group *g = new pi_group;
    g->cfg = c;
    if (hipEventCreateWithFlags(&g->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        delete g;
        return PI_ERR_DEVICE;
    }
    *out = g;
    return PI_OK;
}

pi_status pi_group_destroy(pi_group *g) {
    if (!g) return PI_OK;
    if (g->pending) (void)hipEventSynchronize(g->ev);
    if (g->device >= 0) (void)hipSetDevice(g->device);
    g->d_items.release();
    g->d_ptrs.release();
    g->d_states.release();
    g->d_counter.release();
    g->d_zero_ops.release();
    if (g->h_items) (void)hipHostFree(g->h_items);
    if (g->h_ptrs) (void)hipHostFree(g->h_ptrs);
    if (g->h_states) (void)hipHostFree(g->h_states);
    if (g->ev) (void)hipEventDestroy(g->ev);
    if (g->ev_start) (void)hipEventDestroy(g->ev_start);
    if (g->ev_fused) (void)hipEventDestroy(g->ev_fused);
    if (g->fstream) {
        (void)hipStreamSynchronize(g->fstream);
        (void)hipStreamDestroy(g->fstream);
    }
    for (int k = 0; k < pi_group::LANES; k++) {
        if (g->lane[k]) {
            (void)hipStreamSynchronize(g->lane[k]);
            (void)hipStreamDestroy(g->lane[k]);
        }
        if (g->ev_lane[k]) (void)hipEventDestroy(g->ev_lane[k]);
        pi_group::LaneBuffers &lb = g->lbuf[k];
        lb.sort.release();
        lb.msd.release();
        lb.scan.release();
        lb.bws.release();
        for (pi::DevBuf &b : lb.tmp) b.release();
    }
    for (auto &l : g->graveyard)
        for (void *p : l) (void)hipFree(p);
    if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
    if (g->ev_in) (void)hipEventDestroy(g->ev_in);
    delete g;
    return PI_OK;
}

pi_status pi_group_execute(pi_group *g, pi_index *const *indices, const pi_batch *batches, uint32_t count,
                           pi_stream stream) {
    return pi::group_guarded(g, [&]() -> pi_status {
        const pi_status v = pi::validate(g, indices, batches, count);
        if (v != PI_OK) {
            g->err = "invalid group call";
            return v;
        }
        if (count == 0) return PI_OK;
        PI_HIP(hipSetDevice(g->device));
        pi::run_group(g, indices, batches, count, (hipStream_t)stream, g->cfg.fused_max, nullptr);
        return PI_OK;
    });
}

pi_status pi_group_autotune(pi_group *g, pi_index *const *indices, const pi_batch *batches, uint32_t count,
                            pi_stream stream, uint64_t *fused_max) {
    return pi::group_guarded(g, [&]() -> pi_status {
        const pi_status v = pi::validate(g, indices, batches, count);
        if (v != PI_OK || !fused_max) {
            g->err = "invalid group call";
            return v != PI_OK ? v : PI_ERR_INVALID_ARG;
        }
        *fused_max = g->cfg.fused_max;
        if (count == 0) return PI_OK;
        PI_HIP(hipSetDevice(g->device));
        hipStream_t s = (hipStream_t)stream;
        uint64_t nmax = 0;
        for (uint32_t i = 0; i < count; i++) nmax = std::max<uint64_t>(nmax, batches[i].n);
        // all-SEARCH replays: a zero op array as long as the longest batch
        g->d_zero_ops.ensure(std::max<uint64_t>(nmax, 1));
        PI_HIP(hipMemsetAsync(g->d_zero_ops.p, 0, std::max<uint64_t>(nmax, 1), s));
        const uint64_t candidates[] = {0, 1024, 4096, 16384, 32768, 65536, 131072, 262144, 524288, 1048576};
        double best = 1e30;
        uint64_t pick = g->cfg.fused_max;
        uint64_t prev = 0;
        for (uint64_t t : candidates) {
            if (t > 0 && prev >= nmax) break;  // the previous threshold already fused every batch
            prev = t;
            double tmin = 1e30;
            for (int rep = 0; rep < 2; rep++) {
                PI_HIP(hipStreamSynchronize(s));
                const auto t0 = std::chrono::steady_clock::now();
                pi::run_group(g, indices, batches, count, s, t, g->d_zero_ops.as<uint8_t>());
                PI_HIP(hipStreamSynchronize(s));
                const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                tmin = std::min(tmin, dt);
            }
            if (tmin < best) {
                best = tmin;
                pick = t;
            }
        }
        g->cfg.fused_max = pick;
        *fused_max = pick;
        // then the descent shape of the batches left to the multi-kernel path:
        // threads per workgroup (the key range one workgroup's tiles cover)
        // and the LDS staging depth
        bool any_large = false;
        for (uint32_t i = 0; i < count; i++) any_large |= batches[i].n > pick;
        if (!any_large) return PI_OK;
        struct Shape {
            uint32_t block, lds;
        };
        const Shape shapes[] = {{1024, 12000}, {1024, 4000}, {512, 6000}, {256, 3000}};
        auto apply = [&](const Shape &sh) {
            for (uint32_t i = 0; i < count; i++) {
                pi::Index &ix = indices[i]->ix;
                ix.cfg.descent_block = sh.block;
                ix.cfg.lds_budget = sh.lds;
                pi::select_lds_levels(ix, ix.desc);
            }
        };
        double best_shape = 1e30;
        Shape keep = shapes[0];
        for (const Shape &sh : shapes) {
            apply(sh);
            double tmin = 1e30;
            for (int rep = 0; rep < 2; rep++) {
                PI_HIP(hipStreamSynchronize(s));
                const auto t0 = std::chrono::steady_clock::now();
                pi::run_group(g, indices, batches, count, s, pick, g->d_zero_ops.as<uint8_t>());
                PI_HIP(hipStreamSynchronize(s));
                const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                tmin = std::min(tmin, dt);
            }
            if (tmin < best_shape) {
                best_shape = tmin;
                keep = sh;
            }
        }
        apply(keep);
        g->tuned_block = keep.block;
        g->tuned_lds = keep.lds;
        return PI_OK;
    });
}

pi_status pi_group_tuning(const pi_group *g, uint64_t *fused_max, uint32_t *descent_block, uint32_t *lds_budget) {
    if (!g || !fused_max || !descent_block || !lds_budget) return PI_ERR_INVALID_ARG;
    *fused_max = g->cfg.fused_max;
    *descent_block = g->tuned_block;
    *lds_budget = g->tuned_lds;
    return PI_OK;
}

const char *pi_group_last_error(const pi_group *g) { return g ? g->err.c_str() : ""; }

}  // extern "C"
