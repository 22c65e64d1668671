// Serving loop: continuous batching of an open-loop arrival schedule (host
// side of pi_serve).
//
// Queries arrive in a fixed order at given times.  A micro-batch is a run of
// consecutive arrivals; it closes when its first query has waited the
// deadline or when it is full, and it is enqueued as one batch of the hot
// path as soon as fewer than max_inflight micro-batches are still on the
// device; an idle device takes what has arrived at once.  While it waits for a slot it keeps admitting arrivals, so the
// batch size follows the load: small batches (low latency) when the device
// keeps up, large ones (high throughput) when it does not.  The host never
// blocks on the device while queries are arriving; it polls the completion
// events of the micro-batches in flight and stamps each query with its
// batch's device completion time.
#include <algorithm>
#include <chrono>
#include <deque>
#include <vector>

#include "index.h"

namespace pi {
namespace {

struct EventPool {
    std::vector<hipEvent_t> all, free;
    explicit EventPool(size_t n) {
        for (size_t i = 0; i < n; i++) {
            hipEvent_t e = nullptr;
            PI_HIP(hipEventCreate(&e));
            all.push_back(e);
            free.push_back(e);
        }
    }
    ~EventPool() {
        for (hipEvent_t e : all) (void)hipEventDestroy(e);
    }
    hipEvent_t take() {
        hipEvent_t e = free.back();
        free.pop_back();
        return e;
    }
    void give(hipEvent_t e) { free.push_back(e); }
};

struct Flight {
    hipEvent_t ev;
    uint64_t b, e;
};

}  // namespace

void pipe_open(Index &ix, hipStream_t s) {
    Index::ServePipe &p = ix.pipe;
    if (!p.side) {
        PI_HIP(hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking));
        PI_HIP(hipEventCreateWithFlags(&p.inputs, hipEventDisableTiming));
        for (auto &b : p.set) {
            PI_HIP(hipEventCreateWithFlags(&b.ordered, hipEventDisableTiming));
            PI_HIP(hipEventCreateWithFlags(&b.done, hipEventDisableTiming));
        }
    }
    // the batch arrays the caller filled on s before this call
    PI_HIP(hipEventRecord(p.inputs, s));
    PI_HIP(hipStreamWaitEvent(p.side, p.inputs, 0));
}

void pipe_release(Index &ix) {
    Index::ServePipe &p = ix.pipe;
    if (p.side) (void)hipStreamSynchronize(p.side);
    for (auto &b : p.set) {
        b.sort.release();
        b.msd.release();
        b.scan.release();
        b.bws.release();
        if (b.ordered) (void)hipEventDestroy(b.ordered);
        if (b.done) (void)hipEventDestroy(b.done);
        b.ordered = b.done = nullptr;
        b.used = false;
    }
    if (p.inputs) (void)hipEventDestroy(p.inputs);
    if (p.side) (void)hipStreamDestroy(p.side);
    p.inputs = nullptr;
    p.side = nullptr;
}

uint64_t serve_batch_limit(uint32_t inflight) {
    size_t freeb = 0, total = 0;
    PI_HIP(hipMemGetInfo(&freeb, &total));
    // per query: batch workspaces (ordering 24 B, descent and ownership
    // results ~55 B) and, for an insert, a node (21 B) and its share of the
    // next rebuild; half of the free memory stays free
    const uint64_t per_query = 128;
    const uint64_t lim = (uint64_t)(freeb / 2) / (per_query * std::max<uint32_t>(inflight, 1));
    return std::max<uint64_t>(1, std::min<uint64_t>(lim, 1u << 22));
}

void serve_loop(const double *arrival, uint64_t n, const ServePlan &plan, hipStream_t s,
                const std::function<void(uint64_t, uint64_t)> &launch, double *done_us, uint64_t *batch_end,
                uint64_t &nb) {
    TraceRange tr("pi:serve");
    EventPool pool(plan.max_inflight + 1);
    hipEvent_t ev0 = pool.take();
    const auto clock0 = std::chrono::steady_clock::now();
    PI_HIP(hipEventRecord(ev0, s));
    auto now_us = [&] {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - clock0).count();
    };
    std::deque<Flight> fl;
    // completion time of each retired micro-batch; the per-query times are
    // written after the loop, so that a large micro-batch's stamping (8 B
    // per query) never delays the next launch
    std::vector<std::pair<uint64_t, double>> stamps;  // (end, time)
    auto fill = [&] {
        uint64_t b = 0;
        for (const auto &st : stamps) {
            std::fill(done_us + b, done_us + st.first, st.second);
            b = st.first;
        }
    };
    auto retire = [&](bool wait) {
        while (!fl.empty()) {
            Flight &f = fl.front();
            if (wait) {
                PI_HIP(hipEventSynchronize(f.ev));
            } else {
                const hipError_t q = hipEventQuery(f.ev);
                if (q == hipErrorNotReady) {
                    (void)hipGetLastError();
                    return;
                }
                PI_HIP(q);
            }
            float ms = 0.f;
            PI_HIP(hipEventElapsedTime(&ms, ev0, f.ev));
            stamps.emplace_back(f.e, (double)ms * 1000.0);
            pool.give(f.ev);
            fl.pop_front();
        }
    };
    uint64_t next = 0;
    nb = 0;
    while (next < n) {
        retire(false);
        const double t = now_us();
        if (arrival[next] > t) continue;  // nothing waiting yet
        const double *lim = arrival + std::min<uint64_t>(n, next + plan.max_batch);
        const uint64_t e = (uint64_t)(std::upper_bound(arrival + next, lim, t) - arrival);
        const bool full = e - next >= plan.max_batch;
        // the deadline bounds the wait; with nothing on the device there is
        // nothing to wait for
        const bool due = fl.empty() || t >= arrival[next] + plan.deadline_us;
        if (!full && !due) continue;                  // still collecting
        if (fl.size() >= plan.max_inflight) continue;  // no slot: keep admitting
        try {
            launch(next, e);
        } catch (...) {
            // the micro-batches before this one took effect: stamp them and
            // report them (nb) before passing the error on
            try {
                while (!fl.empty()) retire(true);
                fill();
            } catch (...) {
            }
            throw;
        }
        Flight f{pool.take(), next, e};
        PI_HIP(hipEventRecord(f.ev, s));
        fl.push_back(f);
        batch_end[nb++] = e;
        next = e;
    }
    while (!fl.empty()) retire(true);
    fill();
}

}  // namespace pi
