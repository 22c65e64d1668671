// Background rebuild of the index layer (Section 4.3.5).
//
// The paper keeps the storage layer as it is and has a background thread
// rebuild only the index layer: it walks the storage layer, collects every
// valid node of height > 1 and swaps the new index layer in once the current
// batch is done.  Here the storage layer is the base region (sorted slots)
// plus the nodes inserted since the last full rebuild (one sorted run per
// batch, linked into the list), and the rebuild runs on a second stream while
// batches go on:
//
//   count  (phase 1) the new nodes present when the rebuild starts -- slots
//          [first, snap) -- are ordered by key (the batch ordering), deleted
//          ones dropped, and counted per level of their tower; the counts go
//          to the host
//   build  (phase 2) level 2 is the merge (by rank) of the base keys of height
//          >= 2 with the new ones, each with its storage slot; the higher
//          levels are filtered from it as in a full rebuild, into a second
//          arena
//   switch at the next batch boundary after the build is done, the descent
//          uses the new arena; the old one becomes the next build's target
//
// Nothing waits: the phases move on when their events have completed, at the
// start of later batches.  Correctness does not depend on the snapshot: an
// interception only needs to be some node of the list with key <= q, and no
// node leaves the list before a full rebuild -- nodes inserted after the
// snapshot are reached through the links, nodes deleted after it are
// flagged.  The storage itself is merged (deleted nodes dropped, new nodes
// moved into the base region) by a full rebuild only when new and deleted
// nodes reach compact_percent of the base region.
#include <algorithm>

#include "descent.h"

namespace pi {
namespace {

constexpr int GT = 256;

// new nodes [first, snap): key (deleted -> +infinity so that it sorts last
// and is not indexed)
__global__ void k_bg_gather(const uint64_t *__restrict__ skey, const uint8_t *__restrict__ smeta, uint64_t first,
                            uint64_t n, uint64_t *__restrict__ okeys) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    okeys[i] = (smeta[first + i] & META_DEL) ? KEY_MAX : skey[first + i];
}

__global__ void k_bg_zero(uint32_t *__restrict__ p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// counts of the valid new keys per level of their tower (cnt[l], l >= 2)
__global__ __launch_bounds__(GT) void k_bg_count(const uint64_t *__restrict__ sk, uint64_t n, uint64_t seed,
                                                 uint32_t l2p, uint32_t maxh, uint32_t *__restrict__ cnt) {
    __shared__ uint32_t h[MAX_LEVELS + 1];
    if (threadIdx.x <= MAX_LEVELS) h[threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * GT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * GT) {
        const uint64_t k = sk[i];
        if (k != KEY_MAX) atomicAdd(&h[tower_height(k, seed, l2p, maxh)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < MAX_LEVELS && threadIdx.x >= 2) {
        uint32_t c = 0;
        for (int x = threadIdx.x; x <= MAX_LEVELS; x++) c += h[x];
        if (c) atomicAdd(&cnt[threadIdx.x], c);
    }
}

// flags of height >= 2: base keys (keys[0..n) = slots 1..n) or sorted new keys
__global__ void k_bg_flag2(const uint64_t *__restrict__ keys, uint64_t n, uint64_t seed, uint32_t l2p,
                           uint32_t maxh, uint32_t *__restrict__ flags) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    flags[i] = (k != KEY_MAX && tower_height(k, seed, l2p, maxh) >= 2) ? 1u : 0u;
}

// compaction: out[pos[i]] = (key i, its storage slot) for flagged i; the slot
// is base + i, or first + rel[i] for the sorted new keys
__global__ void k_bg_compact(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ rel, uint64_t n,
                             uint64_t slot0, uint64_t cap, const uint32_t *__restrict__ flags,
                             const uint32_t *__restrict__ pos, uint64_t *__restrict__ okey,
                             uint32_t *__restrict__ oslot) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flags[i]) return;
    const uint32_t p = pos[i];
    if (p >= cap) return;
    okey[p] = keys[i];
    oslot[p] = (uint32_t)(slot0 + (rel ? rel[i] : i));
}

// merge by rank of two sorted key sets with no key in common: element i of a
// lands at i + (number of keys of b below it); positions past m are dropped
__global__ void k_bg_merge(const uint64_t *__restrict__ ak, const uint32_t *__restrict__ as, uint64_t na,
                           const uint64_t *__restrict__ bk, uint64_t nb, uint64_t m, uint64_t *__restrict__ mk,
                           uint32_t *__restrict__ ms) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= na) return;
    const uint64_t k = ak[i];
    uint64_t lo = 0, hi = nb;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (bk[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (i + lo < m) {
        mk[i + lo] = k;
        ms[i + lo] = as[i];
    }
}

uint32_t grid_of(uint64_t n, int t) { return (uint32_t)std::max<uint64_t>(1, (n + t - 1) / t); }

// keys[0..n) flagged by height >= 2 -> (key, slot) at their rank, at most cap
void compact2(Index &ix, const uint64_t *keys, const uint32_t *rel, uint64_t n, uint64_t slot0, uint64_t cap,
              DevBuf &okey, DevBuf &oslot, hipStream_t s) {
    Index::Background &b = ix.bg;
    if (n == 0) return;
    hipLaunchKernelGGL(k_bg_flag2, dim3(grid_of(n, GT)), dim3(GT), 0, s, keys, n, ix.cfg.height_seed,
                       ix.cfg.log2_inv_p, ix.cfg.max_height, b.flags.as<uint32_t>());
    exclusive_scan_u32(b.scanws, b.flags.as<uint32_t>(), b.pos.as<uint32_t>(), n, b.cnt.as<uint32_t>() + 40,
                       nullptr, s);
    hipLaunchKernelGGL(k_bg_compact, dim3(grid_of(n, GT)), dim3(GT), 0, s, keys, rel, n, slot0, cap,
                       b.flags.as<uint32_t>(), b.pos.as<uint32_t>(), okey.as<uint64_t>(), oslot.as<uint32_t>());
    PI_LAUNCH_CHECK();
}

void build_phase(Index &ix) {
    Index::Background &b = ix.bg;
    hipStream_t s = b.side;
    const uint64_t novf = b.snap - b.first;
    uint32_t level_n[MAX_LEVELS] = {};
    for (int l = 2; l < MAX_LEVELS; l++) level_n[l] = ix.base_level_n[l] + b.h_cnt[l];
    uint64_t total = 0;
    b.desc = make_desc(ix, level_n, &total);
    if (b.desc.top < 2) return;
    if (b.akey.bytes < total * 8) b.akey.ensure(total * 8 * 5 / 4);
    if (b.adown.bytes < total * 4) b.adown.ensure(total * 4 * 5 / 4);
    const uint64_t nb = ix.nbase;
    const uint64_t nb2 = ix.base_level_n[2], no2 = b.h_cnt[2], m2 = nb2 + no2;
    const uint64_t nmax = std::max<uint64_t>(std::max<uint64_t>(nb, novf), 1);
    b.flags.ensure(nmax * 4);
    b.pos.ensure(nmax * 4);
    b.b2key.ensure(std::max<uint64_t>(nb2, 1) * 8);
    b.b2slot.ensure(std::max<uint64_t>(nb2, 1) * 4);
    b.o2key.ensure(std::max<uint64_t>(no2, 1) * 8);
    b.o2slot.ensure(std::max<uint64_t>(no2, 1) * 4);
    b.m2key.ensure(std::max<uint64_t>(m2, 1) * 8);
    b.m2slot.ensure(std::max<uint64_t>(m2, 1) * 4);
    // level 2: base keys of height >= 2 (slot 1 + position) merged with the
    // new ones (slot first + position in the run)
    compact2(ix, ix.st.key.as<uint64_t>() + 1, nullptr, nb, 1, nb2, b.b2key, b.b2slot, s);
    compact2(ix, b.sk, b.si, novf, b.first, no2, b.o2key, b.o2slot, s);
    if (nb2)
        hipLaunchKernelGGL(k_bg_merge, dim3(grid_of(nb2, GT)), dim3(GT), 0, s, b.b2key.as<uint64_t>(),
                           b.b2slot.as<uint32_t>(), nb2, b.o2key.as<uint64_t>(), no2, m2, b.m2key.as<uint64_t>(),
                           b.m2slot.as<uint32_t>());
    if (no2)
        hipLaunchKernelGGL(k_bg_merge, dim3(grid_of(no2, GT)), dim3(GT), 0, s, b.o2key.as<uint64_t>(),
                           b.o2slot.as<uint32_t>(), no2, b.b2key.as<uint64_t>(), nb2, m2, b.m2key.as<uint64_t>(),
                           b.m2slot.as<uint32_t>());
    PI_LAUNCH_CHECK();
    // every level from level 2, as in a full rebuild
    scatter_levels(ix, b.m2key.as<uint64_t>(), b.m2slot.as<uint32_t>(), m2, b.desc, b.tcnt, b.ttot, b.akey, b.adown,
                   s);
}

}  // namespace

// The side stream, its events and the pinned count buffer (made once; at
// load time under the background policy, so that no batch call makes them).
static void bg_open(Index &ix) {
    Index::Background &b = ix.bg;
    if (b.side) return;
    PI_HIP(hipStreamCreateWithFlags(&b.side, hipStreamNonBlocking));
    PI_HIP(hipEventCreateWithFlags(&b.ev_main, hipEventDisableTiming));
    PI_HIP(hipEventCreateWithFlags(&b.ev_side, hipEventDisableTiming));
    PI_HIP(hipHostMalloc(&b.h_cnt, 64 * sizeof(uint32_t), hipHostMallocDefault));
}

void bg_start(Index &ix, const DevState &latest, hipStream_t s) {
    Index::Background &b = ix.bg;
    if (b.phase != 0) return;
    const uint64_t first = ix.nbase + 2;
    if (latest.nused <= first) return;  // no new node to index
    bg_open(ix);
    b.first = first;
    b.snap = latest.nused;
    b.changes_at = latest.changes;
    b.live_at = latest.n_live;
    const uint64_t novf = b.snap - b.first;
    // the side stream starts after every batch enqueued so far: the new
    // nodes below snap are written and visible
    PI_HIP(hipEventRecord(b.ev_main, s));
    PI_HIP(hipStreamWaitEvent(b.side, b.ev_main, 0));
    b.okeys.ensure(novf * 8);
    b.cnt.ensure(64 * sizeof(uint32_t));
    hipLaunchKernelGGL(k_bg_gather, dim3(grid_of(novf, GT)), dim3(GT), 0, b.side, ix.st.key.as<uint64_t>(),
                       ix.st.meta.as<uint8_t>(), b.first, novf, b.okeys.as<uint64_t>());
    PI_LAUNCH_CHECK();
    sort_batch_by_range(b.sortws, b.msdws, b.okeys.as<uint64_t>(), nullptr, novf, false, b.side,
                        &b.sk, &b.si);
    hipLaunchKernelGGL(k_bg_zero, dim3(1), dim3(64), 0, b.side, b.cnt.as<uint32_t>(), 64u);
    hipLaunchKernelGGL(k_bg_count, dim3(std::min<uint32_t>(grid_of(novf, GT), 1024)), dim3(GT), 0, b.side, b.sk,
                       novf, ix.cfg.height_seed, ix.cfg.log2_inv_p, ix.cfg.max_height, b.cnt.as<uint32_t>());
    PI_LAUNCH_CHECK();
    PI_HIP(hipMemcpyAsync(b.h_cnt, b.cnt.p, MAX_LEVELS * sizeof(uint32_t), hipMemcpyDeviceToHost, b.side));
    PI_HIP(hipEventRecord(b.ev_side, b.side));
    b.phase = 1;
}

void bg_advance(Index &ix) {
    Index::Background &b = ix.bg;
    if (b.phase == 0) return;
    const hipError_t q = hipEventQuery(b.ev_side);
    if (q == hipErrorNotReady) {
        (void)hipGetLastError();
        return;
    }
    PI_HIP(q);
    if (b.phase == 1) {
        build_phase(ix);
        if (b.desc.top < 2) {
            b.phase = 0;
            return;
        }
        PI_HIP(hipEventRecord(b.ev_side, b.side));
        b.phase = 2;
        return;
    }
    // phase 2 done: switch the descent to the new levels; the old arena is the
    // next build's target (the next build waits for every batch enqueued
    // before it starts)
    std::swap(ix.arena_key, b.akey);
    std::swap(ix.arena_down, b.adown);
    ix.desc = b.desc;
    ix.changes_base = b.changes_at;
    ix.live_at_rebuild = b.live_at;
    b.done++;
    b.phase = 0;
}

void bg_release(Index &ix) {
    Index::Background &b = ix.bg;
    if (b.side) {
        (void)hipStreamSynchronize(b.side);
        (void)hipStreamDestroy(b.side);
    }
    if (b.ev_main) (void)hipEventDestroy(b.ev_main);
    if (b.ev_side) (void)hipEventDestroy(b.ev_side);
    if (b.h_cnt) (void)hipHostFree(b.h_cnt);
    b.side = nullptr;
    b.ev_main = b.ev_side = nullptr;
    b.h_cnt = nullptr;
    b.sortws.release();
    b.msdws.release();
    b.scanws.release();
    for (DevBuf *d : {&b.okeys, &b.flags, &b.pos, &b.cnt, &b.b2key, &b.b2slot, &b.o2key, &b.o2slot, &b.m2key,
                      &b.m2slot, &b.tcnt, &b.ttot, &b.akey, &b.adown})
        d->release();
    b.phase = 0;
}

void bg_reserve(Index &ix) {
    if (ix.cfg.rebuild_policy != PI_REBUILD_BACKGROUND) return;
    bg_open(ix);
    Index::Background &b = ix.bg;
    const uint64_t cap = std::max<uint64_t>(ix.st.cap, 1);
    b.okeys.ensure(cap * 8);
    b.cnt.ensure(64 * sizeof(uint32_t));
    b.sortws.ensure(cap);
    b.msdws.ensure(cap);
    b.scanws.ensure(cap);
    b.flags.ensure(cap * 4);
    b.pos.ensure(cap * 4);
    for (DevBuf *k : {&b.b2key, &b.o2key, &b.m2key}) k->ensure(cap * 8);
    for (DevBuf *k : {&b.b2slot, &b.o2slot, &b.m2slot}) k->ensure(cap * 4);
    scatter_reserve(b.tcnt, b.ttot, cap);
    const uint64_t e = arena_entries_for(cap);
    b.akey.ensure(e * 8);
    b.adown.ensure(e * 4);
}

void bg_quiesce(Index &ix) {
    if (ix.bg.phase == 0) return;
    PI_HIP(hipStreamSynchronize(ix.bg.side));
    ix.bg.phase = 0;
}

}  // namespace pi
