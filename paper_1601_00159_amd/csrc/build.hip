// Construction of the storage base region and the index layer.
//
// Section 3.1: the index layer is built bottom-up by one scan of the ordered
// storage layer; Section 4.1: the scan can be split over workers, each
// building its part of every level, the parts being concatenated level by
// level.  Here a block owns a 4096-node tile of the base region: one pass
// counts, per tile, how many of its keys reach each level (heights come from
// the key), a column scan turns the counts into each tile's offset on each
// level, and a second pass writes every key into all the levels it reaches,
// with its position on the level below as the down pointer.
//
// A rebuild (Section 4.3.5: rebuild the whole index layer from the storage
// layer once enough updates have accumulated, keeping only valid nodes)
// merges the base region with the nodes created since the last rebuild,
// drops deleted nodes, and rebuilds every level from the merged region.
#include <algorithm>
#include <vector>

#include "index.h"

namespace pi {
namespace {

constexpr int BT = 256;
constexpr int BI = 16;
constexpr int BTILE = BT * BI;
constexpr int BNW = BT / 64;

// ---- level construction ----------------------------------------------------

// keys[0 .. n) in increasing order; counts per tile and level of the keys
// whose tower reaches the level
__global__ __launch_bounds__(BT) void k_height_count(const uint64_t *__restrict__ keys, uint32_t nbase,
                                                     uint64_t seed, uint32_t l2p, uint32_t maxh,
                                                     uint32_t *__restrict__ cnt, uint32_t ntiles) {
    __shared__ uint32_t h[MAX_LEVELS + 1];
    const int tid = threadIdx.x;
    if (tid <= MAX_LEVELS) h[tid] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * BTILE;
    for (int j = 0; j < BI; j++) {
        const uint32_t b = base + j * BT + tid;
        if (b < nbase) atomicAdd(&h[tower_height(keys[b], seed, l2p, maxh)], 1u);
    }
    __syncthreads();
    if (tid < MAX_LEVELS) {
        uint32_t c = 0;
        for (int x = tid; x <= MAX_LEVELS; x++) c += h[x];
        cnt[(size_t)tid * ntiles + blockIdx.x] = tid >= 2 ? c : 0u;
    }
}

// writes keys[0 .. n) into every level their tower reaches; the level-2 down
// pointer is slots[b] (the storage slot), or 1 + b when slots is null (the
// base region)
__global__ __launch_bounds__(BT) void k_level_scatter(const uint64_t *__restrict__ keys,
                                                      const uint32_t *__restrict__ slots, uint32_t nbase,
                                                      uint64_t seed, uint32_t l2p, uint32_t maxh,
                                                      const uint32_t *__restrict__ tileoff, uint32_t ntiles,
                                                      IndexDesc desc, uint64_t *__restrict__ lkey,
                                                      uint32_t *__restrict__ ldown, uint32_t first_level) {
    __shared__ uint32_t s_cnt[BNW][MAX_LEVELS];
    __shared__ uint32_t s_toff[MAX_LEVELS];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid >> 6;
    for (int j = tid; j < BNW * MAX_LEVELS; j += BT) (&s_cnt[0][0])[j] = 0;
    if (tid < MAX_LEVELS) s_toff[tid] = tileoff[(size_t)tid * ntiles + blockIdx.x];  // rows 0,1 are zero
    __syncthreads();

    const uint32_t wbase = blockIdx.x * BTILE + w * (BI * 64);
    uint64_t k[BI];
    uint32_t h[BI];
#pragma unroll
    for (int r = 0; r < BI; r++) {
        const uint32_t b = wbase + r * 64 + lane;
        if (b < nbase) {
            k[r] = keys[b];
            h[r] = tower_height(k[r], seed, l2p, maxh);
        } else {
            k[r] = KEY_MAX;
            h[r] = 0;
        }
    }
    // keys of this wave per level
#pragma unroll
    for (int r = 0; r < BI; r++) {
        for (uint32_t l = first_level;; l++) {
            const uint64_t m = ballot64(h[r] >= l);
            if (!m) break;
            if (lane == 0) s_cnt[w][l] += (uint32_t)__popcll(m);
        }
    }
    __syncthreads();
    if (tid < MAX_LEVELS) {
        uint32_t run = 0;
        for (int ww = 0; ww < BNW; ww++) {
            const uint32_t c = s_cnt[ww][tid];
            s_cnt[ww][tid] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < BI; r++) {
        const uint32_t b = wbase + r * 64 + lane;
        // down pointer on first_level: the storage slot (level 2) or the
        // position one level below
        uint32_t prev = slots ? (b < nbase ? slots[b] : 0u) : 1 + b;
        for (uint32_t l = first_level;; l++) {
            const bool in = h[r] >= l;
            const uint64_t m = ballot64(in);
            if (!m) break;
            const uint32_t before = s_cnt[w][l];
            if (in) {
                const uint32_t p = 1 + s_toff[l] + before + mask_rank(m);
                if (p <= desc.n[l]) {  // sizes come from a separate count; never write past the level
                    lkey[desc.off[l] + p] = k[r];
                    ldown[desc.off[l] + p] = prev;
                }
                prev = p;
            }
            if (lane == 0) s_cnt[w][l] = before + (uint32_t)__popcll(m);
        }
    }
}

__global__ void k_level_pad(IndexDesc desc, uint64_t *__restrict__ lkey, uint32_t *__restrict__ ldown) {
    const int l = blockIdx.x;
    if (l < 2 || l > desc.top) return;
    const uint64_t o = desc.off[l];
    if (threadIdx.x == 0) {
        lkey[o] = 0;
        ldown[o] = 0;
    }
    if (threadIdx.x < LEVEL_PAD) {
        lkey[o + desc.n[l] + 1 + threadIdx.x] = KEY_MAX;
        ldown[o + desc.n[l] + 1 + threadIdx.x] = 0;
    }
}

// ---- bulk load ---------------------------------------------------------------

__global__ void k_last_of_run(const uint64_t *__restrict__ sk, uint32_t n, uint32_t *__restrict__ flag) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = sk[i];
    flag[i] = (k != KEY_MAX && (i + 1 == n || sk[i + 1] != k)) ? 1u : 0u;
}

__global__ void k_write_base(const uint64_t *__restrict__ sk, const uint32_t *__restrict__ sidx,
                             const uint64_t *__restrict__ vals, const uint32_t *__restrict__ flag,
                             const uint32_t *__restrict__ pos, uint32_t n, uint64_t *__restrict__ skey,
                             uint64_t *__restrict__ sval, uint8_t *__restrict__ smeta) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const uint64_t slot = 1 + (uint64_t)pos[i];
    skey[slot] = sk[i];
    sval[slot] = vals[sidx[i]];
    smeta[slot] = 0;
}

// head at slot 0 (successor slot 1), tail at nbase+1, and the counters
__global__ void k_reset_region(uint64_t *__restrict__ skey, uint64_t *__restrict__ sval,
                               uint32_t *__restrict__ snext, uint8_t *__restrict__ smeta, uint64_t nbase,
                               DevState *st, int reset_stats) {
    if (threadIdx.x != 0) return;
    skey[0] = 0;
    sval[0] = 0;
    snext[0] = 0;
    smeta[0] = 0;
    skey[nbase + 1] = KEY_MAX;
    sval[nbase + 1] = 0;
    snext[nbase + 1] = 0;
    smeta[nbase + 1] = 0;
    st->nused = nbase + 2;
    st->n_live = nbase;
    st->changes = 0;
    st->has_links = 0;
    st->has_dead = 0;
    if (reset_stats) {
        st->batches = st->queries = st->hits = st->invalid = 0;
        st->new_nodes = st->deletes = st->revives = 0;
        st->errors = 0;
    }
    st->b_writers = st->b_new = st->b_deletes = st->b_revives = st->b_hits = st->b_invalid = 0;
    st->b_n = 0;
    st->b_pad = 0;
}

// ---- merge of the base region with the overflow nodes -----------------------

// For each sorted overflow node: live flag, and p = number of base keys
// smaller than its key (binary search; keys are unique across the list).
__global__ void k_ovf_place(const uint64_t *__restrict__ osk, const uint32_t *__restrict__ orel, uint32_t first,
                            uint64_t novf,
                            const uint64_t *__restrict__ skey, const uint8_t *__restrict__ smeta, uint64_t nbase,
                            uint32_t *__restrict__ olive, uint32_t *__restrict__ opos,
                            uint32_t *__restrict__ hist) {
    const uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= novf) return;
    const uint64_t k = osk[o];
    uint64_t lo = 0, hi = nbase;  // search base slots 1..nbase
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (skey[1 + mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    const uint32_t live = (smeta[first + orel[o]] & META_DEL) ? 0u : 1u;
    olive[o] = live;
    opos[o] = (uint32_t)lo;
    if (live) atomicAdd(&hist[lo], 1u);
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// out position of live base node b = (live base before b) + (live overflow
// nodes placed at or before b); of live overflow node o = (live base before
// its place) + (live overflow before o).
__global__ void k_merge_base(const uint64_t *__restrict__ skey, const uint64_t *__restrict__ sval,
                             const uint8_t *__restrict__ smeta, uint64_t nbase, const uint32_t *__restrict__ A,
                             const uint32_t *__restrict__ Bexcl, const uint32_t *__restrict__ H,
                             uint64_t *__restrict__ okey, uint64_t *__restrict__ oval,
                             uint8_t *__restrict__ ometa, uint64_t slot_off, uint64_t lim, unsigned int *errors) {
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbase) return;
    if (smeta[1 + b] & META_DEL) return;
    const uint64_t o = slot_off + A[b] + Bexcl[b] + H[b];
    if (o >= lim) {  // more live flags than the live counter allows (flagged by the check)
        atomicOr(errors, ERR_LIVE);
        return;
    }
    okey[o] = skey[1 + b];
    oval[o] = sval[1 + b];
    if (ometa) ometa[o] = 0;
}

__global__ void k_merge_ovf(const uint64_t *__restrict__ osk, const uint32_t *__restrict__ orel, uint32_t first,
                            uint64_t novf,
                            const uint64_t *__restrict__ sval, const uint32_t *__restrict__ olive,
                            const uint32_t *__restrict__ C, const uint32_t *__restrict__ opos,
                            const uint32_t *__restrict__ A, uint64_t *__restrict__ okey,
                            uint64_t *__restrict__ oval, uint8_t *__restrict__ ometa, uint64_t slot_off, uint64_t lim,
                            unsigned int *errors) {
    const uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= novf || !olive[o]) return;
    const uint64_t d = slot_off + A[opos[o]] + C[o];
    if (d >= lim) {
        atomicOr(errors, ERR_LIVE);
        return;
    }
    okey[d] = osk[o];
    oval[d] = sval[first + orel[o]];
    if (ometa) ometa[d] = 0;
}

uint32_t blocks_for(uint64_t n, int t) { return (uint32_t)((n + t - 1) / t); }

}  // namespace

// Storage slots beyond the live keys after a bulk load or a storage merge.
// Under the background policy the storage is merged only when new + deleted
// nodes reach compact_percent of the base region, so the room covers that
// many new nodes (plus a quarter): the storage then never grows in between.
uint64_t storage_room(const Index &ix, uint64_t live) {
    uint64_t room = std::max<uint64_t>(live / 4, 1 << 16);
    if (ix.cfg.rebuild_policy == PI_REBUILD_BACKGROUND) {
        const uint64_t pct = ix.cfg.compact_percent ? ix.cfg.compact_percent : 100;
        room += live * pct / 100;
    }
    return room;
}

// Index entries an arena needs for any index over a storage of cap slots.
uint64_t arena_entries_for(uint64_t cap) { return cap + (uint64_t)MAX_LEVELS * (1 + LEVEL_PAD + 16); }

void scatter_reserve(DevBuf &cnt, DevBuf &tot, uint64_t n) {
    cnt.ensure((size_t)MAX_LEVELS * blocks_for(std::max<uint64_t>(n, 1), BTILE) * sizeof(uint32_t));
    tot.ensure(MAX_LEVELS * sizeof(uint32_t));
}

// STORAGE_SLACK slots past the capacity keep the speculative reads of the
// storage walk (up to two slots past a node) inside the allocation.  The
// four arrays share one allocation (each array 256-byte aligned): a fourth
// of the allocations and frees.  Unless exact, the capacity takes whatever
// the allocation's rounding leaves room for.
void Storage::alloc(uint64_t c, bool exact) {
    constexpr uint64_t BYTES_PER_SLOT = 8 + 8 + 4 + 1, ALIGN_PAD = 4 * 256;
    auto up = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
    all.ensure((c + STORAGE_SLACK) * BYTES_PER_SLOT + ALIGN_PAD);
    uint64_t phys = c + STORAGE_SLACK;
    if (!exact) phys = std::max<uint64_t>(phys, (all.bytes - ALIGN_PAD) / BYTES_PER_SLOT);
    cap = phys - STORAGE_SLACK;
    const uint64_t o_val = up(phys * 8), o_next = o_val + up(phys * 8), o_meta = o_next + up(phys * 4);
    auto view = [&](uint64_t off, uint64_t bytes) {
        DevBuf v;
        v.p = static_cast<uint8_t *>(all.p) + off;
        v.bytes = bytes;
        return v;
    };
    key = view(0, phys * 8);
    val = view(o_val, phys * 8);
    next = view(o_next, phys * 4);
    meta = view(o_meta, phys);
}

void Storage::release() {
    all.release();
    key = val = next = meta = DevBuf{};
    cap = 0;
}

void read_state(Index &ix, hipStream_t s, DevState *out) {
    PI_HIP(hipMemcpyAsync(ix.hstate, ix.dstate, sizeof(DevState), hipMemcpyDeviceToHost, s));
    PI_HIP(hipStreamSynchronize(s));
    *out = *ix.hstate;
    ix.used_upper = out->nused;
    if (out->errors) throw Error{PI_ERR_DEVICE, device_error_text(out->errors)};
}

// Level sizes -> descriptor: 128-byte aligned levels in one arena, and the
// top levels that fit the descent's LDS budget (Section 5.1 notes the top
// levels are cache resident anyway; Section 7 proposes pinning them).
IndexDesc make_desc(const Index &ix, const uint32_t *level_n, uint64_t *arena_entries) {
    IndexDesc d{};
    d.top = 1;
    d.lds_from = MAX_LEVELS;
    const uint32_t maxh = ix.cfg.max_height;
    for (int l = 2; l < MAX_LEVELS && l <= (int)maxh; l++) {
        d.n[l] = level_n[l];
        if (level_n[l] > 0) d.top = l;
    }
    uint64_t total = 0;
    for (int l = 2; l <= d.top; l++) {
        d.off[l] = total;
        total += ((uint64_t)d.n[l] + 1 + LEVEL_PAD + 15) & ~15ull;
    }
    *arena_entries = total;
    select_lds_levels(ix, d);
    return d;
}

// The top levels that fit the descent's LDS budget (and the lds_levels cap).
void select_lds_levels(const Index &ix, IndexDesc &d) {
    const uint32_t budget = ix.cfg.lds_budget ? ix.cfg.lds_budget : 12000;  // 12000 entries: 141 KB per block
    uint32_t used = 0;
    int from = d.top + 1;
    const uint32_t want = ix.cfg.lds_levels ? ix.cfg.lds_levels : 64u;
    for (int l = d.top; l >= 2 && (uint32_t)(d.top - l) < want; l--) {
        const uint32_t e = d.n[l] + 1 + LEVEL_PAD;
        if (used + e > budget) break;
        d.lds_off[l] = used;
        used += e;
        from = l;
    }
    d.lds_from = d.top >= 2 ? from : MAX_LEVELS;
    d.lds_entries = used;
}

// Writes the levels of d from keys[0 .. n) (increasing; level-2 down
// pointers from slots, or 1 + position when slots is null) into the arena.
// Asynchronous on s; cnt is per-tile scratch.
void scatter_levels(const Index &ix, const uint64_t *keys, const uint32_t *slots, uint64_t n, const IndexDesc &d,
                    DevBuf &cnt, DevBuf &tot, DevBuf &akey, DevBuf &adown, hipStream_t s, uint32_t first_level) {
    if (n == 0 || d.top < (int)first_level) return;
    const uint32_t ntiles = blocks_for(n, BTILE);
    cnt.ensure((size_t)MAX_LEVELS * ntiles * sizeof(uint32_t));
    tot.ensure(MAX_LEVELS * sizeof(uint32_t));
    hipLaunchKernelGGL(k_height_count, dim3(ntiles), dim3(BT), 0, s, keys, (uint32_t)n, ix.cfg.height_seed,
                       ix.cfg.log2_inv_p, ix.cfg.max_height, cnt.as<uint32_t>(), ntiles);
    PI_LAUNCH_CHECK();
    column_scan(cnt.as<uint32_t>(), MAX_LEVELS, ntiles, tot.as<uint32_t>(), s);
    hipLaunchKernelGGL(k_level_scatter, dim3(ntiles), dim3(BT), 0, s, keys, slots, (uint32_t)n, ix.cfg.height_seed,
                       ix.cfg.log2_inv_p, ix.cfg.max_height, cnt.as<uint32_t>(), ntiles, d, akey.as<uint64_t>(),
                       adown.as<uint32_t>(), first_level);
    hipLaunchKernelGGL(k_level_pad, dim3(MAX_LEVELS), dim3(64), 0, s, d, akey.as<uint64_t>(), adown.as<uint32_t>());
    PI_LAUNCH_CHECK();
}

void level_totals(Index &ix, const uint64_t *keys, uint64_t n, DevBuf &cnt, DevBuf &tot, uint32_t *level_n,
                  hipStream_t s) {
    for (int l = 0; l < MAX_LEVELS; l++) level_n[l] = 0;
    if (n == 0) return;
    const uint32_t ntiles = blocks_for(n, BTILE);
    cnt.ensure((size_t)MAX_LEVELS * ntiles * sizeof(uint32_t));
    tot.ensure(MAX_LEVELS * sizeof(uint32_t));
    hipLaunchKernelGGL(k_height_count, dim3(ntiles), dim3(BT), 0, s, keys, (uint32_t)n, ix.cfg.height_seed,
                       ix.cfg.log2_inv_p, ix.cfg.max_height, cnt.as<uint32_t>(), ntiles);
    PI_LAUNCH_CHECK();
    column_scan(cnt.as<uint32_t>(), MAX_LEVELS, ntiles, tot.as<uint32_t>(), s);
    uint32_t *h = reinterpret_cast<uint32_t *>(ix.hcounts);
    PI_HIP(hipMemcpyAsync(h, tot.p, MAX_LEVELS * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    PI_HIP(hipStreamSynchronize(s));
    for (int l = 0; l < MAX_LEVELS; l++) level_n[l] = h[l];
}

void pad_levels(Index &ix, const IndexDesc &d, hipStream_t s) {
    hipLaunchKernelGGL(k_level_pad, dim3(MAX_LEVELS), dim3(64), 0, s, d, ix.arena_key.as<uint64_t>(),
                       ix.arena_down.as<uint32_t>());
    PI_LAUNCH_CHECK();
}

// Builds every index level from base slots 1..nbase.  Waits for the level
// sizes.
static void build_levels(Index &ix, hipStream_t s) {
    if (ix.cfg.rebuild_policy == PI_REBUILD_SLICES) {
        slice_build(ix, s);
        return;
    }
    const uint64_t nb = ix.nbase;
    uint32_t level_n[MAX_LEVELS] = {};
    if (nb > 0) {
        const uint32_t ntiles = blocks_for(nb, BTILE);
        DevBuf &cnt = ix.tmp[8];  // not the merge's buffers: the merge may still be running
        DevBuf &tot = ix.tmp[9];
        cnt.ensure((size_t)MAX_LEVELS * ntiles * sizeof(uint32_t));
        tot.ensure(MAX_LEVELS * sizeof(uint32_t));
        hipLaunchKernelGGL(k_height_count, dim3(ntiles), dim3(BT), 0, s, ix.st.key.as<uint64_t>() + 1, (uint32_t)nb,
                           ix.cfg.height_seed, ix.cfg.log2_inv_p, ix.cfg.max_height, cnt.as<uint32_t>(), ntiles);
        PI_LAUNCH_CHECK();
        column_scan(cnt.as<uint32_t>(), MAX_LEVELS, ntiles, tot.as<uint32_t>(), s);
        uint32_t *htot = reinterpret_cast<uint32_t *>(ix.hcounts);
        PI_HIP(hipMemcpyAsync(htot, tot.p, MAX_LEVELS * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        PI_HIP(hipStreamSynchronize(s));
        for (int l = 0; l < MAX_LEVELS; l++) level_n[l] = htot[l];
    }
    uint64_t total = 0;
    IndexDesc d = make_desc(ix, level_n, &total);
    if (nb > 0 && d.top >= 2) {
        // a quarter of headroom: levels grow with the inserts between
        // rebuilds, and reallocating costs more than the spare bytes
        // (the background policy sizes it for the whole storage: its rebuilds
        // build into the other arena while batches run, and must not wait)
        const uint64_t want = ix.cfg.rebuild_policy == PI_REBUILD_BACKGROUND
                                  ? std::max<uint64_t>(total, arena_entries_for(ix.st.cap))
                                  : total * 5 / 4;
        if (ix.arena_key.bytes < total * sizeof(uint64_t)) ix.arena_key.ensure(want * sizeof(uint64_t));
        if (ix.arena_down.bytes < total * sizeof(uint32_t)) ix.arena_down.ensure(want * sizeof(uint32_t));
        const uint32_t ntiles = blocks_for(nb, BTILE);
        hipLaunchKernelGGL(k_level_scatter, dim3(ntiles), dim3(BT), 0, s, ix.st.key.as<uint64_t>() + 1, nullptr,
                           (uint32_t)nb, ix.cfg.height_seed, ix.cfg.log2_inv_p, ix.cfg.max_height,
                           ix.tmp[8].as<uint32_t>(), ntiles, d, ix.arena_key.as<uint64_t>(),
                           ix.arena_down.as<uint32_t>(), 2u);
        hipLaunchKernelGGL(k_level_pad, dim3(MAX_LEVELS), dim3(64), 0, s, d, ix.arena_key.as<uint64_t>(),
                           ix.arena_down.as<uint32_t>());
        PI_LAUNCH_CHECK();
    }
    ix.desc = d;
    // the base levels: what a background index rebuild adds the new nodes to
    for (int l = 0; l < MAX_LEVELS; l++) ix.base_level_n[l] = level_n[l];
}

void init_empty(Index &ix, hipStream_t s) {
    ix.nbase = 0;
    hipLaunchKernelGGL(k_reset_region, dim3(1), dim3(64), 0, s, ix.st.key.as<uint64_t>(), ix.st.val.as<uint64_t>(),
                       ix.st.next.as<uint32_t>(), ix.st.meta.as<uint8_t>(), (uint64_t)0, ix.dstate, 1);
    PI_LAUNCH_CHECK();
    ix.used_upper = 2;
    ix.live_at_rebuild = 0;
    build_levels(ix, s);
}

void grow_storage(Index &ix, uint64_t need, uint64_t want, hipStream_t s) {
    if (need <= ix.st.cap) return;
    bg_quiesce(ix);
    DevState cur;
    read_state(ix, s, &cur);
    // into the spare storage (the one the last rebuild replaced) when it is
    // large enough, else into a new one; of the replaced storage and the
    // spare, the larger stays as the spare (allocations and frees wait for
    // the whole device)
    Storage ns;
    if (ix.spare.cap >= need) {
        ns = ix.spare;
        ix.spare = Storage{};
    } else {
        ns.alloc(std::max<uint64_t>(std::max(need, want), ix.st.cap + ix.st.cap / 2), false);
    }
    const uint64_t used = cur.nused;
    PI_HIP(hipMemcpyAsync(ns.key.p, ix.st.key.p, used * 8, hipMemcpyDeviceToDevice, s));
    PI_HIP(hipMemcpyAsync(ns.val.p, ix.st.val.p, used * 8, hipMemcpyDeviceToDevice, s));
    PI_HIP(hipMemcpyAsync(ns.next.p, ix.st.next.p, used * 4, hipMemcpyDeviceToDevice, s));
    PI_HIP(hipMemcpyAsync(ns.meta.p, ix.st.meta.p, used, hipMemcpyDeviceToDevice, s));
    PI_HIP(hipStreamSynchronize(s));
    if (ix.spare.cap < ix.st.cap) {
        ix.spare.release();
        ix.spare = ix.st;
    } else {
        ix.st.release();
    }
    ix.st = ns;
    bg_reserve(ix);
}

void bulk_load(Index &ix, const uint64_t *keys, const uint64_t *vals, uint64_t n, hipStream_t s) {
    TraceRange tr("pi:bulk_load");
    bg_quiesce(ix);
    ix.changes_base = 0;
    const uint64_t *sk = nullptr;
    const uint32_t *sidx = nullptr;
    uint64_t nb = 0;
    if (n > 0) {
        sort_keys_with_index(ix.sortws, keys, nullptr, n, nullptr, s, &sk, &sidx);
        DevBuf &flag = ix.tmp[2];
        DevBuf &pos = ix.tmp[3];
        DevBuf &tot = ix.tmp[1];
        flag.ensure(n * 4);
        pos.ensure(n * 4);
        tot.ensure(MAX_LEVELS * 4);
        hipLaunchKernelGGL(k_last_of_run, dim3(blocks_for(n, 256)), dim3(256), 0, s, sk, (uint32_t)n,
                           flag.as<uint32_t>());
        PI_LAUNCH_CHECK();
        exclusive_scan_u32(ix.scanws, flag.as<uint32_t>(), pos.as<uint32_t>(), n, tot.as<uint32_t>(), nullptr, s);
        uint32_t *h = reinterpret_cast<uint32_t *>(ix.hcounts);
        PI_HIP(hipMemcpyAsync(h, tot.p, 4, hipMemcpyDeviceToHost, s));
        PI_HIP(hipStreamSynchronize(s));
        nb = h[0];
        // a nonzero capacity_hint is a fixed capacity; otherwise leave room to grow
        if (ix.cfg.capacity_hint && nb + 2 > ix.cfg.capacity_hint)
            throw Error{PI_ERR_CAPACITY, "bulk load exceeds capacity_hint"};
        const uint64_t want = ix.cfg.capacity_hint ? ix.cfg.capacity_hint : nb + 2 + storage_room(ix, nb);
        if (want > ix.st.cap) {
            Storage ns;
            ns.alloc(want, ix.cfg.capacity_hint != 0);
            ix.st.release();
            ix.st = ns;
        }
        hipLaunchKernelGGL(k_write_base, dim3(blocks_for(n, 256)), dim3(256), 0, s, sk, sidx, vals,
                           flag.as<uint32_t>(), pos.as<uint32_t>(), (uint32_t)n, ix.st.key.as<uint64_t>(),
                           ix.st.val.as<uint64_t>(), ix.st.meta.as<uint8_t>());
        PI_LAUNCH_CHECK();
    }
    ix.nbase = nb;
    hipLaunchKernelGGL(k_reset_region, dim3(1), dim3(64), 0, s, ix.st.key.as<uint64_t>(), ix.st.val.as<uint64_t>(),
                       ix.st.next.as<uint32_t>(), ix.st.meta.as<uint8_t>(), nb, ix.dstate, 0);
    PI_LAUNCH_CHECK();
    ix.used_upper = nb + 2;
    ix.live_at_rebuild = nb;
    build_levels(ix, s);
    bg_reserve(ix);
}

// Writes the live pairs in key order to okey/oval (+ slot_off), and, when
// ometa is given, clears their flags.  Returns the live count.  Synchronises.
// The rebuild's live counts (base flags, overflow flags, overflow nodes
// placed among the base) against the live counter: a disagreement means the
// flags or the counter are wrong, and fails the handle at its next counter
// read (the host does not wait for this).
__global__ void k_check_live(const uint32_t *__restrict__ t, unsigned long long live, uint32_t has_ovf,
                             unsigned int *errors) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const unsigned long long flags = (unsigned long long)t[0] + (has_ovf ? t[1] : 0u);
    if (flags != live || (has_ovf && t[2] != t[1])) atomicOr(errors, ERR_LIVE);
}

static uint64_t merge_live(Index &ix, uint64_t *okey, uint64_t *oval, uint8_t *ometa, uint64_t slot_off,
                           uint64_t cap, hipStream_t s, bool *too_small, const DevState *known = nullptr,
                           bool sync_end = true) {
    DevState cur;
    if (known)
        cur = *known;
    else
        read_state(ix, s, &cur);
    const uint64_t nb = ix.nbase;
    const uint64_t first = nb + 2;
    const uint64_t novf = cur.nused > first ? cur.nused - first : 0;
    *too_small = cur.n_live > cap;
    if (*too_small) return cur.n_live;
    const uint64_t lim = cap > ~0ull - slot_off ? ~0ull : slot_off + cap;  // output entries [slot_off, lim)
    DevBuf &A = ix.tmp[0];    // exclusive prefix of the base live flags (nb+1)
    DevBuf &H = ix.tmp[1];    // live overflow nodes placed at each base position (nb+1)
    DevBuf &B = ix.tmp[2];    // exclusive prefix of H
    DevBuf &C = ix.tmp[3];    // overflow live flags -> exclusive prefix
    DevBuf &P = ix.tmp[4];    // overflow place
    DevBuf &T = ix.tmp[5];    // totals
    A.ensure((nb + 1) * 4);
    H.ensure((nb + 1) * 4);
    B.ensure((nb + 1) * 4);
    C.ensure((novf + 1) * 4);
    P.ensure((novf + 1) * 4);
    T.ensure(16);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(nb + 1, 256)), dim3(256), 0, s, H.as<uint32_t>(), nb + 1, 0u);
    PI_LAUNCH_CHECK();
    exclusive_scan_live(ix.scanws, ix.st.meta.as<uint8_t>() + 1, nb, A.as<uint32_t>(), T.as<uint32_t>(), s);
    const uint64_t *osk = nullptr;
    const uint32_t *opos_in = nullptr;
    DevBuf &olive = ix.tmp[7];
    if (novf > 0) {
        olive.ensure(novf * 4);
        // the overflow region holds distinct keys: the batch ordering (range
        // groups + in-group fix-up) sorts them fully; the payload is the
        // position in the region, so the slot is first + payload
        sort_batch_by_range(ix.sortws, ix.msdws, ix.st.key.as<uint64_t>() + first, nullptr, novf, false, s, &osk,
                            &opos_in);
        hipLaunchKernelGGL(k_ovf_place, dim3(blocks_for(novf, 256)), dim3(256), 0, s, osk, opos_in, (uint32_t)first,
                           novf, ix.st.key.as<uint64_t>(), ix.st.meta.as<uint8_t>(), nb, olive.as<uint32_t>(),
                           P.as<uint32_t>(), H.as<uint32_t>());
        PI_LAUNCH_CHECK();
        exclusive_scan_u32(ix.scanws, olive.as<uint32_t>(), C.as<uint32_t>(), novf, T.as<uint32_t>() + 1, nullptr, s);
    }
    exclusive_scan_u32(ix.scanws, H.as<uint32_t>(), B.as<uint32_t>(), nb + 1, T.as<uint32_t>() + 2, nullptr, s);
    hipLaunchKernelGGL(k_check_live, dim3(1), dim3(64), 0, s, (const uint32_t *)T.as<uint32_t>(),
                       (unsigned long long)cur.n_live, (uint32_t)(novf > 0), &ix.dstate->errors);
    if (nb > 0)
        hipLaunchKernelGGL(k_merge_base, dim3(blocks_for(nb, 256)), dim3(256), 0, s, ix.st.key.as<uint64_t>(),
                           ix.st.val.as<uint64_t>(), ix.st.meta.as<uint8_t>(), nb, A.as<uint32_t>(),
                           B.as<uint32_t>(), H.as<uint32_t>(), okey, oval, ometa, slot_off, lim, &ix.dstate->errors);
    if (novf > 0)
        hipLaunchKernelGGL(k_merge_ovf, dim3(blocks_for(novf, 256)), dim3(256), 0, s, osk, opos_in, (uint32_t)first, novf,
                           ix.st.val.as<uint64_t>(), olive.as<uint32_t>(), C.as<uint32_t>(), P.as<uint32_t>(),
                           A.as<uint32_t>(), okey, oval, ometa, slot_off, lim, &ix.dstate->errors);
    PI_LAUNCH_CHECK();
    if (sync_end) PI_HIP(hipStreamSynchronize(s));
    return cur.n_live;
}

uint64_t export_live(Index &ix, uint64_t *okeys, uint64_t *ovals, uint64_t cap, hipStream_t s) {
    bool small = false;
    const uint64_t n = merge_live(ix, okeys, ovals, nullptr, 0, cap, s, &small);
    if (small) throw Error{PI_ERR_CAPACITY, "export capacity too small", };
    return n;
}

void rebuild(Index &ix, hipStream_t s, const DevState *known) {
    TraceRange tr("pi:rebuild");
    bg_quiesce(ix);  // a background index rebuild reads the storage about to be replaced
    Profiler::Rec rec{};
    if (ix.prof.on) {
        rec.n = 2;
        rec.e[0] = ix.prof.take();
        PI_HIP(hipEventRecord(rec.e[0], s));
    }
    DevState cur;
    if (known)
        cur = *known;
    else
        read_state(ix, s, &cur);
    const uint64_t live = cur.n_live;
    // room for the largest batch the index has taken as well: a rebuilt
    // storage that the next such batch does not fit would grow again at once
    const uint64_t need = ix.cfg.capacity_hint ? ix.cfg.capacity_hint
                                               : live + 2 + std::max(storage_room(ix, live), ix.batch_peak);
    // the new base region goes to the spare storage (the one replaced by the
    // previous rebuild) when it is large enough; the current one becomes the
    // spare.  A spare that is too small is replaced by one of twice the need
    // (and at least the current capacity): an index that keeps growing
    // between rebuilds then reallocates a logarithmic number of times, not at
    // every rebuild (each allocation and free waits for the whole device).
    Storage ns = ix.spare;
    ix.spare = Storage{};
    if (ns.cap < need || (ix.cfg.capacity_hint && ns.cap != need)) {
        ns.release();
        ns.alloc(ix.cfg.capacity_hint ? need : std::max<uint64_t>(2 * need, ix.st.cap), ix.cfg.capacity_hint != 0);
    }
    bool small = false;
    try {
        // the counters were read above; the merge is ordered before the
        // level build on the stream, so nothing waits for it here
        merge_live(ix, ns.key.as<uint64_t>(), ns.val.as<uint64_t>(), ns.meta.as<uint8_t>(), 1, ns.cap - 2, s, &small,
                   &cur, false);
    } catch (...) {
        ix.spare = ns;
        throw;
    }
    if (small) {  // a fixed capacity below the live keys (cannot happen while inserts are checked)
        ix.spare = ns;
        throw Error{PI_ERR_CAPACITY, "internal error: the live keys do not fit the storage capacity"};
    }
    ix.spare = ix.st;
    ix.st = ns;
    ix.nbase = live;
    hipLaunchKernelGGL(k_reset_region, dim3(1), dim3(64), 0, s, ix.st.key.as<uint64_t>(), ix.st.val.as<uint64_t>(),
                       ix.st.next.as<uint32_t>(), ix.st.meta.as<uint8_t>(), live, ix.dstate, 0);
    PI_LAUNCH_CHECK();
    ix.used_upper = live + 2;
    ix.live_at_rebuild = live;
    ix.changes_base = 0;
    ix.repairs++;
    build_levels(ix, s);
    bg_reserve(ix);
    if (ix.prof.on) {
        rec.e[1] = ix.prof.take();
        PI_HIP(hipEventRecord(rec.e[1], s));
        ix.prof.pending.push_back(rec);
    }
}

}  // namespace pi
