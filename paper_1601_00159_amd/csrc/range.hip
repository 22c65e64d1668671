// Range search on gfx950: the range query of Section 3.2.5, SEARCH only.
//
// For ranges [lo_i, hi_i] the result is every live pair with lo_i <= key <=
// hi_i, in key order.  Two calls: count (sizes and output offsets) and
// collect (the pairs), so that the caller sizes the output in between.
//
//   order    the ranges are ordered by lower bound, as the paper does before
//            the descent (the batch ordering of msd.hip, full key order)
//   locate   k_range_locate: per range, the descent (Algorithm 2) and the
//            storage walk (getNode of Algorithm 4) to the last node with key
//            < lo.  While the storage holds base nodes only, the same is done
//            for the last node with key <= hi, which turns the range into a
//            slot interval [a, b).  Both descents of a lane run together.
//   count    base nodes only: one wave per range counts the live slots of its
//            interval, 64 at a time with a ballot over the delete flags (the
//            interval length when nothing is flagged).  With linked nodes
//            (inserts since the last rebuild): one lane per range walks the
//            storage list from the first node >= lo until a key passes hi.
//   offsets  exclusive scan of the counts (u64; the total can pass 2^32)
//   collect  the same split; waves compact the live slots with ballot and
//            mbcnt and write them at the range's offset, lanes write as they
//            walk.
//
// The paper splits a range whose key span reaches into the next thread's
// interceptions and hands the rest over, in thread order.  Here a range is
// owned by one wave (or lane) from its first node to its last, and the scan
// of counts gives every range its output position, so no hand-over is needed.
#include "descent.h"

namespace pi {
namespace {

constexpr int RT = 256;          // locate block
constexpr int WT = 256;          // wave-per-range kernels
constexpr int ST_ = 256;         // offsets scan block
constexpr int SI_ = 16;          // items per thread
constexpr int STILE_ = ST_ * SI_;

__device__ __forceinline__ uint64_t clamp_hi(uint64_t h) { return h > KEY_MAX - 1 ? KEY_MAX - 1 : h; }

// ra[i]: first node with key >= lo (slot or list node); rb[i]: in the base
// state the slot after the last key <= hi (a == b: empty), else unused.
template <int DT>
__global__ __launch_bounds__(DT) void k_range_locate(IndexDesc desc, const uint64_t *__restrict__ lkey,
                                                     const uint32_t *__restrict__ ldown,
                                                     const uint64_t *__restrict__ skey,
                                                     const uint64_t *__restrict__ sval,
                                                     const uint32_t *__restrict__ snext,
                                                     const uint8_t *__restrict__ smeta,
                                                     const uint64_t *__restrict__ slo,
                                                     const uint32_t *__restrict__ sperm,
                                                     const uint64_t *__restrict__ hi, uint32_t n, DevState *st,
                                                     uint32_t *__restrict__ ra, uint32_t *__restrict__ rb) {
    extern __shared__ uint64_t s_dyn[];
    uint64_t *s_k = s_dyn;
    uint32_t *s_d = reinterpret_cast<uint32_t *>(s_dyn + desc.lds_entries);
    stage_levels(desc, lkey, ldown, s_k, s_d);
    const bool links = st->has_links != 0;
    const uint32_t ntiles = (n + DT - 1) / DT;
    const uint32_t c = xcd_chunk(blockIdx.x, gridDim.x);
    const uint32_t t0 = (uint32_t)((uint64_t)c * ntiles / gridDim.x);
    const uint32_t t1 = (uint32_t)((uint64_t)(c + 1) * ntiles / gridDim.x);
    for (uint32_t t = t0; t < t1; t++) {
        const uint32_t i = t * DT + threadIdx.x;
        const bool in = i < n;
        const uint64_t lo = in ? slo[i] : 0;
        const uint64_t h = in ? clamp_hi(hi[sperm[i]]) : 0;
        // q[0]: the largest key below lo (lo = 0: none, the head); q[1]: hi
        uint64_t q[2] = {lo == 0 ? 0 : lo - 1, h};
        uint32_t pos[2];
        uint64_t ik[2];
        descend_index<2>(q, desc, lkey, ldown, s_k, s_d, pos, ik);
        if (!in) continue;
        uint32_t first;
        if (lo == 0) {
            first = (smeta[HEAD_SLOT] & META_LINK) ? snext[HEAD_SLOT] : HEAD_SLOT + 1;
        } else {
            const Found f = walk_storage(q[0], pos[0], ik[0], links, false, skey, sval, snext, smeta, &st->errors);
            first = f.next;
        }
        ra[i] = first;
        if (!links) {
            const Found g = walk_storage(q[1], pos[1], ik[1], false, false, skey, sval, snext, smeta, &st->errors);
            const uint32_t end = g.node + 1;
            rb[i] = (lo > h || end < first) ? first : end;
        }
    }
}

// Base state: live slots of [a, b) per range, one wave per range.  With
// `out` set, also writes them (at most cap per range) at the range's offset.
__global__ __launch_bounds__(WT) void k_range_slots(const uint32_t *__restrict__ ra, const uint32_t *__restrict__ rb,
                                                    const uint32_t *__restrict__ sperm, uint32_t n,
                                                    const uint64_t *__restrict__ skey,
                                                    const uint64_t *__restrict__ sval,
                                                    const uint8_t *__restrict__ smeta, const DevState *st,
                                                    uint32_t *__restrict__ counts,
                                                    const uint64_t *__restrict__ offsets,
                                                    uint64_t *__restrict__ okeys, uint64_t *__restrict__ ovals) {
    if (st->has_links) return;
    const bool dead = st->has_dead != 0;
    const uint32_t waves = gridDim.x * (WT / 64);
    const uint32_t lane = (uint32_t)lane_id();
    for (uint32_t r = blockIdx.x * (WT / 64) + (threadIdx.x >> 6); r < n; r += waves) {
        const uint32_t a = ra[r], b = rb[r];
        const uint32_t id = sperm[r];
        if (!okeys) {
            if (!dead) {
                if (lane == 0) counts[id] = b - a;
                continue;
            }
            uint32_t cnt = 0;
            for (uint32_t base = a; base < b; base += 64) {
                const uint32_t slot = base + lane;
                const bool live = slot < b && !(smeta[slot] & META_DEL);
                cnt += (uint32_t)__popcll(ballot64(live));
            }
            if (lane == 0) counts[id] = cnt;
            continue;
        }
        const uint64_t off = offsets[id];
        const uint64_t cap = offsets[id + 1] - off;
        uint64_t done = 0;
        for (uint32_t base = a; base < b; base += 64) {
            const uint32_t slot = base + lane;
            const bool live = slot < b && !(dead && (smeta[slot] & META_DEL));
            const uint64_t m = ballot64(live);
            const uint64_t at = done + mask_rank(m);
            if (live && at < cap) {
                okeys[off + at] = skey[slot];
                ovals[off + at] = sval[slot];
            }
            done += (uint64_t)__popcll(m);
        }
    }
}

// Linked state: one lane per range walks the storage list from its first
// node >= lo until a key passes hi (the tail's +infinity always does).  With
// `out` set, writes the live pairs (at most cap) at the range's offset.
__global__ __launch_bounds__(WT) void k_range_walk(const uint32_t *__restrict__ ra, const uint64_t *__restrict__ slo,
                                                   const uint32_t *__restrict__ sperm,
                                                   const uint64_t *__restrict__ hi, uint32_t n,
                                                   const uint64_t *__restrict__ skey,
                                                   const uint64_t *__restrict__ sval,
                                                   const uint32_t *__restrict__ snext,
                                                   const uint8_t *__restrict__ smeta, DevState *st,
                                                   uint32_t *__restrict__ counts,
                                                   const uint64_t *__restrict__ offsets,
                                                   uint64_t *__restrict__ okeys, uint64_t *__restrict__ ovals) {
    if (!st->has_links) return;
    const uint32_t i = blockIdx.x * WT + threadIdx.x;
    if (i >= n) return;
    const uint32_t id = sperm[i];
    const uint64_t lo = slo[i];
    const uint64_t h = clamp_hi(hi[id]);
    uint64_t off = 0, cap = 0;
    if (okeys) {
        off = offsets[id];
        cap = offsets[id + 1] - off;
    }
    uint32_t cnt = 0;
    if (lo <= h) {
        // a well-formed list reaches the tail within nused steps
        const uint64_t limit = (uint64_t)st->nused + 1;
        uint32_t cur = ra[i];
        for (uint64_t steps = 0;; steps++) {
            if (steps > limit) {
                atomicOr(&st->errors, ERR_WALK);
                break;
            }
            const uint64_t k = skey[cur];
            if (k > h) break;
            const uint8_t m = smeta[cur];
            if (!(m & META_DEL)) {
                if (okeys && cnt < cap) {
                    okeys[off + cnt] = k;
                    ovals[off + cnt] = sval[cur];
                }
                cnt++;
            }
            cur = (m & META_LINK) ? snext[cur] : cur + 1;
        }
    }
    if (!okeys) counts[id] = cnt;
}

// ---------------------------------------------------------- offsets (u64) --

__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t x, uint64_t *s, uint64_t *total) {
    const uint32_t t = threadIdx.x;
    s[t] = x;
    __syncthreads();
    for (uint32_t d = 1; d < ST_; d <<= 1) {
        const uint64_t add = t >= d ? s[t - d] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    const uint64_t incl = s[t];
    if (total) *total = s[ST_ - 1];
    __syncthreads();
    return incl - x;
}

__global__ __launch_bounds__(ST_) void k_off_reduce(const uint32_t *__restrict__ counts, uint64_t n,
                                                    uint64_t *__restrict__ tiles) {
    __shared__ uint64_t s[ST_];
    const uint64_t base = (uint64_t)blockIdx.x * STILE_ + (uint64_t)threadIdx.x * SI_;
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < SI_; j++) sum += base + j < n ? counts[base + j] : 0u;
    uint64_t tot;
    block_excl_scan_u64(sum, s, &tot);
    if (threadIdx.x == 0) tiles[blockIdx.x] = tot;
}

__global__ __launch_bounds__(ST_) void k_off_tiles(uint64_t *__restrict__ tiles, uint32_t ntiles,
                                                   uint64_t *__restrict__ total) {
    __shared__ uint64_t s[ST_];
    uint64_t carry = 0;
    for (uint32_t base = 0; base < ntiles; base += ST_) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t v = i < ntiles ? tiles[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_excl_scan_u64(v, s, &tot);
        if (i < ntiles) tiles[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(ST_) void k_off_down(const uint32_t *__restrict__ counts, uint64_t n,
                                                  const uint64_t *__restrict__ tiles, uint64_t *__restrict__ offsets) {
    __shared__ uint64_t s[ST_];
    const uint64_t base = (uint64_t)blockIdx.x * STILE_ + (uint64_t)threadIdx.x * SI_;
    uint32_t v[SI_];
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < SI_; j++) {
        v[j] = base + j < n ? counts[base + j] : 0u;
        sum += v[j];
    }
    uint64_t run = tiles[blockIdx.x] + block_excl_scan_u64(sum, s, nullptr);
#pragma unroll
    for (int j = 0; j < SI_; j++) {
        if (base + j < n) offsets[base + j] = run;
        run += v[j];
    }
}

__global__ void k_zero_u64(uint64_t *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

uint32_t blocks_of(uint64_t n, uint64_t t) { return (uint32_t)((n + t - 1) / t); }

// order + locate; returns the sorted lower bounds and their range ids
void locate(Index &ix, const uint64_t *lo, const uint64_t *hi, uint64_t n, hipStream_t s, const uint64_t **slo,
            const uint32_t **sperm) {
    TraceRange tr("pi:range_locate");
    sort_batch_by_range(ix.sortws, ix.msdws, lo, nullptr, n, false, s, slo, sperm);
    ix.rng[0].ensure(n * 4);
    ix.rng[1].ensure(n * 4);
    const IndexDesc &d = ix.desc;
    const size_t lds = (size_t)d.lds_entries * 12;
    auto kern = k_range_locate<RT>;
    const uint32_t g = persistent_grid(ix, kern, RT, lds, blocks_of(n, RT));
    hipLaunchKernelGGL(kern, dim3(g), dim3(RT), lds, s, d, ix.arena_key.as<uint64_t>(), ix.arena_down.as<uint32_t>(),
                       ix.st.key.as<uint64_t>(), ix.st.val.as<uint64_t>(), ix.st.next.as<uint32_t>(),
                       ix.st.meta.as<uint8_t>(), *slo, *sperm, hi, (uint32_t)n, ix.dstate, ix.rng[0].as<uint32_t>(),
                       ix.rng[1].as<uint32_t>());
    PI_LAUNCH_CHECK();
    // the workspaces now hold the location of these ranges
    ix.rcache = Index::RangeCache{lo, hi, n, ix.epoch, *slo, *sperm};
}

uint32_t wave_grid(const Index &ix, uint64_t n) {
    const uint64_t want = blocks_of(n, WT / 64);
    const uint64_t cap = (uint64_t)ix.num_cus * 8;
    return (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
}

}  // namespace

void range_count(Index &ix, const uint64_t *lo, const uint64_t *hi, uint64_t n, uint64_t *offsets, hipStream_t s) {
    if (n == 0) {
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, offsets);
        PI_LAUNCH_CHECK();
        return;
    }
    const uint64_t *slo;
    const uint32_t *sperm;
    locate(ix, lo, hi, n, s, &slo, &sperm);
    ix.rng[2].ensure(n * 4);
    uint32_t *counts = ix.rng[2].as<uint32_t>();
    hipLaunchKernelGGL(k_range_slots, dim3(wave_grid(ix, n)), dim3(WT), 0, s, ix.rng[0].as<uint32_t>(),
                       ix.rng[1].as<uint32_t>(), sperm, (uint32_t)n, ix.st.key.as<uint64_t>(),
                       ix.st.val.as<uint64_t>(), ix.st.meta.as<uint8_t>(), (const DevState *)ix.dstate, counts,
                       nullptr, nullptr, nullptr);
    hipLaunchKernelGGL(k_range_walk, dim3(blocks_of(n, WT)), dim3(WT), 0, s, ix.rng[0].as<uint32_t>(), slo, sperm, hi,
                       (uint32_t)n, ix.st.key.as<uint64_t>(), ix.st.val.as<uint64_t>(), ix.st.next.as<uint32_t>(),
                       ix.st.meta.as<uint8_t>(), ix.dstate, counts, nullptr, nullptr, nullptr);
    const uint32_t ntiles = blocks_of(n, STILE_);
    ix.rng[3].ensure((uint64_t)ntiles * 8);
    uint64_t *tiles = ix.rng[3].as<uint64_t>();
    hipLaunchKernelGGL(k_off_reduce, dim3(ntiles), dim3(ST_), 0, s, counts, n, tiles);
    hipLaunchKernelGGL(k_off_tiles, dim3(1), dim3(ST_), 0, s, tiles, ntiles, offsets + n);
    hipLaunchKernelGGL(k_off_down, dim3(ntiles), dim3(ST_), 0, s, counts, n, tiles, offsets);
    PI_LAUNCH_CHECK();
}

void range_collect(Index &ix, const uint64_t *lo, const uint64_t *hi, uint64_t n, const uint64_t *offsets,
                   uint64_t *okeys, uint64_t *ovals, hipStream_t s) {
    if (n == 0) return;
    const uint64_t *slo;
    const uint32_t *sperm;
    const Index::RangeCache &c = ix.rcache;
    if (c.epoch == ix.epoch && c.lo == lo && c.hi == hi && c.n == n) {
        // these ranges were the last located: their order and interceptions stand
        slo = c.slo;
        sperm = c.sperm;
    } else {
        locate(ix, lo, hi, n, s, &slo, &sperm);
    }
    hipLaunchKernelGGL(k_range_slots, dim3(wave_grid(ix, n)), dim3(WT), 0, s, ix.rng[0].as<uint32_t>(),
                       ix.rng[1].as<uint32_t>(), sperm, (uint32_t)n, ix.st.key.as<uint64_t>(),
                       ix.st.val.as<uint64_t>(), ix.st.meta.as<uint8_t>(), (const DevState *)ix.dstate, nullptr,
                       offsets, okeys, ovals);
    hipLaunchKernelGGL(k_range_walk, dim3(blocks_of(n, WT)), dim3(WT), 0, s, ix.rng[0].as<uint32_t>(), slo, sperm, hi,
                       (uint32_t)n, ix.st.key.as<uint64_t>(), ix.st.val.as<uint64_t>(), ix.st.next.as<uint32_t>(),
                       ix.st.meta.as<uint8_t>(), ix.dstate, nullptr, offsets, okeys, ovals);
    PI_LAUNCH_CHECK();
}

}  // namespace pi
