// Slice repair of the index layer (rebuild policy SLICES): the finer-grained
// rebuild the paper leaves as future work (Section 7), next to its whole-layer
// rebuild after a threshold of updates (Section 4.3.5).
//
// Layout.  The base region is cut into slices of SL_B consecutive slots; slice
// j owns the key range [first key of slice j, first key of slice j+1).  On the
// lower index levels 2..ls (where a slice holds enough keys to be worth it)
// every slice owns a fixed segment of cap[l] entries of the level array: its
// keys in order, then a gap up to cap[l].  Gap entries repeat the first entry
// (key and down pointer) of the next non-empty segment, or +infinity after
// the last one, so the level reads as a non-decreasing key array and the
// descent (Algorithm 2) needs no change: a run of keys <= q either stops
// before a gap or passes through it to the real entry it repeats.  Down
// pointers of a sliced level point into the same slice's segment one level
// below (level 2: the storage slot).  The levels above ls are small and
// stay contiguous; they are rebuilt whole from level ls.
//
// Repair.  Nodes inserted since the last repair round are ordered by key, and
// each slice that received any is rewritten in place from its current
// level-2 entries merged with its new keys of height >= 2 (the levels above
// follow by the height rule).  Slices without new nodes are not touched, so
// inserts that cluster in a few key ranges repair a few segments instead of
// the whole index layer.  Deleted nodes stay indexed: they are still linked
// into the storage list (Algorithm 4 flags them), so any of them is a valid
// place to start a storage walk.  A segment that would overflow its capacity
// makes the round fall back to a full rebuild, which also merges the storage.
#include <algorithm>
#include <vector>

#include "descent.h"

namespace pi {
namespace {

constexpr int SLT = 256;                  // threads of a slice block
constexpr int SLW = SLT / 64;
constexpr uint32_t SL_M = 4096;           // largest level-2 segment (entries one block holds)
constexpr int SLI = SL_M / SLT;           // entries per thread

uint32_t grid_of(uint64_t n, int t) { return (uint32_t)std::max<uint64_t>(1, (n + t - 1) / t); }

// exclusive scan of one u32 per thread over a slice block; *total = sum
__device__ __forceinline__ uint32_t sl_scan(uint32_t x, uint32_t *s_w, uint32_t *total) {
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan_u32(x);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SLW; i++) {
        if (i < w) pre += s_w[i];
        tot += s_w[i];
    }
    __syncthreads();
    *total = tot;
    return pre + inc - x;
}

// Writes segment j of levels 2..ls from the slice's level-2 candidates
// K[0..m) (key order) with storage slots SLOT[] and heights H[] (in LDS):
// level 2 takes the entries of height >= 2, level l those of height >= l
// with down pointers into segment j of level l-1.  R[] is scratch.  Returns
// false (writing nothing) when a level would overflow its segment.
__device__ bool write_slice(uint32_t j, uint32_t m, const uint64_t *K, const uint32_t *SLOT, const uint8_t *H,
                            uint32_t *R, const IndexDesc &d, const SliceLayout &sl, uint64_t *__restrict__ lkey,
                            uint32_t *__restrict__ ldown, uint32_t *__restrict__ cnt, uint32_t *s_w) {
    const uint32_t S = sl.S;
    // counts first: nothing is written unless every level fits
    __shared__ uint32_t s_ok;
    if (threadIdx.x == 0) s_ok = 1;
    __syncthreads();
    for (int l = 2; l <= sl.ls; l++) {
        uint32_t c = 0;
        for (uint32_t i = threadIdx.x; i < m; i += SLT) c += H[i] >= (uint32_t)l;
        uint32_t tot;
        sl_scan(c, s_w, &tot);
        if (threadIdx.x == 0 && tot > sl.cap[l]) s_ok = 0;
    }
    __syncthreads();
    if (!s_ok) return false;
    for (int l = 2; l <= sl.ls; l++) {
        // blocked: thread t holds entries t*SLI .. t*SLI+SLI-1 (order-preserving ranks)
        const uint32_t i0 = threadIdx.x * SLI;
        uint32_t c = 0;
#pragma unroll
        for (int e = 0; e < SLI; e++) c += (i0 + e < m && H[i0 + e] >= (uint32_t)l) ? 1u : 0u;
        uint32_t tot;
        uint32_t r = sl_scan(c, s_w, &tot);
        const uint64_t seg = d.off[l] + 1 + (uint64_t)j * sl.cap[l];
        const uint64_t below = l > 2 ? 1 + (uint64_t)j * sl.cap[l - 1] : 0;
#pragma unroll
        for (int e = 0; e < SLI; e++) {
            const uint32_t i = i0 + e;
            if (i < m && H[i] >= (uint32_t)l) {
                lkey[seg + r] = K[i];
                ldown[seg + r] = l == 2 ? SLOT[i] : (uint32_t)(below + R[i]);
                R[i] = r;  // this entry's position in the segment, for the level above
                r++;
            }
        }
        if (threadIdx.x == 0) cnt[(size_t)l * S + j] = tot;
        __syncthreads();
    }
    return true;
}

// Full build, step 1: per slice, the number of base keys reaching each level;
// the largest count of each sliced level; the slice boundary keys; the
// number of keys on every level (totals).
__global__ __launch_bounds__(SLT) void k_slice_count(const uint64_t *__restrict__ bkeys, uint64_t nb,
                                                     SliceLayout sl, uint64_t seed, uint32_t l2p, uint32_t maxh,
                                                     uint32_t *__restrict__ cnt, uint64_t *__restrict__ first,
                                                     unsigned int *__restrict__ maxc,
                                                     unsigned long long *__restrict__ totals) {
    __shared__ uint32_t h[MAX_LEVELS + 1];
    const uint32_t j = blockIdx.x;
    if (threadIdx.x <= MAX_LEVELS) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)j * SL_B, b1 = std::min<uint64_t>(b0 + SL_B, nb);
    for (uint64_t b = b0 + threadIdx.x; b < b1; b += SLT)
        atomicAdd(&h[tower_height(bkeys[b], seed, l2p, maxh)], 1u);
    __syncthreads();
    if (threadIdx.x < MAX_LEVELS && threadIdx.x >= 2) {
        const int l = threadIdx.x;
        uint32_t c = 0;
        for (int x = l; x <= MAX_LEVELS; x++) c += h[x];
        if (l <= sl.ls) {
            cnt[(size_t)l * sl.S + j] = c;
            atomicMax(&maxc[l], c);
        }
        if (c) atomicAdd(&totals[l], (unsigned long long)c);
    }
    if (threadIdx.x == 0) first[j] = (j == 0 || b0 >= nb) ? 0 : bkeys[b0];
}

// Full build, step 2: segment j of levels 2..ls from base slots of slice j.
__global__ __launch_bounds__(SLT) void k_slice_build(const uint64_t *__restrict__ bkeys, uint64_t nb,
                                                     SliceLayout sl, IndexDesc d, uint64_t seed, uint32_t l2p,
                                                     uint32_t maxh, uint64_t *__restrict__ lkey,
                                                     uint32_t *__restrict__ ldown, uint32_t *__restrict__ cnt,
                                                     unsigned int *__restrict__ flag) {
    __shared__ uint64_t K[SL_M];
    __shared__ uint32_t SLOT[SL_M];
    __shared__ uint32_t R[SL_M];
    __shared__ uint8_t H[SL_M];
    __shared__ uint32_t s_w[SLW];
    const uint32_t j = blockIdx.x;
    const uint64_t b0 = (uint64_t)j * SL_B;
    const uint32_t m = (uint32_t)(b0 < nb ? std::min<uint64_t>(SL_B, nb - b0) : 0);
    for (uint32_t i = threadIdx.x; i < m; i += SLT) {
        const uint64_t k = bkeys[b0 + i];
        K[i] = k;
        SLOT[i] = (uint32_t)(1 + b0 + i);
        H[i] = (uint8_t)tower_height(k, seed, l2p, maxh);
    }
    __syncthreads();
    if (!write_slice(j, m, K, SLOT, H, R, d, sl, lkey, ldown, cnt, s_w) && threadIdx.x == 0) atomicOr(flag, 1u);
}

// Repair round: slice j merges its current level-2 entries with its new keys
// of height >= 2 (nk[lo..hi), ordered, slots nslot) and rewrites its segments.
// Slices without new keys of height >= 2 return at once.
__global__ __launch_bounds__(SLT) void k_slice_repair(const uint64_t *__restrict__ nk, const uint32_t *__restrict__ nrel,
                                                      uint64_t nnew, uint64_t nfirst, const uint64_t *__restrict__ first,
                                                      SliceLayout sl, IndexDesc d, uint64_t seed, uint32_t l2p,
                                                      uint32_t maxh, uint64_t *__restrict__ lkey,
                                                      uint32_t *__restrict__ ldown, uint32_t *__restrict__ cnt,
                                                      uint32_t *__restrict__ dirty, unsigned int *__restrict__ flag,
                                                      unsigned int *__restrict__ nrepaired) {
    __shared__ uint64_t K[SL_M];
    __shared__ uint32_t SLOT[SL_M];
    __shared__ uint32_t R[SL_M];
    __shared__ uint8_t H[SL_M];
    __shared__ uint32_t NR[2 * SL_M + 1];  // new keys of height >= 2 before each new key of the slice
    __shared__ uint32_t s_w[SLW];
    __shared__ uint32_t s_range[2];
    const uint32_t j = blockIdx.x;
    const uint32_t S = sl.S;
    // the slice's new keys: [lo, hi) of the ordered new keys (+infinity last)
    if (threadIdx.x < 2) {
        const uint32_t b = j + threadIdx.x;
        uint64_t lo = 0, hi = nnew;
        if (b == 0) {
            hi = 0;
        } else if (b >= S) {
            // end of the valid keys: the first +infinity
            const uint64_t kmax = KEY_MAX;
            while (lo < hi) {
                const uint64_t mid = (lo + hi) >> 1;
                if (nk[mid] < kmax) lo = mid + 1; else hi = mid;
            }
        } else {
            const uint64_t fk = first[b];
            while (lo < hi) {
                const uint64_t mid = (lo + hi) >> 1;
                if (nk[mid] < fk) lo = mid + 1; else hi = mid;
            }
        }
        s_range[threadIdx.x] = (uint32_t)lo;
    }
    __syncthreads();
    const uint32_t lo = s_range[0], hi = s_range[1];
    const uint32_t nn = hi - lo;
    if (nn == 0) return;  // clean slice (uniform over the block)
    if (nn > 2 * SL_M) {  // more new keys than a segment could take: full rebuild
        if (threadIdx.x == 0) atomicOr(flag, 1u);
        return;
    }
    // NR[x]: new keys of height >= 2 among the slice's first x new keys
    uint32_t nb2 = 0;
    for (uint32_t x0 = 0; x0 < nn; x0 += SLT) {
        const uint32_t x = x0 + threadIdx.x;
        const bool in = x < nn && tower_height(nk[lo + x], seed, l2p, maxh) >= 2;
        uint32_t tot;
        const uint32_t r = nb2 + sl_scan(in ? 1u : 0u, s_w, &tot);
        if (x < nn) NR[x] = r;
        nb2 += tot;
    }
    if (threadIdx.x == 0) NR[nn] = nb2;
    __syncthreads();
    if (nb2 == 0) return;  // nothing reaches level 2
    const uint64_t seg2 = d.off[2] + 1 + (uint64_t)j * sl.cap[2];
    const uint32_t na = cnt[(size_t)2 * S + j];
    if (na + nb2 > SL_M || na + nb2 > sl.cap[2]) {
        if (threadIdx.x == 0) atomicOr(flag, 1u);
        return;
    }
    // merged order: an old entry lands at its index plus the new keys of
    // height >= 2 below it, a new key at its rank among those plus the old
    // entries below it (the two sets share no key: a node is created only for
    // an absent key)
    for (uint32_t i = threadIdx.x; i < na; i += SLT) {
        const uint64_t k = lkey[seg2 + i];
        uint32_t a = 0, b = nn;  // new keys below k
        while (a < b) {
            const uint32_t mid = (a + b) >> 1;
            if (nk[lo + mid] < k) a = mid + 1; else b = mid;
        }
        const uint32_t p = i + NR[a];
        K[p] = k;
        SLOT[p] = ldown[seg2 + i];
        H[p] = (uint8_t)tower_height(k, seed, l2p, maxh);
    }
    for (uint32_t x = threadIdx.x; x < nn; x += SLT) {
        const uint64_t k = nk[lo + x];
        if (tower_height(k, seed, l2p, maxh) < 2) continue;
        uint32_t a = 0, b = na;  // old entries below k
        while (a < b) {
            const uint32_t mid = (a + b) >> 1;
            if (lkey[seg2 + mid] < k) a = mid + 1; else b = mid;
        }
        const uint32_t p = NR[x] + a;
        K[p] = k;
        SLOT[p] = (uint32_t)(nfirst + nrel[lo + x]);
        H[p] = (uint8_t)tower_height(k, seed, l2p, maxh);
    }
    __syncthreads();  // every read of the old segment is done before it is rewritten
    if (!write_slice(j, na + nb2, K, SLOT, H, R, d, sl, lkey, ldown, cnt, s_w)) {
        if (threadIdx.x == 0) atomicOr(flag, 1u);
        return;
    }
    if (threadIdx.x == 0) {
        dirty[j] = 1;
        atomicAdd(nrepaired, 1u);
    }
}

// Gaps of segment j of level l (one wave per segment): the first entry of the
// next non-empty segment, or +infinity.  With all = 0 only segments whose own
// content or whose next non-empty segment changed (dirty) are refilled.
__global__ __launch_bounds__(256) void k_slice_gapfill(SliceLayout sl, IndexDesc d, uint64_t *__restrict__ lkey,
                                                       uint32_t *__restrict__ ldown, const uint32_t *__restrict__ cnt,
                                                       const uint32_t *__restrict__ dirty, int all) {
    const uint32_t S = sl.S;
    const uint32_t wave = (blockIdx.x * 256 + threadIdx.x) >> 6;
    const uint32_t nl = (uint32_t)(sl.ls - 1);
    if (wave >= S * nl) return;
    const int l = 2 + (int)(wave / S);
    const uint32_t j = wave % S;
    const uint32_t cap = sl.cap[l];
    const uint32_t *row = cnt + (size_t)l * S;
    uint32_t k = j + 1;
    while (k < S && row[k] == 0) k++;
    if (!all && !dirty[j] && !(k < S && dirty[k])) return;
    const uint32_t c = row[j];
    uint64_t gk = KEY_MAX;
    uint32_t gd = 0;
    if (k < S) {
        const uint64_t e = d.off[l] + 1 + (uint64_t)k * cap;
        gk = lkey[e];
        gd = ldown[e];
    }
    const uint64_t seg = d.off[l] + 1 + (uint64_t)j * cap;
    for (uint32_t x = c + (uint32_t)lane_id(); x < cap; x += 64) {
        lkey[seg + x] = gk;
        ldown[seg + x] = gd;
    }
}

// The real entries of level ls, in order, with their positions on the level
// (the input of the levels above): one wave per segment, out offsets from the
// exclusive scan of the segment counts.
__global__ __launch_bounds__(256) void k_slice_collect(SliceLayout sl, IndexDesc d, const uint64_t *__restrict__ lkey,
                                                       const uint32_t *__restrict__ cnt,
                                                       const uint32_t *__restrict__ offs, uint64_t *__restrict__ ukey,
                                                       uint32_t *__restrict__ upos) {
    const uint32_t S = sl.S;
    const uint32_t j = (blockIdx.x * 256 + threadIdx.x) >> 6;
    if (j >= S) return;
    const int l = sl.ls;
    const uint32_t cap = sl.cap[l];
    const uint32_t c = cnt[(size_t)l * S + j];
    const uint64_t seg = d.off[l] + 1 + (uint64_t)j * cap;
    const uint32_t o = offs[j];
    for (uint32_t x = (uint32_t)lane_id(); x < c; x += 64) {
        ukey[o + x] = lkey[seg + x];
        upos[o + x] = (uint32_t)(1 + (uint64_t)j * cap + x);
    }
}

// Level l of a sliced layout as a contiguous key array with down pointers
// given as 1-based positions of the level below without gaps (inspection).
__global__ __launch_bounds__(256) void k_slice_export(SliceLayout sl, IndexDesc d, int l,
                                                      const uint64_t *__restrict__ lkey,
                                                      const uint32_t *__restrict__ ldown,
                                                      const uint32_t *__restrict__ cnt,
                                                      const uint32_t *__restrict__ offs,
                                                      const uint32_t *__restrict__ offs_below,
                                                      uint64_t *__restrict__ okey, uint32_t *__restrict__ odown) {
    const uint32_t S = sl.S;
    const uint32_t j = (blockIdx.x * 256 + threadIdx.x) >> 6;
    if (j >= S) return;
    const uint32_t cap = sl.cap[l];
    const uint32_t c = cnt[(size_t)l * S + j];
    const uint64_t seg = d.off[l] + 1 + (uint64_t)j * cap;
    const uint32_t o = offs[j];
    const uint32_t capb = l > 2 ? sl.cap[l - 1] : 1;
    for (uint32_t x = (uint32_t)lane_id(); x < c; x += 64) {
        okey[o + x] = lkey[seg + x];
        uint32_t dn = ldown[seg + x];
        if (l > 2) {
            const uint32_t jb = (dn - 1) / capb;
            dn = 1 + offs_below[jb] + (dn - 1 - jb * capb);
        }
        odown[o + x] = dn;
    }
}

// down pointers of the first level above the slices, translated like the
// export above (inspection)
__global__ void k_slice_translate(SliceLayout sl, const uint32_t *__restrict__ offs_below, uint32_t *__restrict__ down,
                                  uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t capb = sl.cap[sl.ls];
    const uint32_t dn = down[i];
    const uint32_t jb = (dn - 1) / capb;
    down[i] = 1 + offs_below[jb] + (dn - 1 - jb * capb);
}

__global__ void k_bg_like_gather(const uint64_t *__restrict__ skey, const uint8_t *__restrict__ smeta, uint64_t first,
                                 uint64_t n, uint64_t *__restrict__ okeys) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    okeys[i] = (smeta[first + i] & META_DEL) ? KEY_MAX : skey[first + i];
}

__global__ void k_zero_words(unsigned int *p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

// Lowest level that is not sliced minus one: levels 2..ls are sliced while a
// slice holds at least 32 keys on them on average.
static int sliced_top(const Index &ix) {
    const int per = (int)SL_LOG - 5;  // log2(SL_B / 32)
    const int ls = 1 + per / (int)ix.cfg.log2_inv_p;
    return std::max(2, std::min<int>(ls, (int)ix.cfg.max_height));
}

static void slice_reserve(Index &ix, uint32_t S) {
    Index::Slices &z = ix.slc;
    z.cnt.ensure((size_t)MAX_LEVELS * S * sizeof(uint32_t));
    z.first.ensure((size_t)S * sizeof(uint64_t));
    z.dirty.ensure((size_t)S * sizeof(uint32_t));
    z.offs.ensure((size_t)(S + 1) * sizeof(uint32_t));
    z.offs2.ensure((size_t)(S + 1) * sizeof(uint32_t));
    z.misc.ensure(4096);
}

// Layout of the upper levels (ls+1 .. top, contiguous, after the sliced ones)
// for the given sizes; the arena must already hold them.
static void upper_layout(Index &ix, IndexDesc &d, const uint32_t *upper_n) {
    const SliceLayout &sl = ix.slc.lay;
    uint64_t total = d.off[sl.ls] + (((uint64_t)d.n[sl.ls] + 1 + LEVEL_PAD + 15) & ~15ull);
    d.top = sl.ls;
    for (int l = sl.ls + 1; l < MAX_LEVELS && l <= (int)ix.cfg.max_height; l++) {
        d.n[l] = upper_n[l];
        if (upper_n[l] > 0) d.top = l;
    }
    for (int l = sl.ls + 1; l <= d.top; l++) {
        d.off[l] = total;
        total += ((uint64_t)d.n[l] + 1 + LEVEL_PAD + 15) & ~15ull;
    }
    ix.slc.arena_used = total;
}

// Levels above ls from the real entries of level ls.  Synchronises (sizes).
static void build_upper(Index &ix, hipStream_t s) {
    Index::Slices &z = ix.slc;
    const SliceLayout &sl = z.lay;
    IndexDesc &d = ix.desc;
    uint32_t *cnt = z.cnt.as<uint32_t>();
    uint32_t *misc = z.misc.as<uint32_t>();
    // offsets of every segment's entries of level ls
    exclusive_scan_u32(ix.scanws, cnt + (size_t)sl.ls * sl.S, z.offs.as<uint32_t>(), sl.S, misc + 256, nullptr, s);
    uint32_t *h = reinterpret_cast<uint32_t *>(ix.hcounts);
    PI_HIP(hipMemcpyAsync(h, misc + 256, 4, hipMemcpyDeviceToHost, s));
    PI_HIP(hipStreamSynchronize(s));
    const uint64_t nu = h[0];
    z.ukey.ensure(std::max<uint64_t>(nu, 1) * 8);
    z.upos.ensure(std::max<uint64_t>(nu, 1) * 4);
    hipLaunchKernelGGL(k_slice_collect, dim3(grid_of((uint64_t)sl.S * 64, 256)), dim3(256), 0, s, sl, d,
                       ix.arena_key.as<uint64_t>(), cnt, z.offs.as<uint32_t>(), z.ukey.as<uint64_t>(),
                       z.upos.as<uint32_t>());
    PI_LAUNCH_CHECK();
    uint32_t upper_n[MAX_LEVELS] = {};
    if (nu > 0) {
        level_totals(ix, z.ukey.as<uint64_t>(), nu, z.tcnt, z.ttot, upper_n, s);
        for (int l = 0; l <= sl.ls; l++) upper_n[l] = 0;
    }
    upper_layout(ix, d, upper_n);
    if (ix.arena_key.bytes < z.arena_used * 8 || ix.arena_down.bytes < z.arena_used * 4)
        throw Error{PI_ERR_STATE, "slice layout: upper levels outgrew the arena"};
    if (nu > 0 && d.top > sl.ls)
        scatter_levels(ix, z.ukey.as<uint64_t>(), z.upos.as<uint32_t>(), nu, d, z.tcnt, z.ttot, ix.arena_key,
                       ix.arena_down, s, sl.ls + 1);
    pad_levels(ix, d, s);
    select_lds_levels(ix, d);
    // real key counts of the sliced levels, for the statistics
    uint32_t *tot = misc + 400;
    for (int l = 2; l <= sl.ls; l++)
        exclusive_scan_u32(ix.scanws, cnt + (size_t)l * sl.S, z.offs2.as<uint32_t>(), sl.S, tot + l, nullptr, s);
    PI_HIP(hipMemcpyAsync(h, tot, MAX_LEVELS * 4, hipMemcpyDeviceToHost, s));
    PI_HIP(hipStreamSynchronize(s));
    for (int l = 0; l < MAX_LEVELS; l++) z.real_n[l] = l >= 2 && l <= sl.ls ? h[l] : (l <= d.top ? d.n[l] : 0);
}

// Full build of the sliced layout from base slots 1..nbase.  Synchronises.
void slice_build(Index &ix, hipStream_t s) {
    Index::Slices &z = ix.slc;
    const uint64_t nb = ix.nbase;
    SliceLayout sl{};
    sl.S = (uint32_t)std::max<uint64_t>(1, (nb + SL_B - 1) / SL_B);
    sl.ls = sliced_top(ix);
    slice_reserve(ix, sl.S);
    uint32_t *misc = z.misc.as<uint32_t>();
    unsigned int *maxc = misc;                                          // [MAX_LEVELS]
    unsigned long long *totals = reinterpret_cast<unsigned long long *>(misc + 64);  // [MAX_LEVELS]
    PI_HIP(hipMemsetAsync(z.misc.p, 0, 4096, s));
    const uint64_t *bkeys = ix.st.key.as<uint64_t>() + 1;
    hipLaunchKernelGGL(k_slice_count, dim3(sl.S), dim3(SLT), 0, s, bkeys, nb, sl, ix.cfg.height_seed,
                       ix.cfg.log2_inv_p, ix.cfg.max_height, z.cnt.as<uint32_t>(), z.first.as<uint64_t>(), maxc,
                       totals);
    PI_LAUNCH_CHECK();
    uint64_t *h = ix.hcounts;
    PI_HIP(hipMemcpyAsync(h, z.misc.p, 64 * 4 + MAX_LEVELS * 8, hipMemcpyDeviceToHost, s));
    PI_HIP(hipStreamSynchronize(s));
    const uint32_t *hmax = reinterpret_cast<const uint32_t *>(h);
    const uint64_t *htot = h + 32;
    // segment capacities: the fullest slice plus half as much again, for the
    // keys later repairs add (at most one block's worth on level 2)
    uint64_t total = 0;
    IndexDesc d{};
    d.top = 1;
    for (int l = 2; l <= sl.ls; l++) {
        uint32_t c = (uint32_t)((hmax[l] * 3ull / 2 + 16 + 15) & ~15ull);
        if (l == 2) c = std::min<uint32_t>(c, SL_M);
        sl.cap[l] = std::max<uint32_t>(c, 16);
        d.n[l] = (uint32_t)((uint64_t)sl.S * sl.cap[l]);
        d.off[l] = total;
        total += ((uint64_t)d.n[l] + 1 + LEVEL_PAD + 15) & ~15ull;
        d.top = l;
    }
    z.lay = sl;
    z.on = true;
    // arena: the sliced levels, and room for the levels above at twice their
    // present size (they grow as repairs index new keys)
    uint64_t upper = 0;
    for (int l = sl.ls + 1; l < MAX_LEVELS && l <= (int)ix.cfg.max_height; l++)
        upper += ((2 * htot[l] + 1 + LEVEL_PAD + 15) & ~15ull) + 64;
    const uint64_t want = total + upper + 1024;
    if (ix.arena_key.bytes < want * 8) ix.arena_key.ensure(want * 8);
    if (ix.arena_down.bytes < want * 4) ix.arena_down.ensure(want * 4);
    ix.desc = d;
    unsigned int *flag = misc + 200;
    hipLaunchKernelGGL(k_slice_build, dim3(sl.S), dim3(SLT), 0, s, bkeys, nb, sl, d, ix.cfg.height_seed,
                       ix.cfg.log2_inv_p, ix.cfg.max_height, ix.arena_key.as<uint64_t>(), ix.arena_down.as<uint32_t>(),
                       z.cnt.as<uint32_t>(), flag);
    PI_LAUNCH_CHECK();
    const uint32_t nl = (uint32_t)(sl.ls - 1);
    hipLaunchKernelGGL(k_slice_gapfill, dim3(grid_of((uint64_t)sl.S * nl * 64, 256)), dim3(256), 0, s, sl, d,
                       ix.arena_key.as<uint64_t>(), ix.arena_down.as<uint32_t>(), z.cnt.as<uint32_t>(),
                       z.dirty.as<uint32_t>(), 1);
    PI_LAUNCH_CHECK();
    build_upper(ix, s);
    z.round_first = nb + 2;
    for (int l = 0; l < MAX_LEVELS; l++) ix.base_level_n[l] = 0;
}

// Repair round over the nodes created in storage slots [z.round_first, snap):
// slices that received any are rewritten; the levels above ls are rebuilt.
// Returns false when a segment would overflow (nothing of that slice was
// written; the caller rebuilds everything).  Synchronises.
bool slice_round(Index &ix, uint64_t snap, hipStream_t s) {
    Index::Slices &z = ix.slc;
    const SliceLayout &sl = z.lay;
    const uint64_t first = z.round_first;
    if (snap <= first) return true;
    const uint64_t m = snap - first;
    z.okeys.ensure(m * 8);
    hipLaunchKernelGGL(k_bg_like_gather, dim3(grid_of(m, 256)), dim3(256), 0, s, ix.st.key.as<uint64_t>(),
                       ix.st.meta.as<uint8_t>(), first, m, z.okeys.as<uint64_t>());
    PI_LAUNCH_CHECK();
    const uint64_t *sk = nullptr;
    const uint32_t *si = nullptr;
    sort_batch_by_range(z.sortws, z.msdws, z.okeys.as<uint64_t>(), nullptr, m, false, s, &sk, &si);
    uint32_t *misc = z.misc.as<uint32_t>();
    unsigned int *flag = misc + 200;
    unsigned int *nrep = misc + 201;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, misc + 200, 2u);
    hipLaunchKernelGGL(k_zero_words, dim3(grid_of(sl.S, 256)), dim3(256), 0, s, z.dirty.as<uint32_t>(), sl.S);
    hipLaunchKernelGGL(k_slice_repair, dim3(sl.S), dim3(SLT), 0, s, sk, si, m, first, z.first.as<uint64_t>(), sl,
                       ix.desc, ix.cfg.height_seed, ix.cfg.log2_inv_p, ix.cfg.max_height, ix.arena_key.as<uint64_t>(),
                       ix.arena_down.as<uint32_t>(), z.cnt.as<uint32_t>(), z.dirty.as<uint32_t>(), flag, nrep);
    PI_LAUNCH_CHECK();
    const uint32_t nl = (uint32_t)(sl.ls - 1);
    hipLaunchKernelGGL(k_slice_gapfill, dim3(grid_of((uint64_t)sl.S * nl * 64, 256)), dim3(256), 0, s, sl, ix.desc,
                       ix.arena_key.as<uint64_t>(), ix.arena_down.as<uint32_t>(), z.cnt.as<uint32_t>(),
                       z.dirty.as<uint32_t>(), 0);
    PI_LAUNCH_CHECK();
    uint32_t *h = reinterpret_cast<uint32_t *>(ix.hcounts);
    PI_HIP(hipMemcpyAsync(h, flag, 8, hipMemcpyDeviceToHost, s));
    PI_HIP(hipStreamSynchronize(s));
    const bool ok = h[0] == 0;
    z.repaired += h[1];
    z.rounds++;
    build_upper(ix, s);
    z.round_first = snap;
    return ok;
}

// Level l of the sliced layout without gaps (inspection); returns the count.
uint64_t slice_export_level(Index &ix, int l, uint64_t *okey, uint32_t *odown, uint64_t cap, hipStream_t s) {
    Index::Slices &z = ix.slc;
    const SliceLayout &sl = z.lay;
    const uint64_t n = z.real_n[l];
    if (n > cap) return n;
    uint32_t *cnt = z.cnt.as<uint32_t>();
    uint32_t *misc = z.misc.as<uint32_t>();
    if (l <= sl.ls) {
        exclusive_scan_u32(ix.scanws, cnt + (size_t)l * sl.S, z.offs.as<uint32_t>(), sl.S, misc + 300, nullptr, s);
        if (l > 2)
            exclusive_scan_u32(ix.scanws, cnt + (size_t)(l - 1) * sl.S, z.offs2.as<uint32_t>(), sl.S, misc + 301,
                               nullptr, s);
        hipLaunchKernelGGL(k_slice_export, dim3(grid_of((uint64_t)sl.S * 64, 256)), dim3(256), 0, s, sl, ix.desc, l,
                           ix.arena_key.as<uint64_t>(), ix.arena_down.as<uint32_t>(), cnt, z.offs.as<uint32_t>(),
                           z.offs2.as<uint32_t>(), okey, odown);
        PI_LAUNCH_CHECK();
    } else if (n > 0) {
        const uint64_t o = ix.desc.off[l] + 1;
        PI_HIP(hipMemcpyAsync(okey, ix.arena_key.as<uint64_t>() + o, n * 8, hipMemcpyDeviceToDevice, s));
        PI_HIP(hipMemcpyAsync(odown, ix.arena_down.as<uint32_t>() + o, n * 4, hipMemcpyDeviceToDevice, s));
        if (l == sl.ls + 1) {
            exclusive_scan_u32(ix.scanws, cnt + (size_t)sl.ls * sl.S, z.offs2.as<uint32_t>(), sl.S, misc + 301,
                               nullptr, s);
            hipLaunchKernelGGL(k_slice_translate, dim3(grid_of(n, 256)), dim3(256), 0, s, sl, z.offs2.as<uint32_t>(),
                               odown, n);
            PI_LAUNCH_CHECK();
        }
    }
    PI_HIP(hipStreamSynchronize(s));
    return n;
}

void slice_release(Index &ix) {
    Index::Slices &z = ix.slc;
    for (DevBuf *b : {&z.cnt, &z.first, &z.dirty, &z.offs, &z.offs2, &z.misc, &z.ukey, &z.upos, &z.okeys, &z.tcnt,
                      &z.ttot})
        b->release();
    z.sortws.release();
    z.msdws.release();
    z.on = false;
}

}  // namespace pi
