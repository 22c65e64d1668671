// Ordering of a query batch by key (Definition 3) for gfx950.
//
// The paper keeps each worker's query batch sorted and partitions the sorted
// set by key range (Algorithm 1, Section 4.3.2).  Here the order is produced
// range-first:
//   1. [min, max] of the batch's keys (per-block partials, no atomics); every
//      key gets a 16-, 24- or 32-bit position u inside that span (range_pos)
//   2. one stable 8-bit radix pass per byte of u: the batch is grouped by u,
//      equal u in input order (coalesced writes: 256 destinations per pass)
//   3. k_fixup, in place: windows of ~1920 entries widened to whole groups;
//      a group of equal u holds keys that may differ and must be ordered by
//      (key, input position) -- insertion sort in LDS for the usual tiny
//      groups, a bitonic network for a window with a larger group.  Skipped
//      for batches without updates (the grouping by u is their order).
//   4. windows too large for one block (a group of one hot key repeated many
//      times): k_big_check (all blocks) tests whether the window holds a
//      single key -- then it is already in input order and nothing moves;
//      otherwise k_big_fixup orders it: split around the dominant key, or a
//      stable block-level LSD over the varying digits.
#include <algorithm>

#include "pi_internal.h"

namespace pi {
namespace {

constexpr int MT = 256;
constexpr int MNW = MT / 64;
constexpr uint32_t MM_BLOCKS = 1024;  // min/max partials

constexpr int WT = 256;               // window block
constexpr int WE = 8;                 // entries per thread
constexpr uint32_t WMAX = WT * WE;    // largest window sorted in one block
constexpr uint32_t WNOM = 1920;       // nominal window (room for the last group)
constexpr int WNW = WT / 64;
constexpr int BIG_GRID = 128;

// ---- 1. key span --------------------------------------------------------

// keys equal to +infinity (invalid queries) do not widen the span
__global__ __launch_bounds__(MT) void k_minmax(const uint64_t *__restrict__ keys, uint32_t n,
                                               uint64_t *__restrict__ partials) {
    __shared__ uint64_t s_red[MNW * 2];
    uint64_t lo = ~0ull, hi = 0;
    // pairs of keys with 16-byte loads when the caller's array allows it
    const bool aligned = (reinterpret_cast<uintptr_t>(keys) & 15) == 0;
    const uint32_t npair = aligned ? n / 2 : 0;
    for (uint32_t i = (aligned ? 2 * npair : 0) + blockIdx.x * MT + threadIdx.x; i < n; i += gridDim.x * MT) {
        const uint64_t x = keys[i];
        if (x != KEY_MAX) {
            lo = x < lo ? x : lo;
            hi = x > hi ? x : hi;
        }
    }
    const ulonglong2 *k2 = reinterpret_cast<const ulonglong2 *>(keys);
    for (uint32_t i = blockIdx.x * MT + threadIdx.x; i < npair; i += gridDim.x * MT) {
        const ulonglong2 p = k2[i];
        if (p.x != KEY_MAX) {
            lo = p.x < lo ? p.x : lo;
            hi = p.x > hi ? p.x : hi;
        }
        if (p.y != KEY_MAX) {
            lo = p.y < lo ? p.y : lo;
            hi = p.y > hi ? p.y : hi;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t a = shfl_xor_u64(lo, o), b = shfl_xor_u64(hi, o);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    if (lane_id() == 0) {
        s_red[threadIdx.x >> 6] = lo;
        s_red[MNW + (threadIdx.x >> 6)] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < MNW; i++) {
            lo = s_red[i] < lo ? s_red[i] : lo;
            hi = s_red[MNW + i] > hi ? s_red[MNW + i] : hi;
        }
        partials[2 * blockIdx.x] = lo;
        partials[2 * blockIdx.x + 1] = hi;
    }
}

// The range map from the min/max partials.  Also clears the big-window count
// and the writers flag (when given): the first kernels to touch them run
// after this one.
__global__ __launch_bounds__(MT) void k_make_map(const uint64_t *__restrict__ partials, uint32_t nparts,
                                                 RangeMap *map, unsigned int *nbig, unsigned int *writers,
                                                 uint32_t bits) {
    __shared__ uint64_t s_red[MNW * 2];
    uint64_t lo = ~0ull, hi = 0;
    for (uint32_t i = threadIdx.x; i < nparts; i += MT) {
        const uint64_t a = partials[2 * i], b = partials[2 * i + 1];
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t a = shfl_xor_u64(lo, o), b = shfl_xor_u64(hi, o);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    if (lane_id() == 0) {
        s_red[threadIdx.x >> 6] = lo;
        s_red[MNW + (threadIdx.x >> 6)] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < MNW; i++) {
            lo = s_red[i] < lo ? s_red[i] : lo;
            hi = s_red[MNW + i] > hi ? s_red[MNW + i] : hi;
        }
        *map = span_map(lo, hi, bits);
        *nbig = 0;
        if (writers) *writers = 0;
    }
}

// ---- 3. bitonic sort of a window held 8 entries per thread ----------------

__device__ __forceinline__ bool ki_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

// entries e and e^stride form a pair; blocks of `size` alternate direction
__device__ __forceinline__ void keep_or_take(uint64_t &k, uint32_t &v, uint64_t pk, uint32_t pv, uint32_t e,
                                             uint32_t size, uint32_t stride) {
    const bool up = (e & size) == 0;
    const bool low = (e & stride) == 0;
    const bool less = ki_less(k, v, pk, pv);
    const bool keep = (low == up) ? less : !less;
    if (!keep) {
        k = pk;
        v = pv;
    }
}

template <int S>
__device__ __forceinline__ void intra_thread(uint64_t (&k)[WE], uint32_t (&v)[WE], uint32_t size) {
    const uint32_t base = threadIdx.x * WE;
#pragma unroll
    for (int r = 0; r < WE; r++) {
        if (r & S) continue;
        const int r2 = r + S;
        const bool up = ((base + r) & size) == 0;
        const bool sw = up ? ki_less(k[r2], v[r2], k[r], v[r]) : ki_less(k[r], v[r], k[r2], v[r2]);
        if (sw) {
            const uint64_t tk = k[r];
            k[r] = k[r2];
            k[r2] = tk;
            const uint32_t tv = v[r];
            v[r] = v[r2];
            v[r2] = tv;
        }
    }
}

// Sorts entries 0..P-1 (P a power of two, WE <= P <= WMAX) ascending by
// (key, position); thread t holds entries t*WE .. t*WE+WE-1.
__device__ void bitonic_block(uint64_t (&k)[WE], uint32_t (&v)[WE], uint32_t P, uint64_t *s_k, uint32_t *s_v) {
    const uint32_t t = threadIdx.x;
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= (uint32_t)WE * 64) {  // partner in another wave
#pragma unroll
                for (int r = 0; r < WE; r++) {
                    s_k[t * WE + r] = k[r];
                    s_v[t * WE + r] = v[r];
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < WE; r++) {
                    const uint32_t e = t * WE + r;
                    keep_or_take(k[r], v[r], s_k[e ^ stride], s_v[e ^ stride], e, size, stride);
                }
                __syncthreads();
            } else if (stride >= (uint32_t)WE) {  // partner in another lane of this wave
                const int m = (int)(stride / WE);
#pragma unroll
                for (int r = 0; r < WE; r++) {
                    const uint64_t pk = shfl_xor_u64(k[r], m);
                    const uint32_t pv = __shfl_xor(v[r], m, 64);
                    keep_or_take(k[r], v[r], pk, pv, t * WE + r, size, stride);
                }
            } else if (stride == 4) {
                intra_thread<4>(k, v, size);
            } else if (stride == 2) {
                intra_thread<2>(k, v, size);
            } else {
                intra_thread<1>(k, v, size);
            }
        }
    }
}

// First index after j whose u differs from u(j) (n if none).  u is
// non-decreasing over the grouped array, so one wave probes 64 candidates per
// round: first the next 64 entries, then a 64-ary search.  Wave-uniform.
__device__ uint32_t group_end(const uint64_t *__restrict__ k, uint32_t n, const RangeMap &map, uint32_t j) {
    const int lane = lane_id();
    const uint32_t uj = range_pos(k[j], map);
    {
        const uint32_t i = j + 1 + lane;
        const bool diff = i >= n || range_pos(k[i], map) != uj;
        const uint64_t b = ballot64(diff);
        if (b) return j + 1 + (uint32_t)__builtin_ctzll(b);
    }
    uint32_t lo = j + 64, hi = n;  // u(lo) == uj, first differing index is in (lo, hi]
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63) / 64;
        uint32_t p = lo + (uint32_t)(lane + 1) * step;
        if (p > hi) p = hi;
        const bool diff = p >= n || range_pos(k[p], map) != uj;
        const uint64_t b = ballot64(diff | (p == hi));
        const int f = __builtin_ctzll(b);
        const uint32_t pf = __shfl(p, f, 64);
        const uint32_t pprev = __shfl(p, f > 0 ? f - 1 : 0, 64);
        hi = pf;  // u(hi) differs from uj, or hi == n
        if (f > 0) lo = pprev;  // u(lo) == uj
    }
    return hi;
}

// Adjusted bounds of window b: a group belongs to the window holding its
// first entry.  Called by the first wave of the block.
__device__ __forceinline__ void window_bounds(const uint64_t *__restrict__ k, uint32_t n, const RangeMap &map,
                                              uint32_t b, uint32_t &s, uint32_t &e) {
    const uint32_t s0 = b * WNOM;
    const uint32_t e0 = s0 + WNOM < n ? s0 + WNOM : n;
    s = s0 > 0 ? (range_pos(k[s0 - 1], map) == range_pos(k[s0], map) ? group_end(k, n, map, s0 - 1) : s0) : 0;
    e = e0 < n ? (range_pos(k[e0 - 1], map) == range_pos(k[e0], map) ? group_end(k, n, map, e0 - 1) : e0) : n;
}

// A batch without INSERT/DELETE (writers flag 0) needs the order only for
// locality -- no node gets a writer and no answer depends on the order of
// different keys -- so it stops at the grouping by u; writers == nullptr
// always orders fully.
__global__ __launch_bounds__(WT) void k_fixup(uint64_t *__restrict__ kk, uint32_t *__restrict__ vv, uint32_t n,
                                              const RangeMap *__restrict__ mapp, uint32_t *__restrict__ big,
                                              unsigned int *nbig, unsigned int *dirty,
                                              const unsigned int *writers) {
    __shared__ uint64_t s_k[WMAX];
    __shared__ uint32_t s_v[WMAX];
    __shared__ uint32_t s_h[WMAX + 1];  // group heads, in order
    __shared__ uint8_t s_gd[WMAX];      // per group: some entry has a smaller key than the one before it
    __shared__ uint32_t s_b[2];
    __shared__ uint32_t s_tmp[WNW + 1];
    __shared__ unsigned int s_gmax;
    const RangeMap map = *mapp;
    if (blockIdx.x * WNOM >= n) return;
    if (writers && *writers == 0) return;
    if (threadIdx.x < 64) {
        uint32_t s, e;
        window_bounds(kk, n, map, blockIdx.x, s, e);
        if (threadIdx.x == 0) {
            s_b[0] = s;
            s_b[1] = e;
            s_gmax = 1;
        }
    }
    __syncthreads();
    const uint32_t s = s_b[0], e = s_b[1];
    if (s >= e) return;  // inside a group owned by an earlier window
    // A window longer than WMAX ends with one group that runs past the
    // nominal end (everything before it lies inside the nominal range): that
    // group is handed to the large-window path, the rest is ordered here.
    const bool large = e - s > WMAX;
    const uint32_t e0 = (blockIdx.x + 1) * WNOM;  // < e when large
    uint32_t m = large ? e0 - s : e - s;
    for (uint32_t x = threadIdx.x; x < m; x += WT) {
        s_k[x] = kk[s + x];
        s_v[x] = vv[s + x];
    }
    __syncthreads();
    // group heads (entries t*WE .. t*WE+WE-1 per thread), listed in order
    const uint32_t t0 = threadIdx.x * WE;
    uint32_t hmask = 0, nh = 0;
#pragma unroll
    for (int r = 0; r < WE; r++) {
        const uint32_t x = t0 + r;
        if (x < m && (x == 0 || range_pos(s_k[x], map) != range_pos(s_k[x - 1], map))) {
            hmask |= 1u << r;
            nh++;
        }
    }
    uint32_t nheads;
    uint32_t rank = block_excl_scan_u32<WT>(nh, s_tmp, &nheads);
#pragma unroll
    for (int r = 0; r < WE; r++)
        if (hmask & (1u << r)) s_h[rank++] = t0 + r;
    __syncthreads();
    if (large) {
        const uint32_t g = s_h[nheads - 1];  // start of the group that runs past e0
        if (threadIdx.x == 0) {
            const unsigned int j = atomicAdd(nbig, 1u);
            big[2 * j] = s + g;
            big[2 * j + 1] = e - (s + g);
            dirty[j] = 0;
        }
        m = g;
        nheads -= 1;
    }
    if (threadIdx.x == 0) s_h[nheads] = m;
    for (uint32_t g = threadIdx.x; g < nheads; g += WT) s_gd[g] = 0;
    __syncthreads();
    // The radix passes are stable, so a group is in (key, input position)
    // order unless some entry has a smaller key than the one before it:
    // groups of one key repeated (hot keys) need nothing.  Only the groups
    // with such a descent are ordered.
    bool desc = false;
#pragma unroll
    for (int r = 0; r < WE; r++) {
        const uint32_t x = t0 + r;
        if (x == 0 || x >= m || (hmask & (1u << r)) || s_k[x] >= s_k[x - 1]) continue;
        desc = true;
        uint32_t lo = 0, hi = nheads;  // the group holding x: last head <= x
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_h[mid] <= x) lo = mid; else hi = mid;
        }
        s_gd[lo] = 1;
    }
    if (!__syncthreads_or(desc)) return;  // every group is in order already
    uint32_t gmax = 1;
    for (uint32_t g = threadIdx.x; g < nheads; g += WT)
        if (s_gd[g]) gmax = max(gmax, s_h[g + 1] - s_h[g]);
    if (gmax > 1) atomicMax(&s_gmax, gmax);
    __syncthreads();
    const uint32_t G = s_gmax;
    if (G <= 32) {
        // insertion sort of each such group by (key, input position)
        for (uint32_t g = threadIdx.x; g < nheads; g += WT) {
            const uint32_t a = s_h[g], z = s_h[g + 1];
            if (!s_gd[g]) continue;
            for (uint32_t x = a + 1; x < z; x++) {
                const uint64_t ck = s_k[x];
                const uint32_t cv = s_v[x];
                uint32_t y = x;
                while (y > a && ki_less(ck, cv, s_k[y - 1], s_v[y - 1])) {
                    s_k[y] = s_k[y - 1];
                    s_v[y] = s_v[y - 1];
                    y--;
                }
                s_k[y] = ck;
                s_v[y] = cv;
            }
            for (uint32_t x = a; x < z; x++) {
                kk[s + x] = s_k[x];
                vv[s + x] = s_v[x];
            }
        }
        return;
    }
    // a larger group: bitonic sort of the whole window (the order by key
    // refines the order by position u)
    uint32_t P = WE;
    while (P < m) P <<= 1;
    uint64_t k[WE];
    uint32_t v[WE];
#pragma unroll
    for (int r = 0; r < WE; r++) {
        const uint32_t x = t0 + r;
        k[r] = x < m ? s_k[x] : KEY_MAX;
        v[r] = x < m ? s_v[x] : 0xFFFFFFFFu;
    }
    __syncthreads();  // s_k/s_v become the exchange buffer
    bitonic_block(k, v, P, s_k, s_v);
#pragma unroll
    for (int r = 0; r < WE; r++) {
        const uint32_t x = t0 + r;
        if (x < m) {
            kk[s + x] = k[r];
            vv[s + x] = v[r];
        }
    }
}

// Marks a large window dirty when some entry has a smaller key than the one
// before it (otherwise the stable passes left it in (key, input position)
// order: one key repeated, or keys that arrived in order).  All blocks share
// the work: the windows' sizes are prefix-summed in LDS and the blocks stride
// over fixed-size chunks of the concatenated windows.
constexpr uint32_t CHECK_CHUNK = 4096;
constexpr uint32_t CHECK_LIST = 4096;

__global__ __launch_bounds__(WT) void k_big_check(const uint64_t *__restrict__ kk, const uint32_t *__restrict__ big,
                                                  const unsigned int *nbig, unsigned int *dirty) {
    __shared__ uint32_t s_pre[CHECK_LIST + 1];  // first chunk of each window
    __shared__ uint32_t s_tmp[WNW + 1];
    const unsigned int nb = *nbig;
    if (nb == 0) return;
    if (nb > CHECK_LIST) {  // too many to list: one window per block
        for (unsigned int j = blockIdx.x; j < nb; j += gridDim.x) {
            const uint32_t s = big[2 * j], m = big[2 * j + 1];
            bool desc = false;
            for (uint32_t x = threadIdx.x + 1; x < m; x += WT) desc |= kk[s + x] < kk[s + x - 1];
            if (__syncthreads_or(desc) && threadIdx.x == 0) dirty[j] = 1;
        }
        return;
    }
    for (uint32_t base = 0; base < nb; base += WT) {
        const uint32_t j = base + threadIdx.x;
        const uint32_t c = j < nb ? (big[2 * j + 1] + CHECK_CHUNK - 1) / CHECK_CHUNK : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan_u32<WT>(c, s_tmp, &tot);
        const uint32_t carry = base == 0 ? 0u : s_pre[base];
        if (j < nb) s_pre[j] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_pre[base + WT < nb ? base + WT : nb] = carry + tot;
        __syncthreads();
    }
    const uint32_t nchunks = s_pre[nb];
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        // window of chunk c: last j with s_pre[j] <= c
        uint32_t lo = 0, hi = nb;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_pre[mid] <= c) lo = mid; else hi = mid;
        }
        const uint32_t j = lo;
        const uint32_t s = big[2 * j], m = big[2 * j + 1];
        const uint32_t off = (c - s_pre[j]) * CHECK_CHUNK;
        const uint32_t len = m - off < CHECK_CHUNK ? m - off : CHECK_CHUNK;
        bool desc = false;
        for (uint32_t x = threadIdx.x + (off == 0 ? 1u : 0u); x < len; x += WT)
            desc |= kk[s + off + x] < kk[s + off + x - 1];
        if (__syncthreads_or(desc) && threadIdx.x == 0) dirty[j] = 1;
    }
}

// ---- 4. groups larger than one block ---------------------------------------

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t x, uint32_t *s_w) {
    x = wave_sum_u32(x);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    uint32_t r = 0;
    for (int i = 0; i < WNW; i++) r += s_w[i];
    __syncthreads();
    return r;
}

// stable in-block sort of dst[0..m) (m <= WMAX) in place
__device__ void sort_small_inplace(uint64_t *dk, uint32_t *dv, uint32_t m, uint64_t *s_k, uint32_t *s_v) {
    if (m <= 1) return;
    uint32_t P = WE;
    while (P < m) P <<= 1;
    uint64_t k[WE];
    uint32_t v[WE];
    const uint32_t t0 = threadIdx.x * WE;
#pragma unroll
    for (int r = 0; r < WE; r++) {
        const uint32_t x = t0 + r;
        k[r] = x < m ? dk[x] : KEY_MAX;
        v[r] = x < m ? dv[x] : 0xFFFFFFFFu;
    }
    __syncthreads();
    bitonic_block(k, v, P, s_k, s_v);
#pragma unroll
    for (int r = 0; r < WE; r++) {
        const uint32_t x = t0 + r;
        if (x < m) {
            dk[x] = k[r];
            dv[x] = v[r];
        }
    }
    __syncthreads();
}

// Stable LSD over the varying 8-bit digits of src[0..m), ping-pong with dst;
// the result ends in dst.
__device__ void block_lsd(uint64_t *sk_, uint32_t *si_, uint64_t *dk_, uint32_t *di_, uint32_t m, uint32_t *s_hist,
                          uint32_t *s_cnt /* [WNW][256] */, uint32_t *s_tmp, uint64_t *s_red) {
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    uint64_t o = 0, a = ~0ull;
    for (uint32_t e = threadIdx.x; e < m; e += WT) {
        const uint64_t kk = sk_[e];
        o |= kk;
        a &= kk;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        o |= shfl_xor_u64(o, off);
        a &= shfl_xor_u64(a, off);
    }
    if (lane == 0) {
        s_red[w] = o;
        s_red[WNW + w] = a;
    }
    __syncthreads();
    uint64_t oo = 0, aa = ~0ull;
    for (int i = 0; i < WNW; i++) {
        oo |= s_red[i];
        aa &= s_red[WNW + i];
    }
    __syncthreads();
    const uint64_t diff = oo ^ aa;
    uint64_t *src_k = sk_, *dst_k = dk_;
    uint32_t *src_i = si_, *dst_i = di_;
    for (uint32_t shift = 0; shift < 64; shift += 8) {
        if (((diff >> shift) & 255u) == 0) continue;
        if (threadIdx.x < 256) s_hist[threadIdx.x] = 0;
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < m; e += WT) atomicAdd(&s_hist[(uint32_t)(src_k[e] >> shift) & 255u], 1u);
        __syncthreads();
        {
            uint32_t tot;
            const uint32_t v = threadIdx.x < 256 ? s_hist[threadIdx.x] : 0u;
            const uint32_t ex = block_excl_scan_u32<WT>(v, s_tmp, &tot);
            if (threadIdx.x < 256) s_hist[threadIdx.x] = ex;
        }
        __syncthreads();
        // chunks of WMAX in order; inside a chunk rank stably per wave
        for (uint32_t c0 = 0; c0 < m; c0 += WMAX) {
            for (int j = threadIdx.x; j < WNW * 256; j += WT) s_cnt[j] = 0;
            __syncthreads();
            uint64_t k[WE];
            uint32_t v[WE], rk[WE];
            bool valid[WE];
#pragma unroll
            for (int r = 0; r < WE; r++) {
                const uint32_t e = c0 + w * (WE * 64) + r * 64 + lane;
                valid[r] = e < m;
                k[r] = valid[r] ? src_k[e] : 0;
                v[r] = valid[r] ? src_i[e] : 0;
            }
#pragma unroll
            for (int r = 0; r < WE; r++) {
                const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
                uint64_t msk = ballot64(valid[r]);
#pragma unroll
                for (int b = 0; b < 8; b++) {
                    const bool bit = (d >> b) & 1u;
                    const uint64_t bl = ballot64(bit);
                    msk &= bit ? bl : ~bl;
                }
                const uint32_t before = s_cnt[w * 256 + d];
                if (valid[r] && lane == (int)__builtin_ctzll(msk)) s_cnt[w * 256 + d] = before + (uint32_t)__popcll(msk);
                rk[r] = before + mask_rank(msk);
            }
            __syncthreads();
            if (threadIdx.x < 256) {  // wave offsets inside the chunk, then chunk totals into s_hist
                const uint32_t d = threadIdx.x;
                uint32_t run = s_hist[d];
                for (int ww = 0; ww < WNW; ww++) {
                    const uint32_t c = s_cnt[ww * 256 + d];
                    s_cnt[ww * 256 + d] = run;
                    run += c;
                }
                s_hist[d] = run;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < WE; r++) {
                if (valid[r]) {
                    const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
                    const uint32_t pos = s_cnt[w * 256 + d] + rk[r];
                    dst_k[pos] = k[r];
                    dst_i[pos] = v[r];
                }
            }
            __syncthreads();
        }
        uint64_t *tk = src_k;
        src_k = dst_k;
        dst_k = tk;
        uint32_t *ti = src_i;
        src_i = dst_i;
        dst_i = ti;
        __syncthreads();
    }
    if (src_k != dk_) {
        for (uint32_t e = threadIdx.x; e < m; e += WT) {
            dk_[e] = src_k[e];
            di_[e] = src_i[e];
        }
    }
    __syncthreads();
}

// block_lsd leaving the result in place (dk/dv), with sk/sv as scratch
__device__ void block_lsd_inplace(uint64_t *dk, uint32_t *dv, uint64_t *sk, uint32_t *sv, uint32_t m,
                                  uint32_t *s_hist, uint32_t *s_cnt, uint32_t *s_tmp, uint64_t *s_red) {
    block_lsd(dk, dv, sk, sv, m, s_hist, s_cnt, s_tmp, s_red);
    for (uint32_t e = threadIdx.x; e < m; e += WT) {
        dk[e] = sk[e];
        dv[e] = sv[e];
    }
    __syncthreads();
}

// Orders a dirty large window in place (kk/vv), using the same region of the
// other buffer (sk/sv) as scratch.
__global__ __launch_bounds__(WT) void k_big_fixup(uint64_t *__restrict__ kk, uint32_t *__restrict__ vv,
                                                  uint64_t *__restrict__ sk, uint32_t *__restrict__ sv,
                                                  const uint32_t *__restrict__ big, const unsigned int *nbig,
                                                  const unsigned int *dirty) {
    __shared__ uint64_t s_k[WMAX];
    __shared__ uint32_t s_v[WMAX];
    __shared__ uint32_t s_cnt[WNW * 256];
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_tmp[WNW + 1];
    __shared__ uint32_t s_w[WNW];
    __shared__ uint64_t s_red[2 * WNW];
    const unsigned int nwork = *nbig;
    for (unsigned int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
        if (!dirty[wi]) continue;
        const uint32_t s = big[2 * wi], m = big[2 * wi + 1];
        uint64_t *ak = kk + s, *bk = sk + s;
        uint32_t *ai = vv + s, *bi = sv + s;
        const uint64_t K = ak[m / 2];
        uint32_t lt = 0, eq = 0;
        for (uint32_t e = threadIdx.x; e < m; e += WT) {
            const uint64_t x = ak[e];
            lt += x < K;
            eq += x == K;
        }
        const uint32_t nlt = block_sum_u32(lt, s_w), neq = block_sum_u32(eq, s_w);
        if (2 * (uint64_t)neq < m) {
            block_lsd_inplace(ak, ai, bk, bi, m, s_hist, s_cnt, s_tmp, s_red);
            continue;
        }
        // stable three-way split around the dominant key K into the scratch
        uint32_t run_lt = 0, run_eq = 0, run_gt = 0;
        const uint32_t base_eq = nlt, base_gt = nlt + neq;
        for (uint32_t c0 = 0; c0 < m; c0 += WMAX) {
            uint64_t k[WE];
            uint32_t v[WE];
            uint32_t clt = 0, ceq = 0, cgt = 0;
            const uint32_t t0 = c0 + threadIdx.x * WE;
#pragma unroll
            for (int r = 0; r < WE; r++) {
                const uint32_t x = t0 + r;
                k[r] = x < m ? ak[x] : 0;
                v[r] = x < m ? ai[x] : 0;
                if (x < m) {
                    clt += k[r] < K;
                    ceq += k[r] == K;
                    cgt += k[r] > K;
                }
            }
            uint32_t tlt, teq, tgt;
            uint32_t plt = block_excl_scan_u32<WT>(clt, s_tmp, &tlt);
            uint32_t peq = block_excl_scan_u32<WT>(ceq, s_tmp, &teq);
            uint32_t pgt = block_excl_scan_u32<WT>(cgt, s_tmp, &tgt);
#pragma unroll
            for (int r = 0; r < WE; r++) {
                const uint32_t x = t0 + r;
                if (x >= m) continue;
                uint32_t pos;
                if (k[r] < K)
                    pos = run_lt + plt++;
                else if (k[r] == K)
                    pos = base_eq + run_eq + peq++;
                else
                    pos = base_gt + run_gt + pgt++;
                bk[pos] = k[r];
                bi[pos] = v[r];
            }
            run_lt += tlt;
            run_eq += teq;
            run_gt += tgt;
            __syncthreads();
        }
        // the copies of K are in input order already; order the rest, then
        // copy the window back
        const uint32_t ngt = m - nlt - neq;
        if (nlt <= WMAX)
            sort_small_inplace(bk, bi, nlt, s_k, s_v);
        else
            block_lsd_inplace(bk, bi, ak, ai, nlt, s_hist, s_cnt, s_tmp, s_red);
        if (ngt <= WMAX)
            sort_small_inplace(bk + base_gt, bi + base_gt, ngt, s_k, s_v);
        else
            block_lsd_inplace(bk + base_gt, bi + base_gt, ak + base_gt, ai + base_gt, ngt, s_hist, s_cnt, s_tmp,
                              s_red);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < m; e += WT) {
            ak[e] = bk[e];
            ai[e] = bi[e];
        }
        __syncthreads();
    }
}

}  // namespace

void MsdWorkspace::ensure(uint64_t n) {
    partials.ensure(2 * MM_BLOCKS * sizeof(uint64_t));
    map.ensure(64);
    const uint64_t nw = n / WNOM + 2;
    big.ensure(2 * nw * sizeof(uint32_t));
    dirty.ensure(nw * sizeof(uint32_t));
    nbig.ensure(64);
    wflag.ensure(64);
}

void MsdWorkspace::release() {
    partials.release();
    map.release();
    big.release();
    dirty.release();
    nbig.release();
    wflag.release();
}

void sort_batch_by_range(SortWorkspace &ws, MsdWorkspace &mw, const uint64_t *keys, const uint8_t *ops, uint64_t n,
                         bool batch, hipStream_t s, const uint64_t **out_keys, const uint32_t **out_idx,
                         uint32_t pos_bits) {
    if (pos_bits == 0) pos_bits = n > (1u << 20) ? 32 : 24;
    if (pos_bits != 16 && pos_bits != 24 && pos_bits != 32)
        throw Error{PI_ERR_INVALID_ARG, "internal error: range position width"};
    ws.ensure(n);
    mw.ensure(n);
    uint64_t *ka = ws.keys[0].as<uint64_t>(), *kb = ws.keys[1].as<uint64_t>();
    uint32_t *ia = ws.idx[0].as<uint32_t>(), *ib = ws.idx[1].as<uint32_t>();
    *out_keys = ka;
    *out_idx = ia;
    if (n == 0) return;
    const uint32_t nn = (uint32_t)n;
    RangeMap *map = mw.map.as<RangeMap>();
    const uint32_t parts = std::max<uint32_t>(1, std::min<uint32_t>(MM_BLOCKS, (nn + MT * 16 - 1) / (MT * 16)));
    hipLaunchKernelGGL(k_minmax, dim3(parts), dim3(MT), 0, s, keys, nn, mw.partials.as<uint64_t>());
    unsigned int *wf = batch ? mw.wflag.as<unsigned int>() : nullptr;
    hipLaunchKernelGGL(k_make_map, dim3(1), dim3(MT), 0, s, mw.partials.as<uint64_t>(), parts, map,
                       mw.nbig.as<unsigned int>(), wf, pos_bits);
    PI_LAUNCH_CHECK();
    // group by the position inside the span, one byte per pass; the result
    // lands in (ka, ia) either way
    if (pos_bits == 32) {
        radix_pass(ws, keys, nullptr, ops, nn, 0, map, wf, kb, ib, s);
        radix_pass(ws, kb, ib, nullptr, nn, 8, map, nullptr, ka, ia, s);
        radix_pass(ws, ka, ia, nullptr, nn, 16, map, nullptr, kb, ib, s);
        radix_pass(ws, kb, ib, nullptr, nn, 24, map, nullptr, ka, ia, s);
    } else if (pos_bits == 24) {
        radix_pass(ws, keys, nullptr, ops, nn, 0, map, wf, ka, ia, s);
        radix_pass(ws, ka, ia, nullptr, nn, 8, map, nullptr, kb, ib, s);
        radix_pass(ws, kb, ib, nullptr, nn, 16, map, nullptr, ka, ia, s);
    } else {
        radix_pass(ws, keys, nullptr, ops, nn, 0, map, wf, kb, ib, s);
        radix_pass(ws, kb, ib, nullptr, nn, 8, map, nullptr, ka, ia, s);
    }
    const uint32_t nwin = (nn + WNOM - 1) / WNOM;
    hipLaunchKernelGGL(k_fixup, dim3(nwin), dim3(WT), 0, s, ka, ia, nn, map, mw.big.as<uint32_t>(),
                       mw.nbig.as<unsigned int>(), mw.dirty.as<unsigned int>(), (const unsigned int *)wf);
    hipLaunchKernelGGL(k_big_check, dim3(1024), dim3(WT), 0, s, ka, mw.big.as<uint32_t>(), mw.nbig.as<unsigned int>(),
                       mw.dirty.as<unsigned int>());
    hipLaunchKernelGGL(k_big_fixup, dim3(BIG_GRID), dim3(WT), 0, s, ka, ia, kb, ib, mw.big.as<uint32_t>(),
                       mw.nbig.as<unsigned int>(), mw.dirty.as<unsigned int>());
    PI_LAUNCH_CHECK();
}

}  // namespace pi
