// Device-side pieces of the index descent shared by the batch kernels and
// the range search: the level step (Algorithm 2) in LDS and in global memory,
// the LDS staging of the upper levels, and getNode of Algorithm 4 (the walk
// along the storage list from an interception).
#pragma once

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "index.h"

namespace pi {
namespace {

constexpr uint32_t WALK_LIMIT = 1u << 24;  // bound on storage nodes walked by one query

// ---------------------------------------------------------------- descent --

// One level of the descent (Algorithm 2) for one query.  pos is the entry of
// the key the query stands on (present one level up too), or the head.  The
// first two keys after pos and the down pointers of pos, pos+1, pos+2 are
// requested together -- the paper's wide compare of an entry, with the routing
// table replaced by the down array -- so the common case costs one memory
// round trip; a longer run of keys <= q continues one key at a time.  Reads
// stay inside the level's +infinity pad because q < +infinity.
struct Step {
    uint64_t k1, k2;
    uint32_t d0, d1, d2;
};

template <class KP, class DP>
__device__ __forceinline__ Step step_load(KP K, DP D, uint32_t pos) {
    Step s;
    s.k1 = K[pos + 1];
    s.k2 = K[pos + 2];
    s.d0 = D[pos];
    s.d1 = D[pos + 1];
    s.d2 = D[pos + 2];
    return s;
}

template <class KP, class DP>
__device__ __forceinline__ uint32_t step_finish(KP K, DP D, const Step &s, uint64_t q, uint32_t pos,
                                                uint64_t &last) {
    if (s.k1 > q) return s.d0;
    last = s.k1;
    if (s.k2 > q) return s.d1;
    last = s.k2;
    uint32_t p = pos + 2, dp = s.d2;
    for (;;) {
        const uint64_t kn = K[p + 1];
        const uint32_t dn = D[p + 1];
        if (kn > q) return dp;
        last = kn;
        p++;
        dp = dn;
    }
}

// Length of the run of keys <= q starting at keys[skip] (only the leading
// run counts: entries after the first key > q may hold anything).
template <int N>
__device__ __forceinline__ uint32_t leading_le(const uint64_t (&keys)[N], uint32_t skip, uint64_t q) {
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < N; i++) m |= (keys[i] <= q ? 1u : 0u) << i;
    m >>= skip;
    return (uint32_t)__builtin_ctz(~m);
}

// Level step in global memory with a window of KP key pairs and DQ down
// quads.  Keys are read as 16-byte pairs starting at the even entry at or
// below pos+1 (levels start on 128-byte lines), down pointers as 16-byte quads
// starting at the multiple of 4 at or below pos: with KP = 4, DQ = 3 one round
// trip covers keys pos+1 .. pos+7 (at least) and down pointers pos .. pos+8.
// With p = 1/2 a run of 7 keys <= q on one level is rare enough that a wave of
// queries almost never waits for a second trip.
template <int KP, int DQ>
struct Wide {
    ulonglong2 kp[KP];
    uint4 dq[DQ];
};

template <int KP, int DQ>
__device__ __forceinline__ Wide<KP, DQ> wide_load(const uint64_t *__restrict__ K, const uint32_t *__restrict__ D,
                                                  uint32_t pos) {
    Wide<KP, DQ> w;
    const ulonglong2 *K2 = reinterpret_cast<const ulonglong2 *>(K + ((pos + 1) & ~1u));
    const uint4 *D4 = reinterpret_cast<const uint4 *>(D + (pos & ~3u));
#pragma unroll
    for (int i = 0; i < KP; i++) w.kp[i] = K2[i];
#pragma unroll
    for (int i = 0; i < DQ; i++) w.dq[i] = D4[i];
    return w;
}

template <int KP, int DQ>
__device__ __forceinline__ uint32_t wide_finish(const uint64_t *__restrict__ K, const uint32_t *__restrict__ D,
                                                const Wide<KP, DQ> &w, uint64_t q, uint32_t pos, uint64_t &last) {
    constexpr int NK = 2 * KP, ND = 4 * DQ;
    uint64_t keys[NK];
#pragma unroll
    for (int i = 0; i < KP; i++) {
        keys[2 * i] = w.kp[i].x;
        keys[2 * i + 1] = w.kp[i].y;
    }
    const uint32_t skip = (pos + 1) & 1u;  // entry pos+1 is keys[skip]
    const uint32_t cnt = leading_le<NK>(keys, skip, q);
    uint32_t p = pos + cnt;
    if (cnt > 0) {
        const uint32_t li = skip + cnt - 1;
        uint64_t lk = keys[0];
#pragma unroll
        for (int i = 1; i < NK; i++) lk = ((uint32_t)i == li) ? keys[i] : lk;
        last = lk;
    }
    if (cnt < NK - skip) {
        const uint32_t di = p - (pos & ~3u);
        if (di >= (uint32_t)ND) return D[p];  // run ended past the down window
        uint32_t downs[ND];
#pragma unroll
        for (int i = 0; i < DQ; i++) {
            downs[4 * i] = w.dq[i].x;
            downs[4 * i + 1] = w.dq[i].y;
            downs[4 * i + 2] = w.dq[i].z;
            downs[4 * i + 3] = w.dq[i].w;
        }
        uint32_t d = downs[0];
#pragma unroll
        for (int i = 1; i < ND; i++) d = ((uint32_t)i == di) ? downs[i] : d;
        return d;
    }
    for (;;) {  // window exhausted: the next window from p
        const Wide<KP, DQ> w2 = wide_load<KP, DQ>(K, D, p);
        uint64_t k2[NK];
#pragma unroll
        for (int i = 0; i < KP; i++) {
            k2[2 * i] = w2.kp[i].x;
            k2[2 * i + 1] = w2.kp[i].y;
        }
        const uint32_t sk2 = (p + 1) & 1u;
        const uint32_t c2 = leading_le<NK>(k2, sk2, q);
        if (c2 > 0) {
            const uint32_t li2 = sk2 + c2 - 1;
            uint64_t lk = k2[0];
#pragma unroll
            for (int i = 1; i < NK; i++) lk = ((uint32_t)i == li2) ? k2[i] : lk;
            last = lk;
        }
        const uint32_t p0 = p;
        p += c2;
        if (c2 < NK - sk2) {
            const uint32_t di = p - (p0 & ~3u);
            if (di >= (uint32_t)ND) return D[p];
            uint32_t downs[ND];
#pragma unroll
            for (int i = 0; i < DQ; i++) {
                downs[4 * i] = w2.dq[i].x;
                downs[4 * i + 1] = w2.dq[i].y;
                downs[4 * i + 2] = w2.dq[i].z;
                downs[4 * i + 3] = w2.dq[i].w;
            }
            uint32_t d = downs[0];
#pragma unroll
            for (int i = 1; i < ND; i++) d = ((uint32_t)i == di) ? downs[i] : d;
            return d;
        }
    }
}

// Window of the global levels: 4 key pairs and 3 down quads.  Narrower
// windows (2 pairs) cost a second round trip too often; wider ones buy nothing.
constexpr int WIN_KP = 4;
constexpr int WIN_DQ = 3;

// Shared window of a whole wave.  On the upper global levels the 64 sorted
// queries of a wave stand on the same few entries, yet the per-lane window
// above costs seven vector loads that each pass all 64 lane addresses through
// the texture addresser, the busiest unit of the descent.  When every lane
// stands within UW_SLACK entries of the first lane's entry w0, one load by 12
// lanes fetches the wave's window instead: lanes 0..7 the 8 key pairs from the
// even entry kb at or below w0+1, lanes 8..11 the 4 down quads from the
// multiple of 4 at or below w0.  The keys go to every lane (readlane), and
// each lane counts those <= its query: every key between w0 and the lane's own
// entry is <= its query (it is at most the key the lane stands on), so the
// count is the lane's new entry minus w0.  Its key and down pointer come from
// the holding lane (bpermute).
constexpr uint32_t UW_SLACK = 8;

// Reads keys kb .. kb+15 and downs db .. db+15: inside the level and its
// +infinity pad (w0 <= n, LEVEL_PAD >= 16).
__device__ __forceinline__ uint4 uni_load(const uint64_t *__restrict__ K, const uint32_t *__restrict__ D,
                                          uint32_t w0) {
    const uint32_t lane = (uint32_t)lane_id();
    const uint32_t kb = (w0 + 1) & ~1u, db = w0 & ~3u;
    // one load instruction: a per-lane address into either array
    const uint4 *src = lane < 8 ? reinterpret_cast<const uint4 *>(K + kb) + lane
                                : reinterpret_cast<const uint4 *>(D + db) + (lane - 8);
    uint4 v = make_uint4(0, 0, 0, 0);
    if (lane < 12) v = *src;
    return v;
}

__device__ __forceinline__ uint32_t lane_u32(uint32_t x, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)x);
}

// The u64 held as (lo, hi) by lane i (a wave-uniform value); the halves are
// widened unsigned.
__device__ __forceinline__ uint64_t lane_key(uint32_t lo, uint32_t hi, int i) {
    const uint32_t l = (uint32_t)__builtin_amdgcn_readlane((int)lo, i);
    const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)hi, i);
    return ((uint64_t)h << 32) | l;
}

__device__ __forceinline__ uint32_t uni_finish(const uint64_t *__restrict__ K, const uint32_t *__restrict__ D,
                                               const uint4 &v, uint64_t q, uint32_t w0, uint64_t &last) {
    const uint32_t kb = (w0 + 1) & ~1u, db = w0 & ~3u;
    // keys <= q among entries w0+1 .. kb+15 (entry kb is w0 itself when w0 is even)
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const uint64_t k0 = lane_key(v.x, v.y, i), k1 = lane_key(v.z, v.w, i);
        if (i > 0 || kb > w0) c += k0 <= q ? 1u : 0u;
        c += k1 <= q ? 1u : 0u;
    }
    const uint32_t p = w0 + c;
    // the stop's key and down pointer from the lanes holding them
    const uint32_t ko = p - kb;  // < 16 unless every window key is <= q
    const uint32_t ksrc = (ko >> 1) & 7u;
    const uint32_t x = lane_u32(v.x, ksrc), y = lane_u32(v.y, ksrc), z = lane_u32(v.z, ksrc),
                   w = lane_u32(v.w, ksrc);
    const uint32_t dof = p - db;
    const uint32_t dsrc = 8 + ((dof >> 2) & 3u);
    const uint32_t dx = lane_u32(v.x, dsrc), dy = lane_u32(v.y, dsrc), dz = lane_u32(v.z, dsrc),
                   dw = lane_u32(v.w, dsrc);
    if (p < kb + 15) {
        if (c > 0) last = (ko & 1u) ? (((uint64_t)w << 32) | z) : (((uint64_t)y << 32) | x);
        if (dof >= 16) return D[p];
        const uint32_t s = dof & 3u;
        return s == 0 ? dx : s == 1 ? dy : s == 2 ? dz : dw;
    }
    // every window key <= q: one key at a time from entry kb+15
    uint32_t r = kb + 15;
    last = lane_key(v.z, v.w, 7);
    for (;;) {
        const uint64_t kn = K[r + 1];
        if (kn > q) return D[r];
        last = kn;
        r++;
    }
}

// True (for the whole wave) when the wave is complete and every lane's QPL
// entries lie in [w0, w0 + UW_SLACK], w0 being lane 0's first entry.
template <int QPL>
__device__ __forceinline__ bool uni_fits(const uint32_t (&pos)[QPL], uint32_t &w0) {
    w0 = __builtin_amdgcn_readfirstlane(pos[0]);
    bool ok = true;
#pragma unroll
    for (int j = 0; j < QPL; j++) ok &= (pos[j] - w0) <= UW_SLACK;
    return __builtin_amdgcn_ballot_w64(true) == ~0ull && __builtin_amdgcn_ballot_w64(ok) == ~0ull;
}

// Descends QPL independent queries together, level by level (the group
// processing of Section 4.3.4): every query's loads for a level are issued
// before any of them is used.  Returns, per query, the storage slot of the
// interception (HEAD_SLOT when no indexed key is <= q) and its key.
template <int QPL>
__device__ __forceinline__ void descend_index(const uint64_t (&q)[QPL], const IndexDesc &d,
                                              const uint64_t *__restrict__ lkey, const uint32_t *__restrict__ ldown,
                                              const uint64_t *s_k, const uint32_t *s_d, uint32_t (&pos)[QPL],
                                              uint64_t (&last)[QPL]) {
#pragma unroll
    for (int j = 0; j < QPL; j++) {
        pos[j] = 0;
        last[j] = 0;
    }
    for (int l = d.top; l >= 2; l--) {
        Step st[QPL];
        if (l >= d.lds_from) {
            const uint64_t *K = s_k + d.lds_off[l];
            const uint32_t *D = s_d + d.lds_off[l];
#pragma unroll
            for (int j = 0; j < QPL; j++) st[j] = step_load(K, D, pos[j]);
#pragma unroll
            for (int j = 0; j < QPL; j++) pos[j] = step_finish(K, D, st[j], q[j], pos[j], last[j]);
        } else {
            const uint64_t *K = lkey + d.off[l];
            const uint32_t *D = ldown + d.off[l];
            uint32_t w0;
            if (uni_fits<QPL>(pos, w0)) {
                const uint4 u = uni_load(K, D, w0);
#pragma unroll
                for (int j = 0; j < QPL; j++) pos[j] = uni_finish(K, D, u, q[j], w0, last[j]);
                continue;
            }
            Wide<WIN_KP, WIN_DQ> wd[QPL];
#pragma unroll
            for (int j = 0; j < QPL; j++) wd[j] = wide_load<WIN_KP, WIN_DQ>(K, D, pos[j]);
#pragma unroll
            for (int j = 0; j < QPL; j++) pos[j] = wide_finish(K, D, wd[j], q[j], pos[j], last[j]);
        }
    }
}

__device__ __forceinline__ void stage_levels(const IndexDesc &d, const uint64_t *__restrict__ lkey,
                                             const uint32_t *__restrict__ ldown, uint64_t *s_k, uint32_t *s_d) {
    for (int l = d.top; l >= d.lds_from && l >= 2; l--) {
        const uint32_t len = d.n[l] + 1 + LEVEL_PAD;
        const uint64_t *K = lkey + d.off[l];
        const uint32_t *D = ldown + d.off[l];
        for (uint32_t j = threadIdx.x; j < len; j += blockDim.x) {
            s_k[d.lds_off[l] + j] = K[j];
            s_d[d.lds_off[l] + j] = D[j];
        }
    }
    __syncthreads();
}

struct Found {
    uint32_t node;   // last storage node with key <= q (HEAD_SLOT if none)
    uint32_t next;   // its successor
    bool exists;     // node holds q
    bool live;       // ... and is not flagged deleted
    uint64_t val;    // its value when live
};

// getNode of Algorithm 4: from the interception, follow the storage list to
// the last node whose key is <= q, then read its value.  Without linked nodes
// the successor of a base node is the next slot, so a window of keys is read
// at once.
__device__ __forceinline__ Found walk_storage(uint64_t q, uint32_t cur, uint64_t ck, bool links, bool dead,
                                              const uint64_t *__restrict__ skey, const uint64_t *__restrict__ sval,
                                              const uint32_t *__restrict__ snext,
                                              const uint8_t *__restrict__ smeta, unsigned int *errors) {
    Found f;
    // A step reads the window of the next 8 slots' keys (the same 8-entry
    // window as the index levels).  Without linked nodes the successor of
    // slot i is i+1, so the walk moves through the keys <= q of the window.
    // With linked nodes (most are still base nodes, whose successor is the
    // next slot) it also reads the flags of the slots before those keys,
    // moves up to the first linked slot, and follows its link when it gets
    // there.
    uint32_t nxt = cur + 1;
    for (uint32_t steps = 0;; steps++) {
        if (steps >= WALK_LIMIT) {  // a well-formed list never gets here
            atomicOr(errors, ERR_WALK);
            break;
        }
        const uint32_t a = (cur + 1) & ~1u;  // keys of slots a .. a+7
        const uint32_t skip = (cur + 1) & 1u;
        const ulonglong2 *S2 = reinterpret_cast<const ulonglong2 *>(skey + a);
        ulonglong2 kp[4];
#pragma unroll
        for (int i = 0; i < 4; i++) kp[i] = S2[i];
        // offset of the first linked slot from cur (9: none of cur .. cur+7;
        // a window of 8 successors ends on cur+8, whose flag the next step
        // reads)
        uint32_t firstlink = 9;
        if (links) {
            const uint32_t m0 = cur & ~7u;  // flags of slots m0 .. m0+15
            const uint64_t *M8 = reinterpret_cast<const uint64_t *>(smeta + m0);
            const uint64_t mlo = M8[0], mhi = M8[1];
            const uint32_t sh = 8 * (cur - m0);
            const uint64_t fl = sh ? (mlo >> sh) | (mhi << (64 - sh)) : mlo;  // slots cur .. cur+7
            static_assert(META_LINK == 2, "the flag test below reads bit 1 of each byte");
            const uint64_t lk = (fl >> 1) & 0x0101010101010101ull;
            if (lk) firstlink = (uint32_t)__builtin_ctzll(lk) >> 3;
        }
        const uint64_t keys[8] = {kp[0].x, kp[0].y, kp[1].x, kp[1].y, kp[2].x, kp[2].y, kp[3].x, kp[3].y};
        const uint32_t avail = 8 - skip;                          // successor keys in the window
        const uint32_t cons = firstlink < avail ? firstlink : avail;  // consecutive successors
        uint32_t cnt = leading_le<8>(keys, skip, q);                 // stops at the tail's +infinity
        cnt = cnt < cons ? cnt : cons;
        if (cnt > 0) {
            const uint32_t li = skip + cnt - 1;
            uint64_t kk = keys[0];
#pragma unroll
            for (int i = 1; i < 8; i++) kk = ((uint32_t)i == li) ? keys[i] : kk;
            ck = kk;
            cur += cnt;
        }
        if (cnt < cons) {  // the next key along the list is > q
            nxt = cur + 1;
            break;
        }
        if (cons == firstlink) {  // at a linked slot: one step along its link
            nxt = snext[cur];
            const uint64_t kn = skey[nxt];
            if (kn > q) break;
            cur = nxt;
            ck = kn;
        }
        // else the window ran out with no link: the next window
    }
    // (flags matter only for a node that holds q, and only once some node is
    // flagged deleted)
    const uint8_t mc = dead && cur != HEAD_SLOT && ck == q ? smeta[cur] : (uint8_t)0;
    f.next = nxt;
    f.node = cur;
    f.exists = cur != HEAD_SLOT && ck == q;
    f.live = f.exists && !(mc & META_DEL);
    f.val = f.live ? sval[cur] : 0;
    return f;
}

// Raises a kernel's dynamic LDS limit to at least lds, never lowers it:
// several host threads (a group call's lanes) launch the same kernel with
// different LDS sizes, and a limit lowered between another thread's setting
// and its launch would refuse that launch.
inline void raise_lds_limit(const void *kern, size_t lds) {
    static std::mutex mu;
    static std::unordered_map<const void *, size_t> limit;
    std::lock_guard<std::mutex> lock(mu);
    size_t &cur = limit[kern];
    if (lds <= cur) return;
    PI_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    cur = lds;
}

// Grid of a persistent kernel that stages the upper levels in LDS: as many
// blocks as can be resident on all CUs, at most one per tile, a multiple of 8
// (the XCD count) when there are enough tiles.
template <class Kern>
uint32_t persistent_grid(const Index &ix, Kern kern, int threads, size_t lds, uint64_t ntiles) {
    if (lds > 65536) raise_lds_limit((const void *)kern, lds);
    int per_cu = 0;
    PI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds));
    if (per_cu < 1)
        throw Error{PI_ERR_INVALID_ARG, "descent configuration cannot be resident (queries_per_lane x descent_block "
                                        "x lds_budget too large)"};
    if (ix.cfg.blocks_per_cu) per_cu = std::min<int>(per_cu, (int)ix.cfg.blocks_per_cu);
    uint64_t g = (uint64_t)ix.num_cus * (uint64_t)per_cu;
    if (g > ntiles) g = ntiles;
    if (g >= 8) g &= ~7ull;
    if (!g) g = 1;
    return (uint32_t)g;
}

}  // namespace
}  // namespace pi
