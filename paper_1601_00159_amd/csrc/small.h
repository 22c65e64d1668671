// One batch of at most SB_MAX queries processed by one workgroup (device
// function shared by the single-index small-batch launch and the many-index
// launch).
#pragma once

#include "descent.h"

namespace pi {

constexpr int SBT = 1024;                 // threads of the workgroup
constexpr int SBI = 4;                    // sorted queries per thread (blocked)
constexpr uint32_t SB_MAX = SBT * SBI;    // queries per workgroup batch
constexpr int SBW = SBT / 64;             // waves

// What the kernels need of one index: plain device pointers and its level
// descriptor (with the workgroup's own choice of LDS-staged levels).
struct IndexView {
    IndexDesc desc;
    const uint64_t *lkey;
    const uint32_t *ldown;
    uint64_t *skey;
    uint64_t *sval;
    uint32_t *snext;
    uint8_t *smeta;
    DevState *st;
    uint64_t cap;  // storage capacity: new nodes never go past it
    unsigned long long *owner;  // writer-check shadow (null: check off)
};

struct BatchView {
    const uint8_t *ops;
    const uint64_t *keys;
    const uint64_t *vals;
    uint32_t n;
    uint64_t *out_vals;
    uint8_t *out_status;
    uint32_t unit;  // writer-check unit of the first workgroup chunk
    uint32_t first; // 1: the first chunk of its batch (counts the batch, restarts its writer flag)
};

// Index entries of the upper levels a workgroup stages in LDS next to its
// batch (about 72 KB).
constexpr uint32_t SB_LDS_LEVEL_ENTRIES = 6000;

inline IndexView index_view(const Index &ix) {
    IndexView v;
    v.desc = ix.desc;
    // the top levels that fit the workgroup's spare LDS
    v.desc.lds_from = v.desc.top + 1;
    v.desc.lds_entries = 0;
    uint32_t used = 0;
    for (int l = v.desc.top; l >= 2; l--) {
        const uint32_t e = v.desc.n[l] + 1 + LEVEL_PAD;
        if (used + e > SB_LDS_LEVEL_ENTRIES) break;
        v.desc.lds_off[l] = used;
        used += e;
        v.desc.lds_from = l;
    }
    v.desc.lds_entries = used;
    v.lkey = ix.arena_key.as<uint64_t>();
    v.ldown = ix.arena_down.as<uint32_t>();
    v.skey = ix.st.key.as<uint64_t>();
    v.sval = ix.st.val.as<uint64_t>();
    v.snext = ix.st.next.as<uint32_t>();
    v.smeta = ix.st.meta.as<uint8_t>();
    v.st = ix.dstate;
    v.cap = ix.st.cap;
    v.owner = nullptr;
    return v;
}

// LDS layout of block_batch (dynamic shared memory).
struct SmallLds {
    static constexpr uint32_t key_off = 0;                        // u64 [SB_MAX] sorted keys
    static constexpr uint32_t idx_off = key_off + SB_MAX * 8;     // u32 [SB_MAX] arrival positions
    static constexpr uint32_t pred_off = idx_off + SB_MAX * 4;    // u32 [SB_MAX] new node: predecessor
    static constexpr uint32_t pnext_off = pred_off + SB_MAX * 4;  // u32 [SB_MAX] new node: old successor
    static constexpr uint32_t misc_off = pnext_off + SB_MAX * 4;  // scan scratch, counters
    static constexpr uint32_t misc_bytes = 1024;
    static constexpr uint32_t levels_off = misc_off + misc_bytes;  // staged levels: u64 keys, then u32 downs
    static constexpr uint32_t bytes() { return levels_off + SB_LDS_LEVEL_ENTRIES * 12; }
};

// Segmented "last writer" element: f = a key group starts here, v = sorted
// position of the last INSERT/DELETE so far (-1 none).
struct SSeg {
    uint32_t f;
    int32_t v;
};

__device__ __forceinline__ SSeg sseg_op(SSeg a, SSeg b) {
    SSeg r;
    r.f = a.f | b.f;
    r.v = b.f ? b.v : (a.v > b.v ? a.v : b.v);
    return r;
}

// exclusive scan of one SSeg per thread over the workgroup
__device__ __forceinline__ SSeg block_scan_sseg(SSeg x, SSeg *s_w) {
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    SSeg inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        SSeg y;
        y.f = __shfl_up(inc.f, o, 64);
        y.v = __shfl_up(inc.v, o, 64);
        if (lane >= o) inc = sseg_op(y, inc);
    }
    SSeg ex;
    ex.f = __shfl_up(inc.f, 1, 64);
    ex.v = __shfl_up(inc.v, 1, 64);
    if (lane == 0) ex = SSeg{0, -1};
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    SSeg pre{0, -1};
    for (int i = 0; i < w; i++) pre = sseg_op(pre, s_w[i]);
    __syncthreads();
    return sseg_op(pre, ex);
}

// exclusive scan of one u32 per thread over the workgroup; *total = sum
__device__ __forceinline__ uint32_t block_scan_u32(uint32_t x, uint32_t *s_w, uint32_t *total) {
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan_u32(x);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int i = 0; i < SBW; i++) {
        if (i < w) pre += s_w[i];
        tot += s_w[i];
    }
    __syncthreads();
    *total = tot;
    return pre + inc - x;
}

// Runs one batch (b.n <= SB_MAX) against one index; the calling workgroup
// must be the index's only user while it runs.
__device__ __forceinline__ void block_batch(const IndexView &v, const BatchView &b, uint64_t *s_raw) {
    uint8_t *lds = reinterpret_cast<uint8_t *>(s_raw);
    uint64_t *s_key = reinterpret_cast<uint64_t *>(lds + SmallLds::key_off);
    uint32_t *s_idx = reinterpret_cast<uint32_t *>(lds + SmallLds::idx_off);
    uint32_t *s_pred = reinterpret_cast<uint32_t *>(lds + SmallLds::pred_off);
    uint32_t *s_pnext = reinterpret_cast<uint32_t *>(lds + SmallLds::pnext_off);
    SSeg *s_seg = reinterpret_cast<SSeg *>(lds + SmallLds::misc_off);                  // SBW entries
    uint32_t *s_u = reinterpret_cast<uint32_t *>(lds + SmallLds::misc_off + 256);      // SBW entries
    unsigned int *s_cnt = reinterpret_cast<unsigned int *>(lds + SmallLds::misc_off + 512);  // counters
    const uint32_t n = b.n;
    const uint32_t tid = threadIdx.x;
    const WriterCheck wc{v.owner, b.unit};

    // ---- order: bitonic sort of (key, position) over the next power of two
    uint32_t m = 64;
    while (m < n) m <<= 1;
    if (tid < 8) s_cnt[tid] = 0;
    for (uint32_t i = tid; i < m; i += SBT) {
        uint64_t k = KEY_MAX;
        if (i < n) {
            k = b.keys[i];
            if (b.ops[i] > PI_OP_DELETE) k = KEY_MAX;
        }
        s_key[i] = k;
        s_idx[i] = i;
    }
    __syncthreads();
    for (uint32_t k = 2; k <= m; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = tid; i < m; i += SBT) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint64_t ki = s_key[i], kl = s_key[l];
                    const uint32_t ii = s_idx[i], il = s_idx[l];
                    const bool gt = ki > kl || (ki == kl && ii > il);
                    const bool up = (i & k) == 0;
                    if (gt == up) {
                        s_key[i] = kl;
                        s_key[l] = ki;
                        s_idx[i] = il;
                        s_idx[l] = ii;
                    }
                }
            }
            __syncthreads();
        }
    }

    // ---- descend: per = ceil(n / SBT) consecutive sorted queries per thread,
    // two chains in flight at a time, upper levels from an LDS copy
    uint64_t *s_lk = reinterpret_cast<uint64_t *>(lds + SmallLds::levels_off);
    uint32_t *s_ld = reinterpret_cast<uint32_t *>(s_lk + v.desc.lds_entries);
    stage_levels(v.desc, v.lkey, v.ldown, s_lk, s_ld);
    const bool links = v.st->has_links != 0;
    const bool dead = v.st->has_dead != 0;
    const uint32_t per = (n + SBT - 1) / SBT;  // 1 .. SBI
    const uint32_t i0 = tid * per;
    uint64_t q[SBI];
    Found f[SBI];
#pragma unroll
    for (int e = 0; e < SBI; e++) {
        q[e] = ((uint32_t)e < per && i0 + e < n) ? s_key[i0 + e] : KEY_MAX;
        f[e] = Found{HEAD_SLOT, 0, false, false, 0};
    }
#pragma unroll
    for (int h = 0; h < SBI; h += 2) {
        if ((uint32_t)h >= per) break;  // uniform: per is the same for every thread
        uint64_t qd[2] = {q[h] == KEY_MAX ? KEY_MAX - 1 : q[h], q[h + 1] == KEY_MAX ? KEY_MAX - 1 : q[h + 1]};
        uint32_t pos[2];
        uint64_t ik[2];
        descend_index<2>(qd, v.desc, v.lkey, v.ldown, s_lk, s_ld, pos, ik);
#pragma unroll
        for (int j = 0; j < 2; j++)
            if (q[h + j] != KEY_MAX)
                f[h + j] = walk_storage(q[h + j], pos[j], ik[j], links, dead, v.skey, v.sval, v.snext, v.smeta,
                                        &v.st->errors);
    }

    // ---- ownership: the segmented last-writer scan
    uint8_t op[SBI];
    SSeg el[SBI];
    SSeg run{0, -1};
#pragma unroll
    for (int e = 0; e < SBI; e++) {
        const uint32_t i = i0 + e;
        const bool mine = (uint32_t)e < per && i < n;
        op[e] = (mine && q[e] != KEY_MAX) ? b.ops[s_idx[i]] : (uint8_t)255;
        el[e].f = (mine && (i == 0 || s_key[i - 1] != q[e])) ? 1u : 0u;
        const bool w = op[e] == PI_OP_INSERT || op[e] == PI_OP_DELETE;
        if (w) s_cnt[4] = 1;  // the batch has writers (same value from every writer)
        el[e].v = w ? (int32_t)i : -1;
        run = sseg_op(run, el[e]);
    }
    SSeg pre = block_scan_sseg(run, s_seg);
    uint32_t hits = 0, invalid = 0, dels = 0, revs = 0;
    uint32_t newf[SBI];
    uint64_t newv[SBI];
#pragma unroll
    for (int e = 0; e < SBI; e++) {
        const uint32_t i = i0 + e;
        newf[e] = 0;
        newv[e] = 0;
        const int32_t excl = el[e].f ? -1 : pre.v;
        pre = sseg_op(pre, el[e]);
        const int32_t incl = pre.v;
        if ((uint32_t)e >= per || i >= n) continue;
        const uint32_t id = s_idx[i];
        if (q[e] == KEY_MAX) {
            b.out_vals[id] = 0;
            b.out_status[id] = PI_R_INVALID;
            invalid++;
            continue;
        }
        uint64_t val;
        bool present;
        if (excl >= 0) {
            const uint32_t jd = s_idx[excl];
            present = b.ops[jd] == PI_OP_INSERT;
            val = present ? b.vals[jd] : 0;
        } else {
            present = f[e].live;
            val = f[e].val;
        }
        b.out_vals[id] = val;
        b.out_status[id] = present ? PI_R_PRESENT : PI_R_ABSENT;
        hits += present;
        const bool last = (i + 1 == n) || s_key[i + 1] != q[e];
        if (last && incl >= 0) {
            const uint32_t jd = s_idx[incl];
            const uint32_t node = f[e].node;
            if (b.ops[jd] == PI_OP_INSERT) {
                if (f[e].exists) {
                    wc.note(node, WriterCheck::APPLY, i, &v.st->errors);
                    v.sval[node] = b.vals[jd];
                    if (!f[e].live) {
                        v.smeta[node] = v.smeta[node] & (uint8_t)~META_DEL;
                        revs++;
                    }
                } else {
                    newf[e] = 1;
                    newv[e] = b.vals[jd];
                }
            } else if (f[e].exists && f[e].live) {
                wc.note(node, WriterCheck::APPLY, i, &v.st->errors);
                v.smeta[node] = v.smeta[node] | META_DEL;
                dels++;
            }
        }
    }

    // ---- new nodes: slots by a block-wide prefix sum, then linking
    uint32_t mynew = 0;
#pragma unroll
    for (int e = 0; e < SBI; e++) mynew += newf[e];
    uint32_t nnew = 0;
    uint32_t r = block_scan_u32(mynew, s_u, &nnew);
    const uint64_t base = v.st->nused;
    // the host reserves room before the launch; should that ever fail, the
    // new nodes are dropped rather than written past the capacity
    const bool room = base + nnew <= v.cap;
    if (!room) nnew = 0;
    if (nnew) {
#pragma unroll
        for (int e = 0; e < SBI; e++) {
            if (!newf[e]) continue;
            const uint64_t slot = base + r;
            wc.note((uint32_t)slot, WriterCheck::LINK, r, &v.st->errors);
            v.skey[slot] = q[e];
            v.sval[slot] = newv[e];
            v.smeta[slot] = META_LINK;
            s_pred[r] = f[e].node;
            s_pnext[r] = f[e].next;
            r++;
        }
    }
    __syncthreads();  // node writes of the apply step and the new-node table
    for (uint32_t k = tid; k < nnew; k += SBT) {
        const uint32_t slot = (uint32_t)(base + k);
        const uint32_t pr = s_pred[k];
        v.snext[slot] = (k + 1 < nnew && s_pred[k + 1] == pr) ? slot + 1 : s_pnext[k];
        if (k == 0 || s_pred[k - 1] != pr) {
            wc.note(pr, WriterCheck::LINK, k, &v.st->errors);
            v.snext[pr] = slot;
            v.smeta[pr] = v.smeta[pr] | META_LINK;
        }
    }

    // ---- counters (this workgroup is the index's only writer)
    hits = wave_sum_u32(hits);
    invalid = wave_sum_u32(invalid);
    dels = wave_sum_u32(dels);
    revs = wave_sum_u32(revs);
    if (lane_id() == 0) {
        if (hits) atomicAdd(&s_cnt[0], hits);
        if (invalid) atomicAdd(&s_cnt[1], invalid);
        if (dels) atomicAdd(&s_cnt[2], dels);
        if (revs) atomicAdd(&s_cnt[3], revs);
    }
    __syncthreads();
    if (tid == 0) {
        DevState *st = v.st;
        if (!room) st->errors |= ERR_CAPACITY;
        const unsigned int d = s_cnt[2], rv = s_cnt[3];
        st->nused += nnew;
        st->n_live = st->n_live + nnew + rv - d;
        st->changes += nnew + d;
        if (nnew) st->has_links = 1;
        if (d) st->has_dead = 1;
        if (b.first) {
            st->b_writers = s_cnt[4];
            st->batches += 1;
        } else {
            st->b_writers |= s_cnt[4];
        }
        st->queries += n;
        st->hits += s_cnt[0];
        st->invalid += s_cnt[1];
        st->new_nodes += nnew;
        st->deletes += d;
        st->revives += rv;
    }
    __syncthreads();
}

}  // namespace pi
