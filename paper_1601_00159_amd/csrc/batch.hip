// One batch of queries (Algorithm 1) on gfx950.
//
//   order      stable radix sort of the batch by key (Definition 3); invalid
//              queries sort last with key +infinity
//   descend    k_descend: every query walks the index layer from the top
//              level down (Algorithm 2), level by level for the whole wave
//              (group processing, Section 4.3.4), the upper levels read from
//              an LDS copy, to its interception (Definition 4), then along the
//              storage list to the node with the largest key <= its key
//              (getNode of Algorithm 4).  For a batch without updates this
//              kernel writes the final answers.
//   ownership  queries with equal keys are adjacent and in arrival order; a
//              segmented scan over the sorted batch gives each query the last
//              INSERT/DELETE before it on the same key, hence its answer, and
//              gives each key group one owner -- the group's last query --
//              which alone writes that key's node.  This replaces the
//              message-based hand-over of Algorithm 3: after it, no storage
//              node has two writers (the invariant of Section 3.2.4).
//   apply      owners update values and delete flags in place (Algorithm 4
//              flags instead of unlinking); keys that end the batch live but
//              have no node get one in a key-sorted run appended to the
//              storage; new nodes sharing a predecessor are chained and only
//              the first writes the predecessor's successor.  No atomics, no
//              latches.
//   rebuild    the index layer is not touched by updates; it is rebuilt from
//              the storage layer when enough changes accumulate (Section 4.1,
//              Section 4.3.5), by the host between batches.
#include <algorithm>

#include "descent.h"

namespace pi {
namespace {

constexpr int OT = 256;          // ownership block
constexpr int OI = 4;            // items per thread (blocked)
constexpr int OTILE = OT * OI;
constexpr int ONW = OT / 64;

// MODE 0: sorted batch.  MODE 1: interception of arbitrary keys (inspection).
// Each block of DT threads owns a contiguous range of tiles of DT*QPL sorted
// queries; a lane carries QPL queries of a tile (rows of DT) through the
// descent together.  All waves of the block share one LDS copy of the upper
// levels.
// Sorts the wave's 64 (key, index) pairs by (key, index) across the lanes
// (bitonic network over lane pairs).  A batch without INSERT/DELETE is
// ordered only to 1/65536 of its key span: the queries of one wave come from
// one or two such groups in arrival order, and this puts them back in key
// order, which the descent's shared and per-lane windows rely on for
// locality.  Past-the-end lanes hold +infinity and stay last.
__device__ __forceinline__ void wave_sort_kv(uint64_t &k, uint32_t &v) {
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const uint64_t pk = shfl_xor_u64(k, stride);
            const uint32_t pv = (uint32_t)__shfl_xor((int)v, stride, 64);
            const bool up = (lane & size) == 0;        // this block ascends
            const bool low = (lane & stride) == 0;     // the lower lane of the pair
            const bool pless = pk < k || (pk == k && pv < v);
            if (low == up ? pless : !pless) {          // keep the min below in an ascending block
                k = pk;
                v = pv;
            }
        }
    }
}

template <int MODE, int QPL, int DT>
__global__ __launch_bounds__(DT) void k_descend(IndexDesc desc, const uint64_t *__restrict__ lkey,
                                                const uint32_t *__restrict__ ldown, const uint64_t *__restrict__ skey,
                                                const uint64_t *__restrict__ sval, const uint32_t *__restrict__ snext,
                                                const uint8_t *__restrict__ smeta, const uint64_t *__restrict__ sk,
                                                const uint32_t *__restrict__ sidx, uint32_t n, DevState *st,
                                                uint2 *__restrict__ dpart, const unsigned int *__restrict__ wflag,
                                                uint32_t wsort,
                                                uint64_t *__restrict__ out_vals, uint8_t *__restrict__ out_status,
                                                uint64_t *__restrict__ res_val, uint8_t *__restrict__ res_flags,
                                                uint32_t *__restrict__ loc, uint32_t *__restrict__ locnext,
                                                const uint8_t *__restrict__ ops, const uint64_t *__restrict__ vals,
                                                uint8_t *__restrict__ sop, uint64_t *__restrict__ svin) {
    extern __shared__ uint64_t s_dyn[];
    uint64_t *s_k = s_dyn;
    uint32_t *s_d = reinterpret_cast<uint32_t *>(s_dyn + desc.lds_entries);
    stage_levels(desc, lkey, ldown, s_k, s_d);

    // the batch's counters start here (the ordering before this kernel
    // touches nothing of the index): the later steps read and add to them
    const unsigned int writers = MODE == 0 && n ? *wflag : 0u;  // an empty batch has no ordering step
    if (MODE == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        st->b_writers = writers;
        st->b_new = st->b_deletes = st->b_revives = st->b_hits = st->b_invalid = 0;
        st->b_n = n;
        st->bar = st->join = 0;
        st->parts = st->tile_next = 0;
    }
    const bool mixed = writers != 0;
    const bool links = MODE == 0 && st->has_links != 0;
    const bool dead = MODE == 0 && st->has_dead != 0;

    constexpr uint32_t TQ = DT * QPL;
    const uint32_t ntiles = (n + TQ - 1) / TQ;
    const uint32_t c = xcd_chunk(blockIdx.x, gridDim.x);
    const uint32_t t0 = (uint32_t)((uint64_t)c * ntiles / gridDim.x);
    const uint32_t t1 = (uint32_t)((uint64_t)(c + 1) * ntiles / gridDim.x);
    uint32_t hits = 0, invalid = 0;
    for (uint32_t t = t0; t < t1; t++) {
        uint64_t q[QPL];
        uint32_t idx[QPL];
#pragma unroll
        for (int j = 0; j < QPL; j++) {
            idx[j] = t * TQ + j * DT + threadIdx.x;
            // past the end or invalid: descend as the largest valid key (stays
            // inside the pads), answer nothing
            q[j] = idx[j] < n ? sk[idx[j]] : KEY_MAX;
        }
        if (QPL == 1 && MODE == 0 && wsort && !mixed) wave_sort_kv(q[0], idx[0]);
        uint64_t qd[QPL];
#pragma unroll
        for (int j = 0; j < QPL; j++) qd[j] = q[j] == KEY_MAX ? KEY_MAX - 1 : q[j];
        uint32_t pos[QPL];
        uint64_t ik[QPL];
        descend_index<QPL>(qd, desc, lkey, ldown, s_k, s_d, pos, ik);
#pragma unroll
        for (int j = 0; j < QPL; j++) {
            const uint32_t i = idx[j];
            if (i >= n) continue;
            if (MODE == 1) {
                out_vals[i] = pos[j] == HEAD_SLOT ? 0 : ik[j];
                out_status[i] = pos[j] == HEAD_SLOT ? 1 : 0;
                continue;
            }
            const uint32_t id = sidx[i];
            if (q[j] == KEY_MAX) {
                out_vals[id] = 0;
                out_status[id] = PI_R_INVALID;
                invalid++;
                if (mixed) sop[i] = 255;
                continue;
            }
            const Found f = walk_storage(q[j], pos[j], ik[j], links, dead, skey, sval, snext, smeta, &st->errors);
            if (!mixed) {
                out_vals[id] = f.val;
                out_status[id] = f.live ? PI_R_PRESENT : PI_R_ABSENT;
                hits += f.live;
            } else {
                res_val[i] = f.val;
                res_flags[i] = (uint8_t)((f.exists ? 1 : 0) | (f.live ? 2 : 0));
                loc[i] = f.node;
                locnext[i] = f.next;
                // the op and the inserted value in sorted order, for the
                // ownership kernels (one gather here instead of several there)
                const uint8_t o = ops[id];
                sop[i] = o;
                svin[i] = o == PI_OP_INSERT ? vals[id] : 0;
            }
        }
    }
    if (MODE == 0) {
        // the block's counts go to its own slot (summed at the batch's end),
        // not to shared counters
        __shared__ uint2 s_cnt[DT / 64];
        hits = wave_sum_u32(hits);
        invalid = wave_sum_u32(invalid);
        if (lane_id() == 0) s_cnt[threadIdx.x >> 6] = make_uint2(hits, invalid);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint2 c = make_uint2(0, 0);
            for (int w = 0; w < DT / 64; w++) {
                c.x += s_cnt[w].x;
                c.y += s_cnt[w].y;
            }
            dpart[blockIdx.x] = c;
        }
    }
}

// -------------------------------------------------------------- ownership --

// Segmented "last writer" scan element: f = a key group starts here,
// v = sorted index of the last INSERT/DELETE seen (-1 none).
struct Seg {
    uint32_t f;
    int32_t v;
};

__device__ __forceinline__ Seg seg_op(Seg a, Seg b) {
    Seg r;
    r.f = a.f | b.f;
    r.v = b.f ? b.v : (a.v > b.v ? a.v : b.v);
    return r;
}

__device__ __forceinline__ Seg wave_incl_scan_seg(Seg x) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        Seg y;
        y.f = __shfl_up(x.f, o, 64);
        y.v = __shfl_up(x.v, o, 64);
        if (lane >= o) x = seg_op(y, x);
    }
    return x;
}

// exclusive block scan of one Seg per thread; also returns the block total
__device__ __forceinline__ Seg block_excl_scan_seg(Seg x, Seg *s_w, Seg *total) {
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const Seg inc = wave_incl_scan_seg(x);
    Seg ex;
    ex.f = __shfl_up(inc.f, 1, 64);
    ex.v = __shfl_up(inc.v, 1, 64);
    if (lane_id() == 0) {
        ex.f = 0;
        ex.v = -1;
    }
    if (lane_id() == 63) s_w[w] = inc;
    __syncthreads();
    Seg pre{0, -1};
    for (int i = 0; i < w; i++) pre = seg_op(pre, s_w[i]);
    Seg tot{0, -1};
    for (int i = 0; i < ONW; i++) tot = seg_op(tot, s_w[i]);
    *total = tot;
    __syncthreads();
    return seg_op(pre, ex);
}

__device__ __forceinline__ Seg element(const uint64_t *__restrict__ sk, const uint8_t *__restrict__ sop, uint32_t i,
                                       uint64_t q) {
    Seg e;
    e.f = (i == 0 || sk[i - 1] != q) ? 1u : 0u;
    const uint8_t op = sop[i];
    e.v = (q != KEY_MAX && (op == PI_OP_INSERT || op == PI_OP_DELETE)) ? (int32_t)i : -1;
    return e;
}

// A thread's OI consecutive sorted queries from base (a multiple of OI):
// their keys and ops, read with 16- and 4-byte loads when all OI are inside
// the batch, plus the key before the run (group start) and whether a key
// follows it (group end).  Past n: key +infinity, no op.
struct Run {
    uint64_t k[OI];
    uint8_t op[OI];
    uint64_t prev, next;
    bool has_next;
};

__device__ __forceinline__ Run load_run(const uint64_t *__restrict__ sk, const uint8_t *__restrict__ sop,
                                        uint32_t n, uint32_t base) {
    static_assert(OI == 4, "two key pairs and one op word per run");
    Run r;
    if (base + OI <= n) {
        const ulonglong2 a = *reinterpret_cast<const ulonglong2 *>(sk + base);
        const ulonglong2 b = *reinterpret_cast<const ulonglong2 *>(sk + base + 2);
        r.k[0] = a.x, r.k[1] = a.y, r.k[2] = b.x, r.k[3] = b.y;
        const uint32_t o4 = *reinterpret_cast<const uint32_t *>(sop + base);
#pragma unroll
        for (int e = 0; e < OI; e++) r.op[e] = (uint8_t)(o4 >> (8 * e));
    } else {
#pragma unroll
        for (int e = 0; e < OI; e++) {
            const uint32_t i = base + e;
            r.k[e] = i < n ? sk[i] : KEY_MAX;
            r.op[e] = i < n ? sop[i] : (uint8_t)255;
        }
    }
    r.prev = base > 0 && base <= n ? sk[base - 1] : 0;
    r.has_next = base + OI < n;
    r.next = r.has_next ? sk[base + OI] : KEY_MAX;
    return r;
}

// element e of a run (see element above)
__device__ __forceinline__ Seg run_element(const Run &r, uint32_t base, int e) {
    Seg x;
    const uint64_t q = r.k[e];
    const uint64_t before = e == 0 ? r.prev : r.k[e > 0 ? e - 1 : 0];
    x.f = (base + e == 0 || before != q) ? 1u : 0u;
    const uint8_t op = r.op[e];
    x.v = (q != KEY_MAX && (op == PI_OP_INSERT || op == PI_OP_DELETE)) ? (int32_t)(base + e) : -1;
    return x;
}

// tile t (OTILE sorted queries): aggregate of its segmented scan elements
__device__ __forceinline__ void own_reduce_tile(uint32_t t, const uint64_t *__restrict__ sk,
                                                const uint8_t *__restrict__ sop, uint32_t n, Seg *__restrict__ agg,
                                                Seg *s_w) {
    const uint32_t base = t * OTILE + threadIdx.x * OI;
    const Run r = load_run(sk, sop, n, base);
    Seg run{0, -1};
#pragma unroll
    for (int e = 0; e < OI; e++)
        if (base + e < n) run = seg_op(run, run_element(r, base, e));
    Seg tot;
    block_excl_scan_seg(run, s_w, &tot);
    if (threadIdx.x == 0) agg[t] = tot;
}

__global__ __launch_bounds__(OT) void k_own_reduce(const uint64_t *__restrict__ sk, const uint8_t *__restrict__ sop,
                                                   uint32_t n, const DevState *st, Seg *__restrict__ agg) {
    if (st->b_writers == 0) return;
    __shared__ Seg s_w[ONW];
    own_reduce_tile(blockIdx.x, sk, sop, n, agg, s_w);
}

// one block: exclusive scan of the tile aggregates (in place)
__device__ __forceinline__ void own_prefix_block(Seg *__restrict__ agg, uint32_t ntiles, Seg *s_w) {
    Seg carry{0, -1};
    for (uint32_t base = 0; base < ntiles; base += OT * 4) {
        Seg v[4];
        Seg run{0, -1};
        for (int j = 0; j < 4; j++) {
            const uint32_t i = base + threadIdx.x * 4 + j;
            v[j] = i < ntiles ? agg[i] : Seg{0, -1};
            run = seg_op(run, v[j]);
        }
        Seg tot;
        Seg pre = seg_op(carry, block_excl_scan_seg(run, s_w, &tot));
        for (int j = 0; j < 4; j++) {
            const uint32_t i = base + threadIdx.x * 4 + j;
            if (i < ntiles) agg[i] = pre;
            pre = seg_op(pre, v[j]);
        }
        carry = seg_op(carry, tot);
    }
}

__global__ __launch_bounds__(OT) void k_own_prefix(Seg *__restrict__ agg, uint32_t ntiles, const DevState *st) {
    if (st->b_writers == 0) return;
    __shared__ Seg s_w[ONW];
    own_prefix_block(agg, ntiles, s_w);
}

__device__ __forceinline__ void own_apply_tile(uint32_t t, const uint64_t *__restrict__ sk, const uint32_t *__restrict__ sidx,
                                                  const uint8_t *__restrict__ sop, const uint64_t *__restrict__ svin,
                                                  uint32_t n, const Seg *__restrict__ carry_in,
                                                  const uint64_t *__restrict__ res_val,
                                                  const uint8_t *__restrict__ res_flags,
                                                  const uint32_t *__restrict__ loc, uint64_t *__restrict__ sval,
                                                  uint8_t *__restrict__ smeta, uint64_t *__restrict__ out_vals,
                                                  uint8_t *__restrict__ out_status, uint32_t *__restrict__ newflag,
                                                  int32_t *__restrict__ gw, uint4 *__restrict__ part,
                                                  DevState *st, WriterCheck wc, uint32_t *__restrict__ tilecnt, Seg *s_w) {
    const uint32_t base = t * OTILE + threadIdx.x * OI;
    const Run r = load_run(sk, sop, n, base);
    const bool whole = base + OI <= n;
    Seg el[OI];
    Seg run{0, -1};
#pragma unroll
    for (int e = 0; e < OI; e++) {
        el[e] = base + e < n ? run_element(r, base, e) : Seg{0, -1};
        run = seg_op(run, el[e]);
    }
    // the per-query state of the descent, four at a time when whole
    uint32_t id4[OI], loc4[OI];
    uint8_t fl4[OI];
    uint64_t rv4[OI];
    if (whole) {
        const uint4 a = *reinterpret_cast<const uint4 *>(sidx + base);
        const uint4 l = *reinterpret_cast<const uint4 *>(loc + base);
        const uint32_t f = *reinterpret_cast<const uint32_t *>(res_flags + base);
        const ulonglong2 v0 = *reinterpret_cast<const ulonglong2 *>(res_val + base);
        const ulonglong2 v1 = *reinterpret_cast<const ulonglong2 *>(res_val + base + 2);
        id4[0] = a.x, id4[1] = a.y, id4[2] = a.z, id4[3] = a.w;
        loc4[0] = l.x, loc4[1] = l.y, loc4[2] = l.z, loc4[3] = l.w;
#pragma unroll
        for (int e = 0; e < OI; e++) fl4[e] = (uint8_t)(f >> (8 * e));
        rv4[0] = v0.x, rv4[1] = v0.y, rv4[2] = v1.x, rv4[3] = v1.y;
    } else {
#pragma unroll
        for (int e = 0; e < OI; e++) {
            const uint32_t i = base + e;
            id4[e] = i < n ? sidx[i] : 0;
            loc4[e] = i < n ? loc[i] : 0;
            fl4[e] = i < n ? res_flags[i] : 0;
            rv4[e] = i < n ? res_val[i] : 0;
        }
    }
    Seg tot;
    Seg pre = seg_op(carry_in[t], block_excl_scan_seg(run, s_w, &tot));
    uint32_t hits = 0, dels = 0, revs = 0;
    uint32_t nf4[OI] = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < OI; e++) {
        const uint32_t i = base + e;
        if (i >= n) break;
        const int32_t excl = el[e].f ? -1 : pre.v;
        pre = seg_op(pre, el[e]);
        const int32_t incl = pre.v;
        const uint64_t q = r.k[e];
        if (q == KEY_MAX) continue;  // invalid: answered by the descent, no effect
        const uint32_t id = id4[e];
        const uint8_t fl = fl4[e];
        // answer: the state left by the last update before i on this key,
        // else the state found in storage
        uint64_t v;
        bool present;
        if (excl >= 0) {
            present = sop[excl] == PI_OP_INSERT;
            v = present ? svin[excl] : 0;
        } else {
            present = (fl & 2) != 0;
            v = rv4[e];
        }
        out_vals[id] = v;
        out_status[id] = present ? PI_R_PRESENT : PI_R_ABSENT;
        hits += present;
        // the group's last query owns the key's node
        const bool last = e + 1 < OI ? r.k[e + 1 < OI ? e + 1 : 0] != q : (!r.has_next || r.next != q);
        uint32_t nf = 0;
        if (last && incl >= 0) {
            const uint32_t node = loc4[e];
            const bool exists = fl & 1, live = (fl & 2) != 0;
            if (sop[incl] == PI_OP_INSERT) {
                if (exists) {
                    wc.note(node, WriterCheck::APPLY, i, &st->errors);
                    sval[node] = svin[incl];
                    if (!live) {
                        smeta[node] = smeta[node] & (uint8_t)~META_DEL;
                        revs++;
                    }
                } else {
                    nf = 1;
                    gw[i] = incl;
                }
            } else if (exists && live) {
                wc.note(node, WriterCheck::APPLY, i, &st->errors);
                smeta[node] = smeta[node] | META_DEL;
                dels++;
            }
        }
        nf4[e] = nf;
    }
    if (whole) {
        *reinterpret_cast<uint4 *>(newflag + base) = make_uint4(nf4[0], nf4[1], nf4[2], nf4[3]);
    } else {
#pragma unroll
        for (int e = 0; e < OI; e++)
            if (base + e < n) newflag[base + e] = nf4[e];
    }
    // the tile's counts go to its own slot; the batch's end sums them (one
    // atomic per wave on three shared counters cost more than the apply)
    uint32_t nnew = nf4[0] + nf4[1] + nf4[2] + nf4[3];
    hits = wave_sum_u32(hits);
    dels = wave_sum_u32(dels);
    revs = wave_sum_u32(revs);
    nnew = wave_sum_u32(nnew);
    __shared__ uint32_t s_c[4][ONW];
    if (lane_id() == 0) {
        s_c[0][threadIdx.x >> 6] = hits;
        s_c[1][threadIdx.x >> 6] = dels;
        s_c[2][threadIdx.x >> 6] = revs;
        s_c[3][threadIdx.x >> 6] = nnew;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint4 c = make_uint4(0, 0, 0, 0);
        for (int w = 0; w < ONW; w++) {
            c.x += s_c[0][w];
            c.y += s_c[1][w];
            c.z += s_c[2][w];
            c.w += s_c[3][w];
        }
        part[t] = c;
        if (tilecnt) tilecnt[t] = c.w;
    }
    __syncthreads();  // s_c is reused by the block's next tile
}

// tile counts (hits, deletes, revives, new nodes) go to part[tile]
__global__ __launch_bounds__(OT) void k_own_apply(const uint64_t *__restrict__ sk, const uint32_t *__restrict__ sidx,
                                                  const uint8_t *__restrict__ sop, const uint64_t *__restrict__ svin,
                                                  uint32_t n, const Seg *__restrict__ carry_in,
                                                  const uint64_t *__restrict__ res_val,
                                                  const uint8_t *__restrict__ res_flags,
                                                  const uint32_t *__restrict__ loc, uint64_t *__restrict__ sval,
                                                  uint8_t *__restrict__ smeta, uint64_t *__restrict__ out_vals,
                                                  uint8_t *__restrict__ out_status, uint32_t *__restrict__ newflag,
                                                  int32_t *__restrict__ gw, uint4 *__restrict__ part,
                                                  DevState *st, WriterCheck wc) {
    if (st->b_writers == 0) return;
    __shared__ Seg s_w[ONW];
    own_apply_tile(blockIdx.x, sk, sidx, sop, svin, n, carry_in, res_val, res_flags, loc, sval, smeta, out_vals,
                   out_status, newflag, gw, part, st, wc, nullptr, s_w);
}

// compacts the new nodes (key order) with their predecessor
__global__ void k_new_gather(const uint64_t *__restrict__ sk, const uint64_t *__restrict__ svin,
                             const uint32_t *__restrict__ newflag,
                             const uint32_t *__restrict__ newpos, const int32_t *__restrict__ gw,
                             const uint32_t *__restrict__ loc, const uint32_t *__restrict__ locnext, uint32_t n,
                             const DevState *st, uint64_t *__restrict__ nk, uint64_t *__restrict__ nv,
                             uint32_t *__restrict__ npred, uint32_t *__restrict__ npnext) {
    if (st->b_writers == 0) return;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (!newflag[i]) continue;
        const uint32_t r = newpos[i];
        nk[r] = sk[i];
        nv[r] = svin[gw[i]];
        npred[r] = loc[i];
        npnext[r] = locnext[i];
    }
}

// writes new nodes r (grid-stride from r0 in steps of dr, r < nnew) to slots
// first + r and links them (Algorithm 4 insertNode): a run of new nodes
// sharing a predecessor is chained, and only its first node writes the
// predecessor's successor.  Each node has one writer; no atomics.
__device__ __forceinline__ void link_range(uint32_t r0, uint32_t dr, uint32_t first, uint32_t nnew,
                                           const uint64_t *__restrict__ nk, const uint64_t *__restrict__ nv,
                                           const uint32_t *__restrict__ npred, const uint32_t *__restrict__ npnext,
                                           uint64_t *__restrict__ skey, uint64_t *__restrict__ sval,
                                           uint32_t *__restrict__ snext, uint8_t *__restrict__ smeta,
                                           const WriterCheck &wc, unsigned int *errors) {
    for (uint32_t r = r0; r < nnew; r += dr) {
        const uint32_t slot = first + r;
        const uint32_t pr = npred[r];
        wc.note(slot, WriterCheck::LINK, r, errors);
        skey[slot] = nk[r];
        sval[slot] = nv[r];
        smeta[slot] = META_LINK;
        snext[slot] = (r + 1 < nnew && npred[r + 1] == pr) ? slot + 1 : npnext[r];
        if (r == 0 || npred[r - 1] != pr) {
            wc.note(pr, WriterCheck::LINK, r, errors);
            snext[pr] = slot;
            smeta[pr] = smeta[pr] | META_LINK;
        }
    }
}

// The host reserves room for every batch before it is enqueued; should that
// ever fail, nothing is written past the capacity: the batch's new nodes are
// dropped (k_batch_end flags ERR_CAPACITY, which fails the handle).
__global__ void k_link(const uint64_t *__restrict__ nk, const uint64_t *__restrict__ nv,
                       const uint32_t *__restrict__ npred, const uint32_t *__restrict__ npnext, DevState *st,
                       uint64_t cap, uint64_t *__restrict__ skey, uint64_t *__restrict__ sval,
                       uint32_t *__restrict__ snext, uint8_t *__restrict__ smeta, WriterCheck wc) {
    const uint32_t nnew = st->b_new;
    if (nnew == 0) return;
    if (st->nused + nnew > cap) return;
    link_range(blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, (uint32_t)st->nused, nnew, nk, nv,
               npred, npnext, skey, sval, snext, smeta, wc, &st->errors);
}

// Self-test of the writer check's detection (no storage involved): on a
// two-word shadow, one writer recording twice must pass and two writers of
// one node under one tag must be caught.  out[0], out[1]: error bits of each.
__global__ void k_writer_selftest(unsigned long long *shadow, unsigned int *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    shadow[0] = shadow[1] = 0;
    out[0] = out[1] = 0;
    const WriterCheck wc{shadow, 7};
    wc.note(0, WriterCheck::APPLY, 5, &out[0]);
    wc.note(0, WriterCheck::APPLY, 5, &out[0]);
    wc.note(0, WriterCheck::LINK, 9, &out[0]);  // another phase: no conflict
    wc.note(1, WriterCheck::APPLY, 5, &out[1]);
    wc.note(1, WriterCheck::APPLY, 6, &out[1]);
}

__global__ void k_batch_begin(DevState *st, uint32_t n) {
    if (threadIdx.x != 0) return;
    st->b_writers = st->b_new = st->b_deletes = st->b_revives = st->b_hits = st->b_invalid = 0;
    st->b_n = n;
    st->bar = st->join = st->parts = st->tile_next = 0;
}

// Sums the apply tiles' counts (batches with updates; one 256-thread block),
// then folds the batch into the cumulative counters.
__device__ __forceinline__ void batch_end_block(DevState *st, const uint4 *__restrict__ part, uint32_t ntiles,
                                                uint64_t cap, const uint2 *__restrict__ dpart, uint32_t dgrid) {
    __shared__ uint32_t s_c[3][4];
    __shared__ uint32_t s_d[2][4];
    {
        // the descent blocks' counts: hits of a batch without updates, and
        // invalid queries
        uint32_t h = 0, v = 0;
        for (uint32_t b = threadIdx.x; b < dgrid; b += 256) {
            const uint2 c = dpart[b];
            h += c.x;
            v += c.y;
        }
        h = wave_sum_u32(h);
        v = wave_sum_u32(v);
        if (lane_id() == 0) {
            s_d[0][threadIdx.x >> 6] = h;
            s_d[1][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < 4; w++) {
                st->b_hits += s_d[0][w];
                st->b_invalid += s_d[1][w];
            }
    }
    if (st->b_writers != 0) {
        uint32_t h = 0, d = 0, r = 0;
        for (uint32_t t = threadIdx.x; t < ntiles; t += 256) {
            const uint4 c = part[t];
            h += c.x;
            d += c.y;
            r += c.z;
        }
        h = wave_sum_u32(h);
        d = wave_sum_u32(d);
        r = wave_sum_u32(r);
        if (lane_id() == 0) {
            s_c[0][threadIdx.x >> 6] = h;
            s_c[1][threadIdx.x >> 6] = d;
            s_c[2][threadIdx.x >> 6] = r;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < 4; w++) {
                st->b_hits += s_c[0][w];
                st->b_deletes += s_c[1][w];
                st->b_revives += s_c[2][w];
            }
    }
    if (threadIdx.x != 0) return;
    unsigned int nn = st->b_new;
    if (st->nused + nn > cap) {  // the link step wrote nothing
        st->errors |= ERR_CAPACITY;
        nn = 0;
    }
    st->nused += nn;
    st->n_live = st->n_live + nn + st->b_revives - st->b_deletes;
    st->changes += nn + st->b_deletes;
    if (nn) st->has_links = 1;
    if (st->b_deletes) st->has_dead = 1;
    st->batches += 1;
    st->queries += st->b_n - st->b_pad;
    st->hits += st->b_hits;
    st->invalid += st->b_invalid - st->b_pad;
    st->b_pad = 0;
    st->new_nodes += nn;
    st->deletes += st->b_deletes;
    st->revives += st->b_revives;
}

__global__ __launch_bounds__(256) void k_batch_end(DevState *st, const uint4 *__restrict__ part, uint32_t ntiles,
                                                   uint64_t cap, const uint2 *__restrict__ dpart, uint32_t dgrid) {
    batch_end_block(st, part, ntiles, cap, dpart, dgrid);
}

// ---------------------------------------------- the fused post-descent step --

// Blocks of the fused step.  A block takes part if it starts before the
// first block reaches the first grid barrier: it joins by adding one to the
// join word, and the first arrival at that barrier closes the word (a bit
// set by atomicOr), which fixes the number of blocks taking part; that
// block publishes the number for the others.  Every block taking part is
// running by then, so every barrier completes whatever else shares the
// device; a block that starts later sees the closed bit and leaves at once.
// One atomic per block to join and one to close: no retry loop, whose cost
// grows with the square of the blocks starting together.  The first phase
// hands its tiles out by a counter, so the blocks that take part cover all
// of them; the later phases split the tiles by rank.
constexpr unsigned int JOIN_CLOSED = 1u << 31;
constexpr unsigned int PART_SET = 1u << 31;

// thread 0: this block's rank among the blocks taking part, or ~0u
__device__ __forceinline__ uint32_t grid_join(unsigned int *join) {
    const unsigned int c = atomicAdd(join, 1u);
    return (c & JOIN_CLOSED) ? ~0u : c;
}

// thread 0: the number of blocks taking part (closing the window if open)
__device__ uint32_t grid_close(unsigned int *join, unsigned int *parts, unsigned int *errors) {
    const unsigned int c = atomicOr(join, JOIN_CLOSED);
    if (!(c & JOIN_CLOSED)) {
        __hip_atomic_store(parts, PART_SET | c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return c;
    }
    // closed by another block, which publishes the count right after
    unsigned int p = __hip_atomic_load(parts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t spins = 0; !(p & PART_SET); spins++) {
        if (spins > (1u << 24)) {
            atomicOr(errors, ERR_BARRIER);
            return 1;
        }
        __builtin_amdgcn_s_sleep(1);
        p = __hip_atomic_load(parts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return p & ~PART_SET;
}

// Barrier of the P blocks taking part.  The spin is bounded anyway; running
// out flags ERR_BARRIER, which fails the handle.
__device__ __forceinline__ void grid_barrier(unsigned int *bar, unsigned int &round, uint32_t P,
                                             unsigned int *errors) {
    __syncthreads();
    round++;
    if (threadIdx.x == 0) {
        __threadfence();  // this block's writes before the arrival
        atomicAdd(bar, 1u);
        const unsigned int target = round * P;
        for (uint32_t spins = 0;
             __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; spins++) {
            if (spins > (1u << 24)) {
                atomicOr(errors, ERR_BARRIER);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();  // the other blocks' writes after it
    }
    __syncthreads();
}

// next tile of a phase for the whole block
__device__ __forceinline__ uint32_t next_tile(unsigned int *ctr, uint32_t *s_t) {
    __syncthreads();  // the block is done with the previous value
    if (threadIdx.x == 0) *s_t = atomicAdd(ctr, 1u);
    __syncthreads();
    return *s_t;
}

// The steps after the descent in one launch (tiles of OTILE sorted queries
// handed out by counters, grid barriers between the steps): the segmented
// last-writer scan (tile aggregates, their prefix), answers and in-place
// updates with per-tile new-node counts, the prefix of those counts (slots
// of the new nodes), the gather of new nodes in key order, their linking,
// and the counters.  A batch without INSERT/DELETE only folds its counters.
__global__ __launch_bounds__(OT) void k_post(const uint64_t *__restrict__ sk, const uint32_t *__restrict__ sidx,
                                             const uint8_t *__restrict__ sop, const uint64_t *__restrict__ svin,
                                             uint32_t n, const uint64_t *__restrict__ res_val,
                                             const uint8_t *__restrict__ res_flags, const uint32_t *__restrict__ loc,
                                             const uint32_t *__restrict__ locnext, uint64_t *__restrict__ skey,
                                             uint64_t *__restrict__ sval, uint32_t *__restrict__ snext,
                                             uint8_t *__restrict__ smeta, uint64_t cap,
                                             uint64_t *__restrict__ out_vals, uint8_t *__restrict__ out_status,
                                             Seg *__restrict__ agg, uint4 *__restrict__ part,
                                             uint32_t *__restrict__ tilecnt, uint32_t *__restrict__ newflag,
                                             int32_t *__restrict__ gw, uint64_t *__restrict__ nk,
                                             uint64_t *__restrict__ nv, uint32_t *__restrict__ npred,
                                             uint32_t *__restrict__ npnext, DevState *st, WriterCheck wc,
                                             const uint2 *__restrict__ dpart, uint32_t dgrid) {
    const uint32_t ntiles = (n + OTILE - 1) / OTILE;
    if (st->b_writers == 0) {
        if (blockIdx.x == 0) batch_end_block(st, part, 0, cap, dpart, dgrid);
        return;
    }
    __shared__ Seg s_w[ONW];
    __shared__ uint32_t s_u[ONW + 1];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) s_t = grid_join(&st->join);
    __syncthreads();
    const uint32_t rank = s_t;
    if (rank == ~0u) return;  // started after the window closed
    unsigned int round = 0;
    for (uint32_t t = next_tile(&st->tile_next, &s_t); t < ntiles; t = next_tile(&st->tile_next, &s_t))
        own_reduce_tile(t, sk, sop, n, agg, s_w);
    __syncthreads();
    if (threadIdx.x == 0) s_t = grid_close(&st->join, &st->parts, &st->errors);
    __syncthreads();
    const uint32_t P = s_t;
    grid_barrier(&st->bar, round, P, &st->errors);
    if (rank == 0) own_prefix_block(agg, ntiles, s_w);
    grid_barrier(&st->bar, round, P, &st->errors);
    for (uint32_t t = rank; t < ntiles; t += P)
        own_apply_tile(t, sk, sidx, sop, svin, n, agg, res_val, res_flags, loc, sval, smeta, out_vals, out_status,
                       newflag, gw, part, st, wc, tilecnt, s_w);
    grid_barrier(&st->bar, round, P, &st->errors);
    if (rank == 0) {
        // slots of the new nodes: exclusive prefix of the tile counts
        uint32_t carry = 0;
        for (uint32_t b0 = 0; b0 < ntiles; b0 += OT * 4) {
            uint32_t v[4], sum = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t t = b0 + threadIdx.x * 4 + k;
                v[k] = t < ntiles ? tilecnt[t] : 0u;
                sum += v[k];
            }
            uint32_t tot;
            uint32_t run = carry + block_excl_scan_u32<OT>(sum, s_u, &tot);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t t = b0 + threadIdx.x * 4 + k;
                if (t < ntiles) tilecnt[t] = run;
                run += v[k];
            }
            carry += tot;
        }
        if (threadIdx.x == 0) {
            st->b_first = (uint32_t)st->nused;
            st->b_new = st->nused + carry > cap ? 0u : carry;  // no room: nothing is linked (the end flags it)
            if (st->nused + carry > cap) st->errors |= ERR_CAPACITY;
        }
    }
    grid_barrier(&st->bar, round, P, &st->errors);
    // new nodes in key order with their predecessors: tile offset plus the
    // rank inside the tile
    const uint32_t nnew = st->b_new;
    if (nnew) {
        for (uint32_t t = rank; t < ntiles; t += P) {
            const uint32_t base = t * OTILE + threadIdx.x * OI;
            uint32_t f[OI], c = 0;
#pragma unroll
            for (int e = 0; e < OI; e++) {
                f[e] = base + e < n ? newflag[base + e] : 0u;
                c += f[e];
            }
            uint32_t tot;
            uint32_t r = tilecnt[t] + block_excl_scan_u32<OT>(c, s_u, &tot);
#pragma unroll
            for (int e = 0; e < OI; e++) {
                if (!f[e]) continue;
                const uint32_t i = base + e;
                nk[r] = sk[i];
                nv[r] = svin[gw[i]];
                npred[r] = loc[i];
                npnext[r] = locnext[i];
                r++;
            }
        }
    }
    grid_barrier(&st->bar, round, P, &st->errors);
    link_range(rank * OT + threadIdx.x, P * OT, st->b_first, nnew, nk, nv, npred, npnext, skey, sval, snext, smeta,
               wc, &st->errors);
    // the counters: rank 0, after its own share of the links (the others
    // read only b_first and b_new, which the end does not change)
    if (rank == 0) {
        __syncthreads();
        batch_end_block(st, part, ntiles, cap, dpart, dgrid);
    }
}

__global__ void k_count_inserts(const uint8_t *__restrict__ ops, const uint64_t *__restrict__ keys, uint32_t n,
                                unsigned int *cnt) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t c = (i < n && ops[i] == PI_OP_INSERT && keys[i] != KEY_MAX) ? 1u : 0u;
    __shared__ uint32_t s_c[4];  // 256-thread blocks: one atomic per block, not per wave
    c = wave_sum_u32(c);
    if (lane_id() == 0) s_c[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = s_c[0] + s_c[1] + s_c[2] + s_c[3];
        if (t) atomicAdd(cnt, t);
    }
}

__global__ void k_zero_u32(unsigned int *p) {
    if (threadIdx.x == 0) *p = 0;
}

uint32_t blocks_for(uint64_t n, int t) { return (uint32_t)((n + t - 1) / t); }

template <int MODE, int QPL, int DT>
uint32_t launch_descend_q(Index &ix, hipStream_t s, const uint64_t *sk, const uint32_t *sidx, uint64_t n,
                          uint64_t *out_vals, uint8_t *out_status, uint64_t *res_val, uint8_t *res_flags, uint32_t *loc,
                          uint32_t *locnext, const uint8_t *ops, const uint64_t *vals, uint8_t *sop, uint64_t *svin,
                          uint2 *dpart, const unsigned int *wflag, uint32_t wsort) {
    const IndexDesc &d = ix.desc;
    const size_t lds = (size_t)d.lds_entries * 12;
    auto kern = k_descend<MODE, QPL, DT>;
    const uint32_t g = persistent_grid(ix, kern, DT, lds, blocks_for(n, DT * QPL));
    hipLaunchKernelGGL(kern, dim3(g), dim3(DT), lds, s, d, ix.arena_key.as<uint64_t>(), ix.arena_down.as<uint32_t>(),
                       ix.st.key.as<uint64_t>(), ix.st.val.as<uint64_t>(), ix.st.next.as<uint32_t>(),
                       ix.st.meta.as<uint8_t>(), sk, sidx, (uint32_t)n, ix.dstate, dpart, wflag, wsort, out_vals,
                       out_status, res_val, res_flags, loc, locnext, ops, vals, sop, svin);
    PI_LAUNCH_CHECK();
    return g;
}

template <int MODE, int DT>
uint32_t launch_descend_b(Index &ix, hipStream_t s, const uint64_t *sk, const uint32_t *sidx, uint64_t n,
                          uint64_t *out_vals, uint8_t *out_status, uint64_t *res_val, uint8_t *res_flags,
                          uint32_t *loc, uint32_t *locnext, const uint8_t *ops, const uint64_t *vals, uint8_t *sop,
                          uint64_t *svin, uint2 *dpart, const unsigned int *wflag, uint32_t wsort) {
    switch (ix.cfg.queries_per_lane) {
        case 2:
            return launch_descend_q<MODE, 2, DT>(ix, s, sk, sidx, n, out_vals, out_status, res_val, res_flags, loc,
                                                 locnext, ops, vals, sop, svin, dpart, wflag, wsort);
        case 4:
            return launch_descend_q<MODE, 4, DT>(ix, s, sk, sidx, n, out_vals, out_status, res_val, res_flags, loc,
                                                 locnext, ops, vals, sop, svin, dpart, wflag, wsort);
        default:
            return launch_descend_q<MODE, 1, DT>(ix, s, sk, sidx, n, out_vals, out_status, res_val, res_flags, loc,
                                                 locnext, ops, vals, sop, svin, dpart, wflag, wsort);
    }
}

// Launches the descent; returns its grid (the number of per-block count
// slots it writes in dpart).
template <int MODE>
uint32_t launch_descend(Index &ix, hipStream_t s, const uint64_t *sk, const uint32_t *sidx, uint64_t n,
                        uint64_t *out_vals, uint8_t *out_status, uint64_t *res_val, uint8_t *res_flags, uint32_t *loc,
                        uint32_t *locnext, const uint8_t *ops, const uint64_t *vals, uint8_t *sop, uint64_t *svin,
                        uint2 *dpart, const unsigned int *wflag, uint32_t wsort) {
    switch (ix.cfg.descent_block) {
        case 256:
            return launch_descend_b<MODE, 256>(ix, s, sk, sidx, n, out_vals, out_status, res_val, res_flags, loc,
                                               locnext, ops, vals, sop, svin, dpart, wflag, wsort);
        case 512:
            return launch_descend_b<MODE, 512>(ix, s, sk, sidx, n, out_vals, out_status, res_val, res_flags, loc,
                                               locnext, ops, vals, sop, svin, dpart, wflag, wsort);
        default:
            return launch_descend_b<MODE, 1024>(ix, s, sk, sidx, n, out_vals, out_status, res_val, res_flags, loc,
                                                locnext, ops, vals, sop, svin, dpart, wflag, wsort);
    }
}

}  // namespace

void BatchWorkspace::ensure(uint64_t m) {
    if (m <= n) return;
    const uint64_t c = m;
    res_val.ensure(c * 8);
    res_flags.ensure(c);
    loc.ensure(c * 4);
    locnext.ensure(c * 4);
    newflag.ensure(c * 4);
    newpos.ensure(c * 4);
    gw.ensure(c * 4);
    const uint64_t nt = (c + OTILE - 1) / OTILE + 1;
    agg.ensure(nt * sizeof(Seg));
    part.ensure(nt * sizeof(uint4));
    dpart.ensure(DPART * sizeof(uint2));
    sop.ensure(c);
    svin.ensure(c * 8);
    nk.ensure(c * 8);
    nv.ensure(c * 8);
    npred.ensure(c * 4);
    npnext.ensure(c * 4);
    n = m;
}

void BatchWorkspace::release() {
    DevBuf *all[] = {&res_val, &res_flags, &loc, &locnext, &newflag, &newpos, &gw, &agg,
                     &part, &dpart, &nk, &nv, &npred, &npnext, &sop, &svin};
    for (DevBuf *b : all) b->release();
    n = 0;
}

uint64_t count_inserts(Index &ix, const uint8_t *ops, const uint64_t *keys, uint64_t n, hipStream_t s,
                       unsigned int *cnt) {
    if (!cnt) {
        ix.tmp[5].ensure(16);
        cnt = ix.tmp[5].as<unsigned int>();
    }
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, cnt);
    hipLaunchKernelGGL(k_count_inserts, dim3(blocks_for(n, 256)), dim3(256), 0, s, ops, keys, (uint32_t)n, cnt);
    PI_LAUNCH_CHECK();
    unsigned int h = 0;
    PI_HIP(hipMemcpyAsync(ix.hcounts, cnt, 4, hipMemcpyDeviceToHost, s));
    PI_HIP(hipStreamSynchronize(s));
    h = *reinterpret_cast<unsigned int *>(ix.hcounts);
    return h;
}

void execute_batch(Index &ix, const uint8_t *ops, const uint64_t *keys, const uint64_t *vals, uint64_t n,
                   uint64_t *out_vals, uint8_t *out_status, hipStream_t s) {
    execute_batch(ix, BatchBuffers{ix.sortws, ix.msdws, ix.scanws, ix.bws}, ops, keys, vals, n, out_vals,
                  out_status, s);
}

void execute_batch(Index &ix, const BatchBuffers &buf, const uint8_t *ops, const uint64_t *keys,
                   const uint64_t *vals, uint64_t n, uint64_t *out_vals, uint8_t *out_status, hipStream_t s) {
    TraceRange tr("pi:batch");
    Profiler::Rec rec{};
    auto mark = [&](int k) {
        if (!ix.prof.on) return;
        rec.e[k] = ix.prof.take();
        PI_HIP(hipEventRecord(rec.e[k], s));
    };
    mark(0);
    const uint64_t *sk = nullptr;
    const uint32_t *sidx = nullptr;
    const uint32_t bits = order_bits(ix, n);
    order_batch(buf, ops, keys, n, s, &sk, &sidx, bits);
    mark(1);
    finish_batch(ix, buf, sk, sidx, ops, vals, n, out_vals, out_status, s, ix.prof.on ? &rec : nullptr, bits);
}

uint32_t order_bits(const Index &ix, uint64_t n) {
    // (16 relies on the descent's wave sort, which serves one query per lane)
    const uint32_t narrow = ix.cfg.queries_per_lane > 1 ? 24 : 16;
    const uint32_t b = ix.cfg.order_bits;
    if (b) return b == 16 ? narrow : b;
    if (!ix.recent_writers) return narrow;
    return n > (1u << 20) ? 32 : 24;
}

void order_batch(const BatchBuffers &buf, const uint8_t *ops, const uint64_t *keys, uint64_t n, hipStream_t so,
                 const uint64_t **sk, const uint32_t **sidx, uint32_t pos_bits) {
    TraceRange tr("pi:order");
    sort_batch_by_range(buf.sort, buf.msd, keys, ops, n, true, so, sk, sidx, pos_bits);
}

void finish_batch(Index &ix, const BatchBuffers &buf, const uint64_t *sk, const uint32_t *sidx, const uint8_t *ops,
                  const uint64_t *vals, uint64_t n, uint64_t *out_vals, uint8_t *out_status, hipStream_t s,
                  Profiler::Rec *prec, uint32_t pos_bits) {
    TraceRange tr("pi:descend+update");
    buf.bws.ensure(n);
    DevState *st = ix.dstate;
    auto mark = [&](int k) {
        if (!prec) return;
        prec->e[k] = ix.prof.take();
        PI_HIP(hipEventRecord(prec->e[k], s));
    };
    if (n == 0) {  // (otherwise the descent starts the per-batch counters)
        hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(64), 0, s, st, (uint32_t)n);
        PI_LAUNCH_CHECK();
    }

    BatchWorkspace &w = buf.bws;
    const WriterCheck wc = writer_check(ix, 1);
    const uint32_t dgrid = launch_descend<0>(ix, s, sk, sidx, n, out_vals, out_status, w.res_val.as<uint64_t>(),
                                             w.res_flags.as<uint8_t>(), w.loc.as<uint32_t>(), w.locnext.as<uint32_t>(),
                                             ops, vals, w.sop.as<uint8_t>(), w.svin.as<uint64_t>(),
                                             w.dpart.as<uint2>(), buf.msd.wflag.as<unsigned int>(),
                                             pos_bits == 16 ? 1u : 0u);
    if (dgrid > BatchWorkspace::DPART) throw Error{PI_ERR_DEVICE, "internal error: descent grid above its count slots"};
    PI_LAUNCH_CHECK();
    mark(2);

    const uint32_t otiles = blocks_for(n, OTILE);
    Seg *agg = w.agg.as<Seg>();
    // The steps after the descent in one launch with grid barriers, or as
    // separate kernels.  The one launch saves ~9 dispatches on a batch
    // without INSERT/DELETE (it only folds the counters), but its barriers
    // and its blocks that take part cost more than the separate kernels on
    // a batch with updates; the host cannot see which kind this batch is,
    // so it goes by the latest counters that reached it.  Under graph
    // capture always separate (a replay gives no say over which other
    // kernels share the device).
    hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
    PI_HIP(hipStreamIsCapturing(s, &cap_status));
    const uint32_t form = ix.cfg.post_form;
    const bool fused = cap_status == hipStreamCaptureStatusNone &&
                       (form == 1 || (form == 0 && !ix.recent_writers));
    if (fused) {
        static const int occ = [] {  // once per process, thread-safe
            int o = 0;
            PI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k_post, OT, 0));
            if (o < 1) throw Error{PI_ERR_DEVICE, "fused post-descent step cannot be resident"};
            return o;
        }();
        // two blocks per CU: every block that takes part costs same-address
        // atomics (joining, each barrier), slow with five blocks per CU
        const uint32_t grid =
            std::max<uint32_t>(1, std::min<uint32_t>(otiles, (uint32_t)ix.num_cus * std::min(occ, 2)));
        hipLaunchKernelGGL(k_post, dim3(grid), dim3(OT), 0, s, sk, sidx, w.sop.as<uint8_t>(), w.svin.as<uint64_t>(),
                           (uint32_t)n, w.res_val.as<uint64_t>(), w.res_flags.as<uint8_t>(), w.loc.as<uint32_t>(),
                           w.locnext.as<uint32_t>(), ix.st.key.as<uint64_t>(), ix.st.val.as<uint64_t>(),
                           ix.st.next.as<uint32_t>(), ix.st.meta.as<uint8_t>(), ix.st.cap, out_vals, out_status, agg,
                           w.part.as<uint4>(), w.newpos.as<uint32_t>() /* per-tile new-node counts, then their prefix */,
                           w.newflag.as<uint32_t>(), w.gw.as<int32_t>(), w.nk.as<uint64_t>(), w.nv.as<uint64_t>(),
                           w.npred.as<uint32_t>(), w.npnext.as<uint32_t>(), st, wc, (const uint2 *)w.dpart.as<uint2>(),
                           dgrid);
        PI_LAUNCH_CHECK();
        mark(3);  // the fused step counts as the ownership stage
    } else {
        hipLaunchKernelGGL(k_own_reduce, dim3(otiles), dim3(OT), 0, s, sk, w.sop.as<uint8_t>(), (uint32_t)n, st, agg);
        hipLaunchKernelGGL(k_own_prefix, dim3(1), dim3(OT), 0, s, agg, otiles, st);
        hipLaunchKernelGGL(k_own_apply, dim3(otiles), dim3(OT), 0, s, sk, sidx, w.sop.as<uint8_t>(),
                           w.svin.as<uint64_t>(), (uint32_t)n, agg,
                           w.res_val.as<uint64_t>(), w.res_flags.as<uint8_t>(), w.loc.as<uint32_t>(),
                           ix.st.val.as<uint64_t>(), ix.st.meta.as<uint8_t>(), out_vals, out_status,
                           w.newflag.as<uint32_t>(), w.gw.as<int32_t>(), w.part.as<uint4>(), st, wc);
        PI_LAUNCH_CHECK();
        mark(3);
        exclusive_scan_u32(buf.scan, w.newflag.as<uint32_t>(), w.newpos.as<uint32_t>(), n, &st->b_new,
                           &st->b_writers, s);
        // grid-stride launches of at most 8 blocks per CU: batches without
        // updates leave at once, and a smaller grid dispatches faster
        const uint32_t lgrid = std::min<uint32_t>(blocks_for(n, 256), (uint32_t)ix.num_cus * 8);
        hipLaunchKernelGGL(k_new_gather, dim3(lgrid), dim3(256), 0, s, sk, w.svin.as<uint64_t>(),
                           w.newflag.as<uint32_t>(), w.newpos.as<uint32_t>(), w.gw.as<int32_t>(), w.loc.as<uint32_t>(),
                           w.locnext.as<uint32_t>(), (uint32_t)n, st, w.nk.as<uint64_t>(), w.nv.as<uint64_t>(),
                           w.npred.as<uint32_t>(), w.npnext.as<uint32_t>());
        hipLaunchKernelGGL(k_link, dim3(lgrid), dim3(256), 0, s, w.nk.as<uint64_t>(), w.nv.as<uint64_t>(),
                           w.npred.as<uint32_t>(), w.npnext.as<uint32_t>(), st, ix.st.cap, ix.st.key.as<uint64_t>(),
                           ix.st.val.as<uint64_t>(), ix.st.next.as<uint32_t>(), ix.st.meta.as<uint8_t>(), wc);
        hipLaunchKernelGGL(k_batch_end, dim3(1), dim3(256), 0, s, st, (const uint4 *)w.part.as<uint4>(), otiles,
                           ix.st.cap, (const uint2 *)w.dpart.as<uint2>(), dgrid);
        PI_LAUNCH_CHECK();
    }
    mark(4);
    if (prec) {
        prec->n = 5;
        ix.prof.pending.push_back(*prec);
        if (ix.prof.pending.size() > 4096) ix.prof.drain(false);
    }
}

hipEvent_t Profiler::take() {
    if (pool.empty()) {
        hipEvent_t e;
        PI_HIP(hipEventCreate(&e));
        return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
}

void Profiler::drain(bool wait) {
    size_t done = 0;
    for (; done < pending.size(); done++) {
        Rec &r = pending[done];
        if (wait) {
            PI_HIP(hipEventSynchronize(r.e[r.n - 1]));
        } else if (hipEventQuery(r.e[r.n - 1]) != hipSuccess) {
            (void)hipGetLastError();
            break;
        }
        float t[4] = {0, 0, 0, 0};
        for (int k = 0; k + 1 < r.n; k++) PI_HIP(hipEventElapsedTime(&t[k], r.e[k], r.e[k + 1]));
        if (r.n == 5) {
            acc.batches++;
            acc.sort_ms += t[0];
            acc.descend_ms += t[1];
            acc.own_ms += t[2];
            acc.link_ms += t[3];
        } else {
            acc.rebuilds++;
            acc.rebuild_ms += t[0];
        }
        for (int k = 0; k < r.n; k++) pool.push_back(r.e[k]);
    }
    pending.erase(pending.begin(), pending.begin() + done);
}

void Profiler::release() {
    for (auto &r : pending)
        for (int k = 0; k < r.n; k++) pool.push_back(r.e[k]);
    pending.clear();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
}

namespace {

// Copies a batch into the staging buffers of a graph of capacity cap; the
// tail [n, cap) becomes invalid queries (op 255, key +infinity), which sort
// last, change nothing and are subtracted from the counters.
__global__ void k_stage_in(const uint8_t *__restrict__ ops, const uint64_t *__restrict__ keys,
                           const uint64_t *__restrict__ vals, uint64_t n, uint64_t cap, uint8_t *__restrict__ sops,
                           uint64_t *__restrict__ skeys, uint64_t *__restrict__ svals, DevState *st) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) st->b_pad = (unsigned int)(cap - n);
    if (i >= cap) return;
    if (i < n) {
        sops[i] = ops[i];
        skeys[i] = keys[i];
        svals[i] = vals[i];
    } else {
        sops[i] = 255;
        skeys[i] = KEY_MAX;
        svals[i] = 0;
    }
}

__global__ void k_stage_out(const uint64_t *__restrict__ sv, const uint8_t *__restrict__ ss, uint64_t n,
                            uint64_t *__restrict__ ov, uint8_t *__restrict__ os) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ov[i] = sv[i];
    os[i] = ss[i];
}

// Everything a captured graph bakes in: buffer addresses and launch shape.
std::vector<uint64_t> fingerprint(const Index &ix) {
    std::vector<uint64_t> f;
    auto add = [&](const DevBuf &b) {
        f.push_back((uint64_t)(uintptr_t)b.p);
        f.push_back(b.bytes);
    };
    add(ix.st.key), add(ix.st.val), add(ix.st.next), add(ix.st.meta);
    add(ix.arena_key), add(ix.arena_down);
    for (const DevBuf &b : ix.sortws.keys) add(b);
    for (const DevBuf &b : ix.sortws.idx) add(b);
    add(ix.sortws.tile_hist), add(ix.sortws.digit_tot);
    add(ix.msdws.partials), add(ix.msdws.map), add(ix.msdws.big), add(ix.msdws.nbig), add(ix.msdws.dirty);
    add(ix.scanws.tiles);
    const BatchWorkspace &w = ix.bws;
    add(w.res_val), add(w.res_flags), add(w.loc), add(w.locnext), add(w.newflag), add(w.newpos), add(w.gw);
    add(w.agg), add(w.part), add(w.dpart), add(w.nk), add(w.nv), add(w.npred), add(w.npnext), add(w.sop),
        add(w.svin);
    for (const DevBuf &b : ix.stage) add(b);
    f.push_back((uint64_t)(uintptr_t)ix.dstate);
    const uint64_t *d = reinterpret_cast<const uint64_t *>(&ix.desc);
    for (size_t i = 0; i < sizeof(IndexDesc) / 8; i++) f.push_back(d[i]);
    f.push_back(ix.cfg.descent_block), f.push_back(ix.cfg.queries_per_lane), f.push_back(ix.cfg.blocks_per_cu);
    f.push_back((uint64_t)ix.num_cus);
    return f;
}

}  // namespace

void release_graphs(Index &ix) {
    for (auto &g : ix.graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.fp.clear();
    }
    for (auto &b : ix.stage) b.release();
    if (ix.cap_stream) (void)hipStreamDestroy(ix.cap_stream);
    ix.cap_stream = nullptr;
}

void execute_batch_graph(Index &ix, const uint8_t *ops, const uint64_t *keys, const uint64_t *vals, uint64_t n,
                         uint64_t *out_vals, uint8_t *out_status, hipStream_t s) {
    int lg = 12;
    while ((1ull << lg) < n) lg++;
    const uint64_t cap = 1ull << lg;
    // every buffer the hot path touches, at the class size, before capture
    ix.stage[0].ensure(cap);
    ix.stage[1].ensure(cap * 8);
    ix.stage[2].ensure(cap * 8);
    ix.stage[3].ensure(cap * 8);
    ix.stage[4].ensure(cap);
    ix.bws.ensure(cap);
    ix.sortws.ensure(cap);
    ix.msdws.ensure(cap);
    ix.scanws.ensure(cap);
    uint8_t *sops = ix.stage[0].as<uint8_t>();
    uint64_t *skeys = ix.stage[1].as<uint64_t>(), *svals = ix.stage[2].as<uint64_t>();
    uint64_t *sov = ix.stage[3].as<uint64_t>();
    uint8_t *sos = ix.stage[4].as<uint8_t>();
    Index::Graph &g = ix.graphs[lg];
    std::vector<uint64_t> fp = fingerprint(ix);
    if (!g.exec || g.fp != fp) {
        if (g.exec) PI_HIP(hipGraphExecDestroy(g.exec));
        g.exec = nullptr;
        if (!ix.cap_stream) PI_HIP(hipStreamCreateWithFlags(&ix.cap_stream, hipStreamNonBlocking));
        PI_HIP(hipStreamBeginCapture(ix.cap_stream, hipStreamCaptureModeThreadLocal));
        hipGraph_t graph = nullptr;
        try {
            execute_batch(ix, sops, skeys, svals, cap, sov, sos, ix.cap_stream);
        } catch (...) {
            (void)hipStreamEndCapture(ix.cap_stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        PI_HIP(hipStreamEndCapture(ix.cap_stream, &graph));
        const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        PI_HIP(e);
        // capture must not have moved any buffer
        if (fingerprint(ix) != fp) throw Error{PI_ERR_DEVICE, "internal error: buffers moved during graph capture"};
        g.fp = fp;
    }
    hipLaunchKernelGGL(k_stage_in, dim3(blocks_for(cap, 256)), dim3(256), 0, s, ops, keys, vals, n, cap, sops, skeys,
                       svals, ix.dstate);
    PI_LAUNCH_CHECK();
    PI_HIP(hipGraphLaunch(g.exec, s));
    hipLaunchKernelGGL(k_stage_out, dim3(blocks_for(n, 256)), dim3(256), 0, s, sov, sos, n, out_vals, out_status);
    PI_LAUNCH_CHECK();
}

WriterCheck writer_check(Index &ix, uint32_t units) {
    WriterCheck wc{nullptr, 0};
    if (!ix.cfg.check_writers) return wc;
    const size_t need = (size_t)(ix.st.cap + STORAGE_SLACK) * sizeof(unsigned long long);
    if (ix.owner.bytes < need || !ix.owner.p) {
        ix.owner.ensure(need);
        PI_HIP(hipMemset(ix.owner.p, 0, ix.owner.bytes));  // tag 0: no writer yet
    }
    wc.owner = ix.owner.as<unsigned long long>();
    if (ix.writer_unit + units >= (1u << 30)) {  // units wrap: forget every recorded writer
        ix.writer_unit = 0;
        PI_HIP(hipMemset(ix.owner.p, 0, ix.owner.bytes));
    }
    wc.unit = ix.writer_unit + 1;
    ix.writer_unit += units;
    return wc;
}

bool writer_selftest(Index &ix, hipStream_t s, uint32_t *same_writer_err, uint32_t *two_writer_err) {
    ix.tmp[6].ensure(64);
    unsigned long long *shadow = ix.tmp[6].as<unsigned long long>();
    unsigned int *out = reinterpret_cast<unsigned int *>(shadow + 2);
    hipLaunchKernelGGL(k_writer_selftest, dim3(1), dim3(64), 0, s, shadow, out);
    PI_LAUNCH_CHECK();
    PI_HIP(hipMemcpyAsync(ix.hcounts, out, 8, hipMemcpyDeviceToHost, s));
    PI_HIP(hipStreamSynchronize(s));
    const uint32_t *h = reinterpret_cast<const uint32_t *>(ix.hcounts);
    *same_writer_err = h[0];
    *two_writer_err = h[1];
    return true;
}

void debug_interceptions(Index &ix, const uint64_t *keys, uint64_t n, uint64_t *icpt_keys, uint8_t *is_head,
                         hipStream_t s) {
    launch_descend<1>(ix, s, keys, nullptr, n, icpt_keys, is_head, nullptr, nullptr, nullptr, nullptr, nullptr,
                      nullptr, nullptr, nullptr, nullptr, nullptr, 0u);
}

}  // namespace pi
