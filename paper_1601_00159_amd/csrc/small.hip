// A whole batch in one workgroup: the hot path for batches of at most
// SB_MAX queries, in one launch.
//
// The multi-kernel path pays about 26 launches per batch; below a few
// thousand queries that host cost, not the device, sets the batch rate.  Here
// one 1024-thread workgroup runs every step with barriers in between:
//
//   order      bitonic sort of (key, arrival position) in LDS -- the stable
//              key order of Definition 3 (invalid queries sort last as
//              +infinity)
//   descend    each thread takes ceil(n / 1024) <= 4 consecutive sorted
//              queries through the index levels (Algorithm 2, two chains at
//              a time; the top levels from an LDS copy) and along the
//              storage list (getNode of Algorithm 4)
//   ownership  a block-wide segmented "last writer" scan over the sorted
//              queries gives every answer and makes each key group's last
//              query the only writer of its node (the hand-over of
//              Algorithm 3 done by a prefix scan)
//   apply      owners update values and delete flags; new nodes take the
//              next free slots (a block-wide prefix sum over the owners that
//              insert) and are linked behind their predecessor, chained when
//              they share one (Algorithm 4)
//
// The workgroup is the only writer of the index while it runs, so the
// counters are updated by one thread at the end.  The same device function
// serves one index per workgroup in the many-index launch.
#include "small.h"

namespace pi {

uint32_t small_batch_lds_bytes() { return SmallLds::bytes(); }

namespace {

__global__ __launch_bounds__(SBT) void k_batch_block(IndexView v, BatchView b) {
    extern __shared__ uint64_t s_raw[];
    block_batch(v, b, s_raw);
}

}  // namespace

void execute_batch_small(Index &ix, const uint8_t *ops, const uint64_t *keys, const uint64_t *vals, uint64_t n,
                         uint64_t *out_vals, uint8_t *out_status, hipStream_t s) {
    IndexView v = index_view(ix);
    const WriterCheck wc = writer_check(ix, 1);
    v.owner = wc.owner;
    BatchView b{ops, keys, vals, (uint32_t)n, out_vals, out_status, wc.unit, 1};
    const uint32_t lds = SmallLds::bytes();
    // once per process (thread-safe: calls on different indices may run in
    // parallel threads)
    static const bool attr = [&] {
        PI_HIP(hipFuncSetAttribute((const void *)k_batch_block, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        return true;
    }();
    (void)attr;
    hipLaunchKernelGGL(k_batch_block, dim3(1), dim3(SBT), lds, s, v, b);
    PI_LAUNCH_CHECK();
}

}  // namespace pi
