// Device-wide exclusive prefix sum of u32 (reduce, scan of tile sums,
// down-sweep).  Used to turn per-item flags into dense positions: new storage
// nodes of a batch, surviving nodes of a rebuild, de-duplicated keys of a bulk
// load.
#include "pi_internal.h"

namespace pi {
namespace {

constexpr int CT = 256;
constexpr int CI = 16;
constexpr int CTILE = CT * CI;
constexpr int NW = CT / 64;

// Sources of the scanned values: a u32 array, or the live flags of the base
// region read straight from the node flags (flag i = slot 1 + i is not
// deleted, for i < nbase; 0 at i = nbase).
struct SrcU32 {
    const uint32_t *p;
    __device__ __forceinline__ uint32_t at(uint64_t i) const { return p[i]; }
    // CI consecutive values from i0 (16-byte loads when aligned and in range)
    __device__ __forceinline__ void block(uint64_t i0, uint64_t n, uint32_t (&v)[CI]) const {
        const uint32_t *q = p + i0;
        if (i0 + CI <= n && (reinterpret_cast<uintptr_t>(q) & 15u) == 0) {
#pragma unroll
            for (int j = 0; j < CI / 4; j++) {
                const uint4 x = reinterpret_cast<const uint4 *>(q)[j];
                v[4 * j] = x.x;
                v[4 * j + 1] = x.y;
                v[4 * j + 2] = x.z;
                v[4 * j + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < CI; j++) v[j] = i0 + j < n ? q[j] : 0u;
        }
    }
};

struct SrcLive {
    const uint8_t *meta;  // flags of slot 1 onwards
    uint64_t nbase;
    __device__ __forceinline__ uint32_t at(uint64_t i) const {
        return (i < nbase && !(meta[i] & META_DEL)) ? 1u : 0u;
    }
    __device__ __forceinline__ void block(uint64_t i0, uint64_t n, uint32_t (&v)[CI]) const {
#pragma unroll
        for (int j = 0; j < CI; j++) v[j] = i0 + j < n ? at(i0 + j) : 0u;
    }
};

template <class Src>
__global__ __launch_bounds__(CT) void k_scan_reduce(Src src, uint64_t n, uint32_t *__restrict__ tiles,
                                                    const unsigned int *en) {
    if (en && *en == 0) return;
    __shared__ uint32_t s_w[NW];
    const uint64_t base = (uint64_t)blockIdx.x * CTILE;
    uint32_t sum = 0;
#pragma unroll 4
    for (int j = 0; j < CI; j++) {
        const uint64_t i = base + (uint64_t)j * CT + threadIdx.x;
        if (i < n) sum += src.at(i);
    }
    sum = wave_sum_u32(sum);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < NW; w++) t += s_w[w];
        tiles[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(CT) void k_scan_tiles(uint32_t *__restrict__ tiles, uint32_t ntiles,
                                                   uint32_t *__restrict__ total, const unsigned int *en) {
    if (en && *en == 0) {
        if (threadIdx.x == 0 && total) *total = 0;
        return;
    }
    __shared__ uint32_t s_tmp[NW + 1];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < ntiles; base += CT * 4) {
        uint32_t v[4];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t i = base + threadIdx.x * 4 + j;
            v[j] = i < ntiles ? tiles[i] : 0u;
            sum += v[j];
        }
        uint32_t tot;
        uint32_t run = carry + block_excl_scan_u32<CT>(sum, s_tmp, &tot);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t i = base + threadIdx.x * 4 + j;
            if (i < ntiles) tiles[i] = run;
            run += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <class Src>
__global__ __launch_bounds__(CT) void k_scan_down(Src src, uint32_t *__restrict__ out, uint64_t n,
                                                  const uint32_t *__restrict__ tiles, const unsigned int *en) {
    if (en && *en == 0) return;
    __shared__ uint32_t s_tmp[NW + 1];
    const uint64_t base = (uint64_t)blockIdx.x * CTILE + (uint64_t)threadIdx.x * CI;
    uint32_t v[CI];
    src.block(base, n, v);
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < CI; j++) sum += v[j];
    uint32_t tot;
    uint32_t run = tiles[blockIdx.x] + block_excl_scan_u32<CT>(sum, s_tmp, &tot);
    uint32_t r[CI];
#pragma unroll
    for (int j = 0; j < CI; j++) {
        r[j] = run;
        run += v[j];
    }
    uint32_t *o = out + base;
    if (base + CI <= n && (reinterpret_cast<uintptr_t>(o) & 15u) == 0) {
#pragma unroll
        for (int j = 0; j < CI / 4; j++)
            reinterpret_cast<uint4 *>(o)[j] = make_uint4(r[4 * j], r[4 * j + 1], r[4 * j + 2], r[4 * j + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < CI; j++)
            if (base + j < n) o[j] = r[j];
    }
}

template <class Src>
void scan_impl(ScanWorkspace &ws, Src src, uint32_t *out, uint64_t n, uint32_t *d_total,
               const unsigned int *d_enable, hipStream_t s) {
    ws.ensure(n);
    const uint32_t ntiles = (uint32_t)((n + CTILE - 1) / CTILE);
    uint32_t *tiles = ws.tiles.as<uint32_t>();
    if (n == 0) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(CT), 0, s, tiles, 0u, d_total, d_enable);
        PI_LAUNCH_CHECK();
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce<Src>, dim3(ntiles), dim3(CT), 0, s, src, n, tiles, d_enable);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(CT), 0, s, tiles, ntiles, d_total, d_enable);
    hipLaunchKernelGGL(k_scan_down<Src>, dim3(ntiles), dim3(CT), 0, s, src, out, n, tiles, d_enable);
    PI_LAUNCH_CHECK();
}

}  // namespace

void ScanWorkspace::ensure(uint64_t n) {
    const uint64_t ntiles = (n + CTILE - 1) / CTILE + 1;
    tiles.ensure(ntiles * sizeof(uint32_t));
}

void ScanWorkspace::release() { tiles.release(); }

void exclusive_scan_u32(ScanWorkspace &ws, const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *d_total,
                        const unsigned int *d_enable, hipStream_t s) {
    scan_impl(ws, SrcU32{in}, out, n, d_total, d_enable, s);
}

void exclusive_scan_live(ScanWorkspace &ws, const uint8_t *meta_slot1, uint64_t nbase, uint32_t *out,
                         uint32_t *d_total, hipStream_t s) {
    scan_impl(ws, SrcLive{meta_slot1, nbase}, out, nbase + 1, d_total, nullptr, s);
}

}  // namespace pi
