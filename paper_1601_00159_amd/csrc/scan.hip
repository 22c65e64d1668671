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

__global__ __launch_bounds__(CT) void k_scan_reduce(const uint32_t *__restrict__ in, uint64_t n,
                                                    uint32_t *__restrict__ tiles, const unsigned int *en) {
    if (en && *en == 0) return;
    __shared__ uint32_t s_w[NW];
    const uint64_t base = (uint64_t)blockIdx.x * CTILE;
    uint32_t sum = 0;
#pragma unroll 4
    for (int j = 0; j < CI; j++) {
        const uint64_t i = base + (uint64_t)j * CT + threadIdx.x;
        if (i < n) sum += in[i];
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

__global__ __launch_bounds__(CT) void k_scan_down(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                  uint64_t n, const uint32_t *__restrict__ tiles,
                                                  const unsigned int *en) {
    if (en && *en == 0) return;
    __shared__ uint32_t s_tmp[NW + 1];
    const uint64_t base = (uint64_t)blockIdx.x * CTILE + (uint64_t)threadIdx.x * CI;
    uint32_t v[CI];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < CI; j++) {
        const uint64_t i = base + j;
        v[j] = i < n ? in[i] : 0u;
        sum += v[j];
    }
    uint32_t tot;
    uint32_t run = tiles[blockIdx.x] + block_excl_scan_u32<CT>(sum, s_tmp, &tot);
#pragma unroll
    for (int j = 0; j < CI; j++) {
        const uint64_t i = base + j;
        if (i < n) out[i] = run;
        run += v[j];
    }
}

}  // namespace

void ScanWorkspace::ensure(uint64_t n) {
    const uint64_t ntiles = (n + CTILE - 1) / CTILE + 1;
    tiles.ensure(ntiles * sizeof(uint32_t));
}

void ScanWorkspace::release() { tiles.release(); }

void exclusive_scan_u32(ScanWorkspace &ws, const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *d_total,
                        const unsigned int *d_enable, hipStream_t s) {
    ws.ensure(n);
    const uint32_t ntiles = (uint32_t)((n + CTILE - 1) / CTILE);
    uint32_t *tiles = ws.tiles.as<uint32_t>();
    if (n == 0) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(CT), 0, s, tiles, 0u, d_total, d_enable);
        PI_LAUNCH_CHECK();
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(ntiles), dim3(CT), 0, s, in, n, tiles, d_enable);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(CT), 0, s, tiles, ntiles, d_total, d_enable);
    hipLaunchKernelGGL(k_scan_down, dim3(ntiles), dim3(CT), 0, s, in, out, n, tiles, d_enable);
    PI_LAUNCH_CHECK();
}

}  // namespace pi
