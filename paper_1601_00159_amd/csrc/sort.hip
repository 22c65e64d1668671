// Stable LSD radix sort of (u64 key, u32 payload) pairs for gfx950.
//
// This is the ordering step of the batch (Definition 3: a query set is
// ordered by key; equal keys keep arrival order so that the batched answers
// equal the serial ones) and of the bulk-load / rebuild paths.
//
// Each 8-bit pass is three launches:
//   k_hist     per 4096-item tile digit counts (LDS atomics), column-major
//   k_colscan  one block per digit: exclusive scan of that digit's column
//   k_scatter  rank every item inside its tile (ballot match of the 8 digit
//              bits gives the lanes of a wave holding the same digit; a
//              per-wave LDS counter gives the running count), reorder the
//              tile in LDS by digit, then write each digit run contiguously.
// Ranks follow tile order, wave order, round order and lane order, which is
// the input order, so every pass is stable.
#include "pi_internal.h"

namespace pi {
namespace {

constexpr int ST = 512;           // threads per block
constexpr int SI = 8;             // items per thread
constexpr int STILE = ST * SI;    // items per tile
constexpr int CT = 256;           // column-scan block
constexpr int RBITS = 8;
constexpr int R = 1 << RBITS;     // digits per pass
constexpr int NW = ST / 64;       // waves per block

static_assert(R <= ST, "one digit per thread in the per-digit steps");

struct Digit {
    RangeMap map;
    uint32_t shift;
    bool ranged;
    __device__ __forceinline__ uint32_t operator()(uint64_t k) const {
        const uint64_t x = ranged ? (uint64_t)range_pos(k, map) : k;
        return (uint32_t)(x >> shift) & (R - 1);
    }
};

__device__ __forceinline__ Digit make_digit(uint32_t shift, const RangeMap *map) {
    Digit d;
    d.shift = shift;
    d.ranged = map != nullptr;
    if (map) d.map = *map;
    return d;
}

__global__ __launch_bounds__(ST) void k_hist(const uint64_t *__restrict__ keys, const uint8_t *__restrict__ ops,
                                             uint32_t n, uint32_t shift, const RangeMap *map,
                                             uint32_t *__restrict__ tile_hist, uint32_t ntiles,
                                             unsigned int *writers_flag) {
    __shared__ uint32_t h[R];
    const Digit dg = make_digit(shift, map);
    const int tid = threadIdx.x;
    if (tid < R) h[tid] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * STILE;
    uint32_t writers = 0;
#pragma unroll 4
    for (int j = 0; j < SI; j++) {
        const uint32_t i = base + j * ST + tid;
        if (i < n) {
            uint64_t k = keys[i];
            if (ops) {
                const uint8_t op = ops[i];
                if (op > PI_OP_DELETE)
                    k = KEY_MAX;
                else if (op != PI_OP_SEARCH && k != KEY_MAX)
                    writers++;
            }
            atomicAdd(&h[dg(k)], 1u);
        }
    }
    // the writers flag (nonzero: the batch has INSERT/DELETE queries): one
    // plain store per tile that has any, not an atomic per wave on one word
    const int any = __syncthreads_or(writers != 0);
    if (tid < R) tile_hist[(size_t)tid * ntiles + blockIdx.x] = h[tid];
    if (writers_flag && any && tid == 0) *writers_flag = 1;
}

__global__ __launch_bounds__(CT) void k_colscan(uint32_t *__restrict__ tile_hist, uint32_t ntiles,
                                                uint32_t *__restrict__ digit_tot) {
    __shared__ uint32_t s_tmp[CT / 64 + 1];
    uint32_t *col = tile_hist + (size_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < ntiles; base += CT * 8) {
        uint32_t v[8];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t i = base + threadIdx.x * 8 + j;
            v[j] = i < ntiles ? col[i] : 0u;
            sum += v[j];
        }
        uint32_t tot;
        uint32_t run = carry + block_excl_scan_u32<CT>(sum, s_tmp, &tot);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t i = base + threadIdx.x * 8 + j;
            if (i < ntiles) col[i] = run;
            run += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(ST) void k_scatter(const uint64_t *__restrict__ keys_in,
                                                const uint32_t *__restrict__ idx_in,
                                                const uint8_t *__restrict__ ops, uint32_t n, uint32_t shift,
                                                const RangeMap *map, const uint32_t *__restrict__ tile_hist,
                                                uint32_t ntiles, const uint32_t *__restrict__ digit_tot,
                                                uint64_t *__restrict__ keys_out, uint32_t *__restrict__ idx_out) {
    __shared__ uint32_t s_cnt[NW][R];
    const Digit dg = make_digit(shift, map);
    __shared__ uint32_t s_tstart[R];
    __shared__ uint32_t s_gstart[R];
    __shared__ uint32_t s_tmp[NW + 1];
    __shared__ uint64_t s_key[STILE];
    __shared__ uint32_t s_idx[STILE];

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid >> 6;
    for (int j = tid; j < NW * R; j += ST) (&s_cnt[0][0])[j] = 0;
    {
        uint32_t tot;
        const uint32_t ex = block_excl_scan_u32<ST>(tid < R ? digit_tot[tid] : 0u, s_tmp, &tot);
        if (tid < R) s_gstart[tid] = ex + tile_hist[(size_t)tid * ntiles + blockIdx.x];
    }
    __syncthreads();

    const uint32_t base = blockIdx.x * STILE;
    const uint32_t wbase = base + w * (SI * 64);
    uint64_t k[SI];
    uint32_t v[SI];
    uint32_t rk[SI];
#pragma unroll
    for (int r = 0; r < SI; r++) {
        const uint32_t i = wbase + r * 64 + lane;
        if (i < n) {
            uint64_t kk = keys_in[i];
            if (ops && ops[i] > PI_OP_DELETE) kk = KEY_MAX;
            k[r] = kk;
            v[r] = idx_in ? idx_in[i] : i;
        } else {
            k[r] = KEY_MAX;
            v[r] = 0;
        }
    }
#pragma unroll
    for (int r = 0; r < SI; r++) {
        const bool valid = (wbase + r * 64 + lane) < n;
        const uint32_t d = dg(k[r]);
        uint64_t m = ballot64(valid);
#pragma unroll
        for (int b = 0; b < RBITS; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bl = ballot64(bit);
            m &= bit ? bl : ~bl;
        }
        const uint32_t before = s_cnt[w][d];
        if (valid && lane == (int)__builtin_ctzll(m)) s_cnt[w][d] = before + (uint32_t)__popcll(m);
        rk[r] = before + mask_rank(m);
    }
    __syncthreads();
    {
        const uint32_t d = tid;
        uint32_t run = 0;
        if (tid < R) {
#pragma unroll
            for (int ww = 0; ww < NW; ww++) {
                const uint32_t c = s_cnt[ww][d];
                s_cnt[ww][d] = run;
                run += c;
            }
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan_u32<ST>(run, s_tmp, &tot);
        if (tid < R) s_tstart[d] = ex;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SI; r++) {
        if ((wbase + r * 64 + lane) < n) {
            const uint32_t d = dg(k[r]);
            const uint32_t p = s_tstart[d] + s_cnt[w][d] + rk[r];
            s_key[p] = k[r];
            s_idx[p] = v[r];
        }
    }
    __syncthreads();
    const uint32_t cnt = (n - base) < (uint32_t)STILE ? (n - base) : (uint32_t)STILE;
#pragma unroll 4
    for (int j = 0; j < SI; j++) {
        const uint32_t p = j * ST + tid;
        if (p < cnt) {
            const uint64_t kk = s_key[p];
            const uint32_t d = dg(kk);
            const uint32_t o = s_gstart[d] + (p - s_tstart[d]);
            keys_out[o] = kk;
            idx_out[o] = s_idx[p];
        }
    }
}

void sort_impl(SortWorkspace &ws, const uint64_t *keys, const uint32_t *payload, const uint8_t *ops,
               uint64_t n, unsigned int *writers, hipStream_t s, const uint64_t **out_keys,
               const uint32_t **out_idx) {
    ws.ensure(n);
    if (n == 0) {
        *out_keys = ws.keys[0].as<uint64_t>();
        *out_idx = ws.idx[0].as<uint32_t>();
        return;
    }
    const uint32_t nn = (uint32_t)n;
    const uint32_t ntiles = (uint32_t)((n + STILE - 1) / STILE);
    uint32_t *hist = ws.tile_hist.as<uint32_t>();
    uint32_t *tot = ws.digit_tot.as<uint32_t>();
    const uint64_t *kin = keys;
    const uint32_t *iin = payload;
    const uint8_t *opin = ops;
    for (int pass = 0; pass < 64 / RBITS; pass++) {
        const uint32_t shift = pass * RBITS;
        uint64_t *kout = ws.keys[pass & 1].as<uint64_t>();
        uint32_t *iout = ws.idx[pass & 1].as<uint32_t>();
        hipLaunchKernelGGL(k_hist, dim3(ntiles), dim3(ST), 0, s, kin, opin, nn, shift, (const RangeMap *)nullptr,
                           hist, ntiles, pass == 0 ? writers : nullptr);
        hipLaunchKernelGGL(k_colscan, dim3(R), dim3(CT), 0, s, hist, ntiles, tot);
        hipLaunchKernelGGL(k_scatter, dim3(ntiles), dim3(ST), 0, s, kin, iin, opin, nn, shift,
                           (const RangeMap *)nullptr, hist, ntiles, tot, kout, iout);
        PI_LAUNCH_CHECK();
        kin = kout;
        iin = iout;
        opin = nullptr;
    }
    *out_keys = kin;
    *out_idx = iin;
}

}  // namespace

void SortWorkspace::ensure(uint64_t n) {
    const uint64_t m = n ? n : 1;
    const uint64_t ntiles = (m + STILE - 1) / STILE;
    for (int i = 0; i < 2; i++) {
        keys[i].ensure(m * sizeof(uint64_t));
        idx[i].ensure(m * sizeof(uint32_t));
    }
    tile_hist.ensure(ntiles * R * sizeof(uint32_t));
    digit_tot.ensure(R * sizeof(uint32_t));
}

void SortWorkspace::release() {
    for (int i = 0; i < 2; i++) {
        keys[i].release();
        idx[i].release();
    }
    tile_hist.release();
    digit_tot.release();
}

void radix_pass(SortWorkspace &ws, const uint64_t *kin, const uint32_t *iin, const uint8_t *ops, uint32_t n,
                uint32_t shift, const RangeMap *map, unsigned int *writers, uint64_t *kout, uint32_t *iout,
                hipStream_t s) {
    if (n == 0) return;
    const uint32_t ntiles = (n + STILE - 1) / STILE;
    uint32_t *hist = ws.tile_hist.as<uint32_t>();
    uint32_t *tot = ws.digit_tot.as<uint32_t>();
    hipLaunchKernelGGL(k_hist, dim3(ntiles), dim3(ST), 0, s, kin, ops, n, shift, map, hist, ntiles, writers);
    hipLaunchKernelGGL(k_colscan, dim3(R), dim3(CT), 0, s, hist, ntiles, tot);
    hipLaunchKernelGGL(k_scatter, dim3(ntiles), dim3(ST), 0, s, kin, iin, ops, n, shift, map, hist, ntiles, tot,
                       kout, iout);
    PI_LAUNCH_CHECK();
}

void column_scan(uint32_t *cols, uint32_t ncols, uint32_t len, uint32_t *totals, hipStream_t s) {
    if (ncols == 0) return;
    hipLaunchKernelGGL(k_colscan, dim3(ncols), dim3(CT), 0, s, cols, len, totals);
    PI_LAUNCH_CHECK();
}

void sort_keys_with_index(SortWorkspace &ws, const uint64_t *keys, const uint8_t *ops, uint64_t n,
                          unsigned int *writers, hipStream_t s, const uint64_t **out_keys,
                          const uint32_t **out_idx) {
    sort_impl(ws, keys, nullptr, ops, n, writers, s, out_keys, out_idx);
}

void sort_pairs(SortWorkspace &ws, const uint64_t *keys, const uint32_t *payload, uint64_t n, hipStream_t s,
                const uint64_t **out_keys, const uint32_t **out_payload) {
    sort_impl(ws, keys, payload, nullptr, n, nullptr, s, out_keys, out_payload);
}

}  // namespace pi
