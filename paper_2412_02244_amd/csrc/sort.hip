// Device-wide primitives: exclusive scan of uint32 and a stable LSD radix
// sort of (uint32 key, int32 value) pairs with 8-bit digits.
//
// The sort orders points (once per run) and, for large k, centroids (every
// iteration) along the Morton curve.  Stability makes the result a pure
// function of the input, so every build of the index is deterministic.
#include "ekm_internal.hpp"

namespace ekm {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / WAVE;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;

// ---------------------------------------------------------------- scan
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total, uint32_t *sh)
{
    // sh: SCAN_THREADS/WAVE + 1 words of LDS
    int lane = lane_id(), wid = threadIdx.x / WAVE;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    if (lane == WAVE - 1)
        sh[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) {
            uint32_t t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[blockDim.x / WAVE] = run;
    }
    __syncthreads();
    uint32_t r = x - v + sh[wid];
    *total = sh[blockDim.x / WAVE];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const uint32_t *data, int64_t n, uint32_t *sums)
{
    __shared__ uint32_t sh[SCAN_THREADS / WAVE + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        if (idx < n)
            s += data[idx];
    }
    uint32_t tot;
    block_exclusive_scan(s, &tot, sh);
    if (threadIdx.x == 0)
        sums[blockIdx.x] = tot;
}

// Single-block exclusive scan of the per-tile sums (in place).
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_sums(uint32_t *sums, int64_t m)
{
    __shared__ uint32_t sh[SCAN_THREADS / WAVE + 1];
    uint32_t carry = 0;
    for (int64_t base = 0; base < m; base += SCAN_THREADS) {
        int64_t idx = base + threadIdx.x;
        uint32_t v = idx < m ? sums[idx] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, &tot, sh);
        if (idx < m)
            sums[idx] = ex + carry;
        carry += tot;
    }
}

// Each tile: scan its elements in order (thread t owns SCAN_ITEMS consecutive ones).
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_apply(uint32_t *data, int64_t n, const uint32_t *sums)
{
    __shared__ uint32_t sh[SCAN_THREADS / WAVE + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + i;
        v[i] = idx < n ? data[idx] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, &tot, sh) + sums[blockIdx.x];
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + i;
        if (idx < n)
            data[idx] = run;
        run += v[i];
    }
}

size_t scan_scratch_words(int64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE) + 1; }

hipError_t exclusive_scan_u32(uint32_t *data, int64_t n, uint32_t *tmp, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, s, data, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, s, tmp, tiles);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, s, data, n, tmp);
    return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort
__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint32_t *keys, int64_t n, int shift, uint32_t *hist,
                                                        int64_t ntiles)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int64_t idx = base + (int64_t)r * RS_THREADS + threadIdx.x;
        if (idx < n)
            atomicAdd(&h[(keys[idx] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: elements of a tile are processed in index order, 256 per
// round; within a wave the rank among equal digits comes from ballots.
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint32_t *kin, const int32_t *vin, uint32_t *kout,
                                                           int32_t *vout, int64_t n, int shift, const uint32_t *offs,
                                                           int64_t ntiles)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[RS_WAVES][256];
    int wid = threadIdx.x / WAVE;
    base[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
    int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        if (tile0 + (int64_t)r * RS_THREADS >= n)
            break; // uniform across the block
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w)
            wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        int64_t idx = tile0 + (int64_t)r * RS_THREADS + threadIdx.x;
        bool valid = idx < n;
        uint32_t key = valid ? kin[idx] : 0u;
        int32_t val = valid ? vin[idx] : 0;
        uint32_t dig = (key >> shift) & 0xffu;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((dig >> b) & 1u);
            m &= ((dig >> b) & 1u) ? bal : ~bal;
        }
        int rank = __popcll(m & lanemask_lt());
        if (valid && rank == 0)
            wcnt[wid][dig] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t pos = base[dig] + (uint32_t)rank;
        for (int w = 0; w < wid; ++w)
            pos += wcnt[w][dig];
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w)
            add += wcnt[w][threadIdx.x];
        base[threadIdx.x] += add;
        if (valid) {
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

size_t radix_scratch_words(int64_t n)
{
    int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    return (size_t)(256 * tiles);
}

hipError_t radix_sort_u32(uint32_t *keys, int32_t *vals, uint32_t *keys_tmp, int32_t *vals_tmp, int64_t n, int bits,
                          uint32_t *hist, uint32_t *scan_tmp, hipStream_t s, bool *result_in_tmp)
{
    int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    uint32_t *ka = keys, *kb = keys_tmp;
    int32_t *va = vals, *vb = vals_tmp;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)tiles), dim3(RS_THREADS), 0, s, ka, n, shift, hist, tiles);
        hipError_t e = exclusive_scan_u32(hist, 256 * tiles, scan_tmp, s);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)tiles), dim3(RS_THREADS), 0, s, ka, va, kb, vb, n, shift,
                           hist, tiles);
        uint32_t *tk = ka;
        ka = kb;
        kb = tk;
        int32_t *tv = va;
        va = vb;
        vb = tv;
    }
    *result_in_tmp = (passes & 1) != 0;
    return hipGetLastError();
}

} // namespace ekm
