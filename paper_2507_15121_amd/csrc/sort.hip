// Device side of the per-mode layout builder (preprocessing, Sec. 5.7; not
// part of the timed MTTKRP): a stable least-significant-digit radix sort of
// (key, value) pairs, 8 bits per pass.
//
// One pass over n pairs, with tiles of kTile consecutive pairs per block:
//   1. histogram: each block counts the digits of its tile (LDS atomics) and
//      writes the 256 counts digit-major, hist[digit * nblocks + block];
//   2. scan: an exclusive prefix sum over that array gives, for every (digit,
//      block), where the block's pairs with that digit start in the output;
//   3. scatter: each block walks its tile again in order, 256 pairs per round.
//      A pair's rank among equal digits of the tile is the count from earlier
//      rounds + from earlier waves of the round + from earlier lanes of its
//      wave (lanes with the same digit are found by matching the 8 digit bits
//      with ballots), so equal digits keep their input order and every pass,
//      hence the whole sort, is stable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace amped {
namespace {

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kRounds = 16;
constexpr int64_t kTile = (int64_t)kSortBlock * kRounds;  // pairs per block
constexpr int kRadix = 256;
constexpr int kScanItems = 16;                              // per thread in the scan kernels
constexpr int64_t kScanTile = (int64_t)kSortBlock * kScanItems;

__global__ void __launch_bounds__(kSortBlock) radix_histogram(const uint32_t* keys, int64_t n, int shift,
                                                              uint32_t* hist, int64_t nblocks)
{
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = t0 + (int64_t)r * kSortBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of kScanTile items per block in place; the tile total goes
// to sums[block].
__global__ void __launch_bounds__(kSortBlock) scan_tiles(uint32_t* a, int64_t n, uint32_t* sums)
{
    __shared__ uint32_t s[kSortBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t tot = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        v[j] = i < n ? a[i] : 0u;
        const uint32_t x = v[j];
        v[j] = tot;
        tot += x;
    }
    s[threadIdx.x] = tot;
    __syncthreads();
    // inclusive Hillis-Steele scan of the thread totals
    for (int off = 1; off < kSortBlock; off <<= 1) {
        const uint32_t y = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    const uint32_t excl = s[threadIdx.x] - tot;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        if (i < n) a[i] = v[j] + excl;
    }
    if (threadIdx.x == kSortBlock - 1) sums[blockIdx.x] = s[threadIdx.x];
}

// Exclusive scan of the tile totals by one block, in order, with a carry.
__global__ void __launch_bounds__(kSortBlock) scan_sums(uint32_t* sums, int64_t m)
{
    __shared__ uint32_t s[kSortBlock];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b = 0; b < m; b += kSortBlock) {
        const int64_t i = b + threadIdx.x;
        const uint32_t x = i < m ? sums[i] : 0u;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < kSortBlock; off <<= 1) {
            const uint32_t y = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < m) sums[i] = carry + s[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == kSortBlock - 1) carry += s[threadIdx.x];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kSortBlock) add_sums(uint32_t* a, int64_t n, const uint32_t* sums)
{
    const uint32_t add = sums[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int j = threadIdx.x; j < kScanTile; j += kSortBlock) {
        const int64_t i = base + j;
        if (i < n) a[i] += add;
    }
}

__global__ void __launch_bounds__(kSortBlock) radix_scatter(const uint32_t* keys_in, const int32_t* vals_in,
                                                            uint32_t* keys_out, int32_t* vals_out, int64_t n,
                                                            int shift, const uint32_t* offsets, int64_t nblocks)
{
    __shared__ uint32_t s_base[kRadix];               // next output position per digit
    __shared__ uint32_t s_cnt[kSortWaves][kRadix];    // per wave, digit counts of the round
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    s_base[tid] = offsets[(int64_t)tid * nblocks + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) s_cnt[w][tid] = 0;
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = t0 + (int64_t)r * kSortBlock + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? keys_in[i] : 0u;
        const int32_t val = valid ? vals_in[i] : 0;
        const uint32_t dg = (key >> shift) & (kRadix - 1);
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t ones = __ballot(valid && bit);
            same &= bit ? ones : ~ones;
        }
        const uint32_t rank = (uint32_t)__popcll(same & below);
        if (valid && rank == 0) s_cnt[wave][dg] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pos = s_base[dg] + rank;
            for (int w = 0; w < wave; ++w) pos += s_cnt[w][dg];
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            tot += s_cnt[w][tid];
            s_cnt[w][tid] = 0;
        }
        s_base[tid] += tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kSortBlock) iota_kernel(int32_t* a, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = (int32_t)i;
}

int grid_for(int64_t items, int64_t per_block)
{
    return (int)std::max<int64_t>(1, (items + per_block - 1) / per_block);
}

}  // namespace

int64_t sort_scratch_words(int64_t n)
{
    const int64_t nblocks = (n + kTile - 1) / kTile;
    const int64_t hist = nblocks * kRadix;
    const int64_t tiles = (hist + kScanTile - 1) / kScanTile;
    return hist + tiles + 64;
}

hipError_t launch_iota(int32_t* a, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_kernel, dim3(std::min(grid_for(n, kSortBlock), 8192)), dim3(kSortBlock), 0, st, a, n);
    return hipGetLastError();
}

hipError_t launch_stable_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt,
                                    uint32_t* scratch, int64_t n, int key_bits, bool* result_in_alt,
                                    hipStream_t st)
{
    *result_in_alt = false;
    if (n <= 1 || key_bits <= 0) return hipSuccess;
    const int64_t nblocks = (n + kTile - 1) / kTile;
    const int64_t hist_len = nblocks * kRadix;
    const int64_t tiles = (hist_len + kScanTile - 1) / kScanTile;
    uint32_t* hist = scratch;
    uint32_t* sums = scratch + hist_len;
    uint32_t *ki = keys, *ko = keys_alt;
    int32_t *vi = vals, *vo = vals_alt;
    for (int shift = 0; shift < key_bits; shift += 8) {
        hipLaunchKernelGGL(radix_histogram, dim3((unsigned)nblocks), dim3(kSortBlock), 0, st, ki, n, shift, hist,
                           nblocks);
        hipLaunchKernelGGL(scan_tiles, dim3((unsigned)tiles), dim3(kSortBlock), 0, st, hist, hist_len, sums);
        hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kSortBlock), 0, st, sums, tiles);
        hipLaunchKernelGGL(add_sums, dim3((unsigned)tiles), dim3(kSortBlock), 0, st, hist, hist_len, sums);
        hipLaunchKernelGGL(radix_scatter, dim3((unsigned)nblocks), dim3(kSortBlock), 0, st, ki, vi, ko, vo, n, shift,
                           hist, nblocks);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(ki, ko);
        std::swap(vi, vo);
        *result_in_alt = !*result_in_alt;
    }
    return hipSuccess;
}

}  // namespace amped
