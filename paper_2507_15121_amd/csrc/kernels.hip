// gfx950 kernels for sparse MTTKRP (Eq. 1, Sec. 2.1), its bfloat16-factor
// form, the sparse CP loss and the fused residual + MTTKRP gradient.
//
// Work decomposition (one GPU's share of the paper's scheme, Sec. 3-4):
//  * A mode's nonzeros are sorted by output index (Sec. 3.1: all nonzeros of
//    one output index together) and cut into chunks of CH nonzeros, the
//    equal-size inter-shard partitions of Sec. 3.1/3.2.
//  * A persistent grid of wave64s replaces the hardware block scheduler of
//    Sec. 4.2: each wave takes the next chunk from a device atomic counter
//    until none is left, so skewed slices spread over all CUs.
//  * Inside a chunk the wave is G groups of LPR lanes.  Each lane holds RPL
//    consecutive columns of a factor row (16 bytes), so a group loads a whole
//    row with one coalesced access.  Group g walks its own contiguous run of
//    the chunk's nonzeros in order and keeps the running sum of the current
//    output row in registers (the elementwise computation, EC of Sec. 3,
//    reduced over consecutive equal output indices instead of one atomic per
//    nonzero as in Alg. 2).
//  * A row that starts and ends inside one group's run is written once with a
//    plain store.  Pieces of rows that cross group boundaries are parked in
//    LDS and summed at the end of the chunk; only rows that cross a chunk
//    boundary are added to memory with fp32 atomics (Sec. 3.2 uses atomics
//    between SMs), after the init kernel has zeroed them.
//  * Untouched output rows are zeroed once, by the init kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <unordered_map>
#include <utility>

#include "kernel_impl.h"

#ifndef AMPED_BUFFER_LOADS
#define AMPED_BUFFER_LOADS 1
#endif

namespace amped {
namespace dev {

// ----------------------------------------------------------------- init kernel
// Resets the work-queue counters (and the loss) and zeroes the output rows
// the MTTKRP kernel does not store: rows that several chunks add into,
// untouched rows of short runs (both in the zero-row list) and long runs of
// untouched rows.  vec4: ld, col0 and ncols are multiples of 4 (16-byte stores).
__global__ void __launch_bounds__(kBlock) init_kernel(float* out, int64_t ld, int col0, int ncols, bool vec4,
                                                      const int32_t* zrows, int64_t n_zero,
                                                      const int32_t* gaps, int64_t n_gaps, unsigned* queue,
                                                      double* loss)
{
    if (blockIdx.x == 0) {
        if (queue && threadIdx.x < kQueueSlots) queue[threadIdx.x] = 0u;
        if (loss && threadIdx.x == 0) *loss = 0.0;
    }
    if (!out) return;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int nv = vec4 ? ncols / 4 : ncols;  // stores per row
    const int64_t total = n_zero * nv;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += nthreads) {
        const int64_t r = zrows[i / nv];
        const int j = (int)(i % nv);
        if (vec4) *reinterpret_cast<float4*>(out + r * ld + col0 + 4 * j) = make_float4(0.f, 0.f, 0.f, 0.f);
        else out[r * ld + col0 + j] = 0.f;
    }
    // one (start, length) range per workgroup, at most about kGapPiece rows
    for (int64_t gi = blockIdx.x; gi < n_gaps; gi += gridDim.x) {
        const int64_t start = gaps[2 * gi], len = gaps[2 * gi + 1];
        const int64_t n = len * nv;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            const int64_t r = start + i / nv;
            const int j = (int)(i % nv);
            if (vec4) *reinterpret_cast<float4*>(out + r * ld + col0 + 4 * j) = make_float4(0.f, 0.f, 0.f, 0.f);
            else out[r * ld + col0 + j] = 0.f;
        }
    }
}

// A factor of `rows` rows is read through a 32-bit buffer offset when one
// more row still fits: padding entries use row -1, whose offset (2^32 - one
// row + column bytes) then lies past the end and reads zeros.
bool fits_buffer(int64_t rows, int rank, int elem_bytes)
{
    return (uint64_t)(rows + 1) * (uint64_t)rank * (uint64_t)elem_bytes <= (1ull << 32);
}

// Vector path: one 16-byte load per lane covers the row (rank * size / 16
// lanes).  Returns 0 when the rank needs the scalar column-tile path.
int vector_lpr(int rank, int elem_bytes)
{
    if ((rank * elem_bytes) % 16) return 0;
    const int lpr = rank * elem_bytes / 16;
    if (lpr < 2 || lpr > 64 || (lpr & (lpr - 1))) return 0;
    return lpr;
}

// Launch shape of an MTTKRP-kernel instance on the current device: the
// hot-row cache slots K (largest power of two whose LDS, with the kernel's
// static LDS, fits one block; capped by AMPED_HOT_MAX if set, 0 = no cache),
// the dynamic LDS bytes and the persistent grid (every CU filled to the
// occupancy that LDS allows).
struct Shape {
    int hot_k = 0;
    size_t dyn = 16;
    int grid = 0;
};

// Work-queue stripes per launch (1..kQueueSlots): AMPED_QUEUE_STRIPES, read
// once per process, else the default.
#ifndef AMPED_DEFAULT_STRIPES
#define AMPED_DEFAULT_STRIPES 8
#endif
int queue_stripes()
{
    static const int n = [] {
        const char* e = std::getenv("AMPED_QUEUE_STRIPES");
        const int v = (e && *e) ? std::atoi(e) : AMPED_DEFAULT_STRIPES;
        return std::max(1, std::min(v, kQueueSlots));
    }();
    return n;
}

#if AMPED_QUEUE_STATS
// Diagnostic build: the per-wave records of the last MTTKRP-shaped launch.
struct QueueStats {
    unsigned long long* dev = nullptr;
    int64_t cap = 0, n = 0;
    int waves_per_block = 0;
} g_qstats;
std::mutex g_qstats_mu;

hipError_t qstats_attach(KParams& k, int grid, int block, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_qstats_mu);
    const int64_t n = (int64_t)grid * (block / 64);
    if (n > g_qstats.cap) {
        if (g_qstats.dev) (void)hipFree(g_qstats.dev);
        g_qstats.dev = nullptr;
        g_qstats.cap = 0;
        hipError_t e = hipMalloc(&g_qstats.dev, (size_t)n * 4 * sizeof(unsigned long long));
        if (e != hipSuccess) return e;
        g_qstats.cap = n;
    }
    g_qstats.n = n;
    g_qstats.waves_per_block = block / 64;
    k.qstats = g_qstats.dev;
    return hipMemsetAsync(g_qstats.dev, 0, (size_t)n * 4 * sizeof(unsigned long long), st);
}
#endif

int hot_cap()
{
    static const int cap = [] {
        const char* e = std::getenv("AMPED_HOT_MAX");
        if (!e || !*e) return kHotMax;
        const int v = std::atoi(e);
        return v < 0 ? 0 : std::min(v, kHotMax);
    }();
    return cap;
}

Shape launch_shape(KernelFn fn, int block, int nin, int row_bytes, bool cache)
{
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, int, int, bool>, Shape> memo;
    int dev = 0;
    Shape sh;
    if (hipGetDevice(&dev) != hipSuccess) return sh;
    const void* f = reinterpret_cast<const void*>(fn);
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_tuple(dev, f, nin, row_bytes, cache);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    int cus = 0, max_lds = 0;
    hipFuncAttributes attr{};
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipFuncGetAttributes(&attr, f) != hipSuccess)
        return sh;
    if (cache) {
        for (int k = hot_cap(); k >= 16; k >>= 1)
            if (attr.sharedSizeBytes + hot_lds_bytes(nin, k, row_bytes) <= (size_t)max_lds) {
                sh.hot_k = k;
                break;
            }
    }
    // hot_cap() may not be a power of two: round down
    while (sh.hot_k & (sh.hot_k - 1)) sh.hot_k &= sh.hot_k - 1;
    sh.dyn = hot_lds_bytes(nin, sh.hot_k, row_bytes);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, block, sh.dyn) != hipSuccess || nb < 1) nb = 1;
    sh.grid = nb * cus;
    memo.emplace(key, sh);
    return sh;
}

hipError_t launch_init(const ModeDev& m, float* out, int64_t ld, int col0, int ncols, double* loss,
                       hipStream_t st)
{
    const bool vec4 = (ld % 4 == 0) && (col0 % 4 == 0) && (ncols % 4 == 0) &&
                      (reinterpret_cast<uintptr_t>(out) % 16 == 0);
    const int64_t work = std::max<int64_t>(m.n_zero * (vec4 ? ncols / 4 : ncols), m.n_gaps * kBlock);
    int grid = (int)std::min<int64_t>(std::max<int64_t>(1, (work + kBlock - 1) / kBlock), 4096);
    hipLaunchKernelGGL(init_kernel, dim3(grid), dim3(kBlock), 0, st, out, ld, col0, ncols, vec4, m.zero_rows,
                       out ? m.n_zero : 0, m.gaps, out ? m.n_gaps : 0, m.queue, loss);
    return hipGetLastError();
}

// Point the kernel at the K-slot hot tables of its inputs (K = 0: no cache;
// also when a table is missing).
void set_hot(KParams& k, int hot_k, const int32_t* const* in_hot, int nin)
{
    for (int w = 0; w < nin; ++w)
        if (!in_hot[w]) hot_k = 0;
    k.hot_k = hot_k;
    for (int w = 0; w < nin; ++w) k.hot[w] = hot_k ? in_hot[w] + (hot_k - 1) : nullptr;
}

KParams base_params(const ModeDev& m)
{
    KParams k{};
    k.out_idx = m.out_idx;
    for (int w = 0; w < kMaxIn; ++w) k.in_idx[w] = m.in_idx[w];
    k.val = m.val;
    k.queue = m.queue;
    k.n_stripes = queue_stripes();
    k.nnz = m.nnz;
    k.chunk = m.chunk;
    k.n_chunks = m.n_chunks;
    k.rows = m.rows;
    k.zero_row = m.zero_row;
    k.sink = m.sink;
    k.prev_key = m.prev_key;
    k.next_key = m.next_key;
    return k;
}

// dst[p] = src[perm[p]] for 32-bit words (layout build).
__global__ void __launch_bounds__(kBlock) permute_kernel(uint32_t* dst, const uint32_t* src, const int32_t* perm,
                                                         int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) dst[p] = src[perm[p]];
}

KernelFn pick_mttkrp(int nin, FactorType ft, Kind kind, int lpr, bool scalar, bool buf)
{
    if (kind == Kind::ResidualGrad) return ft == FactorType::F32 ? pick_grad(nin, lpr, scalar, buf) : nullptr;
    if (kind == Kind::ResidualGradLoss) return ft == FactorType::F32 ? pick_grad_loss(nin, lpr, scalar, buf) : nullptr;
    return ft == FactorType::F32 ? pick_mttkrp_f32(nin, lpr, scalar, buf) : pick_mttkrp_bf16(nin, lpr, scalar, buf);
}

}  // namespace dev

using namespace dev;

hipError_t launch_permute32(void* dst, const void* src, const int32_t* perm, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(permute_kernel, dim3(grid), dim3(kBlock), 0, st, static_cast<uint32_t*>(dst),
                       static_cast<const uint32_t*>(src), perm, n);
    return hipGetLastError();
}

hipError_t launch_mttkrp(const LaunchArgs& a)
{
    const ModeDev& m = *a.m;
    const int eb = (a.ftype == FactorType::F32) ? 4 : 2;
    const int lpr = vector_lpr(a.rank, eb);
    // buffer addressing when every factor the kernel reads fits in 32-bit
    // offsets with one row to spare
    bool buf = AMPED_BUFFER_LOADS != 0;
    for (int w = 0; w < a.nin; ++w)
        if (!fits_buffer(a.in_rows[w], a.rank, eb)) buf = false;
    const bool grad = a.kind != Kind::Mttkrp;   // the residual forms read the output mode's factor
    if (grad && !fits_buffer(m.rows, a.rank, 4)) buf = false;
    KernelFn fn = lpr ? pick_mttkrp(a.nin, a.ftype, a.kind, lpr, false, buf) : nullptr;
    const bool scalar = (fn == nullptr);
    // the fused residual form needs the whole row in one launch (rank <= 64
    // on the scalar path)
    if (scalar && grad && a.rank > 64) return hipErrorNotSupported;
    if (scalar) fn = pick_mttkrp(a.nin, a.ftype, a.kind, 64, true, false);
    if (!fn) return hipErrorNotSupported;
    KParams k = base_params(m);
    for (int w = 0; w < a.nin; ++w) {
        k.fac[w] = a.in_factors[w];
        k.fbytes[w] = buf ? (uint32_t)((uint64_t)a.in_rows[w] * a.rank * eb) : 0u;
    }
    k.own = a.own_factor;
    k.own_bytes = (buf && grad) ? (uint32_t)((uint64_t)m.rows * a.rank * 4) : 0u;
    k.out = a.out;
    k.loss = a.kind == Kind::ResidualGradLoss ? a.loss : nullptr;
    k.ld = a.rank;
    k.scale = a.scale;
    const int block = mttkrp_block(a.kind == Kind::Mttkrp ? 0 : 1);
    const Shape sh = launch_shape(fn, block, a.nin, a.rank * eb, !scalar && hot_cache_kind(a.kind == Kind::Mttkrp ? 0 : 1));
    if (sh.grid <= 0) return hipErrorInvalidDevice;
    set_hot(k, sh.hot_k, a.in_hot, a.nin);
    const int tile = scalar ? 64 : a.rank;
    for (int col0 = 0; col0 < a.rank; col0 += tile) {
        const int ncols = std::min(tile, a.rank - col0);
        // the loss (one launch: the residual forms never tile columns) is reset
        // by the init kernel unless this launch adds to it
        hipError_t e = launch_init(m, a.out, a.rank, col0, ncols, a.loss_accumulate ? nullptr : k.loss, a.stream);
        if (e != hipSuccess) return e;
        if (m.n_chunks == 0) continue;
        k.col0 = col0;
        k.ncols = ncols;
#if AMPED_QUEUE_STATS
        if ((e = qstats_attach(k, sh.grid, block, a.stream)) != hipSuccess) return e;
#endif
        void* args[] = {&k};
        e = hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(sh.grid), dim3(block), args, sh.dyn, a.stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

#if AMPED_QUEUE_STATS
hipError_t queue_stats_copy(unsigned long long* host, int64_t max_records, int64_t* n_records, int* waves_per_block)
{
    std::lock_guard<std::mutex> lk(g_qstats_mu);
    *n_records = g_qstats.n;
    *waves_per_block = g_qstats.waves_per_block;
    if (!host || g_qstats.n == 0) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    const int64_t n = std::min(max_records, g_qstats.n);
    return hipMemcpy(host, g_qstats.dev, (size_t)n * 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost);
}
#endif

hipError_t launch_cp_loss(const LossArgs& a)
{
    const ModeDev& m = *a.m;
    const int lpr = vector_lpr(a.rank, 4);
    bool buf = AMPED_BUFFER_LOADS != 0 && fits_buffer(m.rows, a.rank, 4);
    for (int w = 0; w < a.order - 1; ++w)
        if (!fits_buffer(a.in_rows[w], a.rank, 4)) buf = false;
    KernelFn fn = lpr ? pick_loss(a.order - 1, lpr, false, buf) : nullptr;
    const bool scalar = (fn == nullptr);
    if (scalar && a.rank > 64) return hipErrorNotSupported;
    if (scalar) fn = pick_loss(a.order - 1, 64, true, false);
    if (!fn) return hipErrorNotSupported;
    KParams k = base_params(m);
    for (int w = 0; w < a.order - 1; ++w) {
        k.fac[w] = a.in_factors[w];
        k.fbytes[w] = buf ? (uint32_t)((uint64_t)a.in_rows[w] * a.rank * 4) : 0u;
    }
    k.own = a.own_factor;
    k.own_bytes = buf ? (uint32_t)((uint64_t)m.rows * a.rank * 4) : 0u;
    k.loss = a.loss;
    k.ld = a.rank;
    k.col0 = 0;
    k.ncols = a.rank;
    hipError_t e = launch_init(m, nullptr, 0, 0, 0, a.accumulate ? nullptr : a.loss, a.stream);
    if (e != hipSuccess) return e;
    if (m.n_chunks == 0) return hipSuccess;
    const int block = mttkrp_block(2);
    const Shape sh = launch_shape(fn, block, a.order - 1, a.rank * 4, !scalar && hot_cache_kind(2));
    if (sh.grid <= 0) return hipErrorInvalidDevice;
    set_hot(k, sh.hot_k, a.in_hot, a.order - 1);
#if AMPED_QUEUE_STATS
    if ((e = qstats_attach(k, sh.grid, block, a.stream)) != hipSuccess) return e;
#endif
    void* args[] = {&k};
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(sh.grid), dim3(block), args, sh.dyn, a.stream);
}

}  // namespace amped
