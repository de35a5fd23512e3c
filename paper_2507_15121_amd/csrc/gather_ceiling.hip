// Row-gather ceiling of the GPU: how fast random 128-byte rows (32 fp32) can
// be read from a table of a given size, with the same load shape as the
// MTTKRP kernel's gathers (16 bytes per lane, one row per group of 8 lanes,
// several rows per lane in flight).  Where the table fits the L2 this is the
// L2's rate; where it fits the Infinity Cache but not the L2, and where it
// only fits HBM, it is the rate at which the fabric returns L2 misses, the
// ceiling of any kernel whose time goes into L2 misses of row gathers.
//
//   gather_ceiling ROWS GATHERS ZIPF_S [BLOCKS_PER_CU]
//
// ROWS table rows, GATHERS rows read per launch, ZIPF_S 0 for uniform row
// indices, else the exponent of a Zipf law over the rows (ranks scattered by
// a multiplicative bijection).  Prints one line per lane layout: lanes per
// row segment LPR = 8 (whole rows per group, as the kernel), 4 and 2 (half
// and quarter rows, twice and four times as many rows per instruction).
//
//   gather_ceiling stream BYTES
//
// Sequential streaming rates over arrays of BYTES bytes (16-byte loads and
// stores, 8 per thread in flight, grid-stride): read only, write only, and
// copy (read + write), at 2, 4, 8 and 16 blocks of 256 threads per CU: what
// a streaming kernel of this GPU reaches against the 8 TB/s HBM peak.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#define CHECK(x)                                                                           \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) {                                                            \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(1);                                                                  \
        }                                                                                  \
    } while (0)

// LPR lanes read one 16*LPR-byte segment of a row; a wave instruction covers
// 64/LPR segments.  U loads per lane are in flight; the indices of the next
// step are loaded while the current step's rows are summed.
template <int LPR, int U>
__global__ __launch_bounds__(512) void gather(const float4* __restrict__ table, const int* __restrict__ idx,
                                              long nidx, float* out)
{
    constexpr int G = 64 / LPR;     // segments per instruction
    constexpr int SPR = 8 / LPR;    // segments per row
    const int lane = threadIdx.x & 63, g = lane / LPR, s = lane % LPR;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
    const long nitems = nidx * SPR;
    const long step = nwaves * G * U;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int r[U];
    long base = wave * G * U;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const long it = base + u * G + g;
        r[u] = it < nitems ? idx[it / SPR] : -1;
    }
    for (; base < nitems; base += step) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long it = base + u * G + g;
            const int q = (int)(it % SPR);
            v[u] = r[u] >= 0 ? table[(long)r[u] * 8 + q * LPR + s] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        const long nb = base + step;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long it = nb + u * G + g;
            r[u] = it < nitems ? idx[it / SPR] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
            acc.z += v[u].z;
            acc.w += v[u].w;
        }
    }
    float t = acc.x + acc.y + acc.z + acc.w;
    for (int m = 1; m < 64; m <<= 1) t += __shfl_xor(t, m, 64);
    if (lane == 0) out[wave] = t;
}

template <int LPR, int U>
float time_ms(const float4* table, const int* idx, long nidx, float* out, int grid)
{
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    for (int w = 0; w < 2; ++w) hipLaunchKernelGGL((gather<LPR, U>), dim3(grid), dim3(512), 0, 0, table, idx, nidx, out);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(a));
    const int reps = 5;
    for (int w = 0; w < reps; ++w) hipLaunchKernelGGL((gather<LPR, U>), dim3(grid), dim3(512), 0, 0, table, idx, nidx, out);
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
    return ms / reps;
}

// Streaming kernels over n 16-byte elements, U in flight per thread.
template <int U>
__global__ __launch_bounds__(256) void stream_copy(const float4* __restrict__ a, float4* __restrict__ b, long n)
{
    const long stride = (long)gridDim.x * 256 * U;
    for (long base = (long)blockIdx.x * 256 * U + threadIdx.x; base < n; base += stride) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long i = base + (long)u * 256;
            v[u] = i < n ? a[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long i = base + (long)u * 256;
            if (i < n) b[i] = v[u];
        }
    }
}

template <int U>
__global__ __launch_bounds__(256) void stream_read(const float4* __restrict__ a, float* out, long n)
{
    const long stride = (long)gridDim.x * 256 * U;
    float s = 0.f;
    for (long base = (long)blockIdx.x * 256 * U + threadIdx.x; base < n; base += stride) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long i = base + (long)u * 256;
            v[u] = i < n ? a[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    out[(long)blockIdx.x * 256 + threadIdx.x] = s;   // one float per thread keeps the loads
}

__global__ __launch_bounds__(256) void stream_write(float4* b, long n)
{
    const long stride = (long)gridDim.x * 256;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) b[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

int stream_main(long bytes)
{
    const long n = bytes / 16;
    if (n < 1) {
        std::fprintf(stderr, "BYTES must be at least 16\n");
        return 2;
    }
    int cus = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    float4 *a, *b;
    float* out;
    CHECK(hipMalloc(&a, n * 16));
    CHECK(hipMalloc(&b, n * 16));
    CHECK(hipMalloc(&out, (long)cus * 16 * 256 * sizeof(float)));
    CHECK(hipMemset(a, 0, n * 16));
    CHECK(hipMemset(b, 0, n * 16));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    auto timed = [&](auto launch) {
        launch();
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(e0, 0));
        for (int k = 0; k < 5; ++k) launch();
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        CHECK(hipGetLastError());
        return ms / 5;
    };
    for (int bpc : {2, 4, 8, 16}) {
        const int grid = cus * bpc;
        const float r = timed([&] { hipLaunchKernelGGL(stream_read<8>, dim3(grid), dim3(256), 0, 0, a, out, n); });
        const float w = timed([&] { hipLaunchKernelGGL(stream_write, dim3(grid), dim3(256), 0, 0, b, n); });
        const float c = timed([&] { hipLaunchKernelGGL(stream_copy<8>, dim3(grid), dim3(256), 0, 0, a, b, n); });
        std::printf("stream %.3g GB, %d blocks/CU: read %.3f ms %.0f GB/s, write %.3f ms %.0f GB/s, "
                    "copy %.3f ms %.0f GB/s (read + write bytes)\n",
                    n * 16e-9, bpc, r, n * 16 / (r * 1e-3) / 1e9, w, n * 16 / (w * 1e-3) / 1e9, c,
                    2.0 * n * 16 / (c * 1e-3) / 1e9);
    }
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(out));
    return 0;
}

int main(int argc, char** argv)
{
    if (argc == 3 && std::string(argv[1]) == "stream") return stream_main(std::atol(argv[2]));
    if (argc < 4) {
        std::fprintf(stderr, "usage: %s ROWS GATHERS ZIPF_S [BLOCKS_PER_CU] | %s stream BYTES\n", argv[0], argv[0]);
        return 2;
    }
    const long rows = std::atol(argv[1]);
    const long nidx = std::atol(argv[2]);
    const double zipf_s = std::atof(argv[3]);
    const int blocks_per_cu = argc > 4 ? std::atoi(argv[4]) : 2;
    if (rows < 1 || rows > (1L << 31) - 1 || nidx < 1 || blocks_per_cu < 1) {
        std::fprintf(stderr, "ROWS must be in [1, 2^31), GATHERS and BLOCKS_PER_CU >= 1\n");
        return 2;
    }
    std::vector<int> h(nidx);
    std::mt19937_64 rng(12345);
    if (zipf_s <= 0) {
        std::uniform_int_distribution<long> d(0, rows - 1);
        for (long i = 0; i < nidx; ++i) h[i] = (int)d(rng);
    } else {
        std::vector<double> cdf(rows);
        double s = 0;
        for (long k = 0; k < rows; ++k) {
            s += std::pow((double)(k + 1), -zipf_s);
            cdf[k] = s;
        }
        std::uniform_real_distribution<double> u(0, s);
        for (long i = 0; i < nidx; ++i) {
            long k = std::lower_bound(cdf.begin(), cdf.end(), u(rng)) - cdf.begin();
            if (k >= rows) k = rows - 1;
            h[i] = (int)(((unsigned long long)k * 2654435761ull) % (unsigned long long)rows);
        }
    }
    for (long i = 0; i < nidx; ++i)
        if (h[i] < 0 || h[i] >= rows) {
            std::fprintf(stderr, "index out of range\n");
            return 1;
        }
    float4* table;
    int* idx;
    float* out;
    CHECK(hipMalloc(&table, rows * 128));
    CHECK(hipMemset(table, 0, rows * 128));
    CHECK(hipMalloc(&idx, nidx * 4));
    CHECK(hipMemcpy(idx, h.data(), nidx * 4, hipMemcpyHostToDevice));
    int cus = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const int grid = cus * blocks_per_cu;
    CHECK(hipMalloc(&out, (long)grid * 8 * sizeof(float)));
    struct Res {
        const char* name;
        float ms;
    } res[] = {{"LPR 8, 8 in flight", time_ms<8, 8>(table, idx, nidx, out, grid)},
               {"LPR 4, 8 in flight", time_ms<4, 8>(table, idx, nidx, out, grid)},
               {"LPR 2, 8 in flight", time_ms<2, 8>(table, idx, nidx, out, grid)}};
    for (const auto& r : res)
        std::printf("rows %ld (%.3g GB), gathers %ld, zipf %.2f, %d blocks/CU, %s: %.3f ms, %.1f G rows/s, %.0f GB/s\n",
                    rows, rows * 128e-9, nidx, zipf_s, blocks_per_cu, r.name, r.ms, nidx / (r.ms * 1e-3) / 1e9,
                    nidx * 128.0 / (r.ms * 1e-3) / 1e9);
    CHECK(hipFree(table));
    CHECK(hipFree(idx));
    CHECK(hipFree(out));
    return 0;
}
