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
//  * Untouched output rows are zeroed once: short runs by the wave that
//    reaches them, long runs by the init kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <unordered_map>
#include <utility>

#include "internal.h"

namespace amped {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxIn = kMaxOrder - 1;

// Tuning knobs (compile-time): sub-steps whose gathers are issued together
// (for up to 2 input modes; half of it above), and the waves per SIMD the
// register allocation must allow (0 = compiler's choice).
#ifndef AMPED_UMAX
#define AMPED_UMAX 8
#endif
#ifndef AMPED_FIBER
#define AMPED_FIBER 0
#endif
#ifndef AMPED_MIN_WAVES
#define AMPED_MIN_WAVES 0
#endif
#if AMPED_MIN_WAVES > 0
#define AMPED_OCCUPANCY __attribute__((amdgpu_waves_per_eu(AMPED_MIN_WAVES)))
#else
#define AMPED_OCCUPANCY
#endif

typedef int i32x4 __attribute__((ext_vector_type(4)));

struct KParams {
    const int32_t* out_idx;
    const int32_t* in_idx[kMaxIn];
    const float* val;
    const void* fac[kMaxIn];
    const float* own;
    float* out;
    double* loss;
    int* queue;
    int64_t nnz, chunk, n_chunks, rows;
    int64_t ld;     // row stride of factors and output, in elements
    int col0;       // first column handled by this launch
    int ncols;      // columns handled by this launch
    float scale;
};

// ------------------------------------------------------------ compile-time loops
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Value of lane (group base + J) for every lane of an LPR-lane group.
template <int LPR, int J>
__device__ __forceinline__ int group_bcast(int x)
{
    if constexpr (LPR == 1) {
        return x;
    } else if constexpr (LPR == 64) {
        return __builtin_amdgcn_readlane(x, J);
    } else {
        // ds_swizzle bit mode inside 32-lane halves: lane' = (lane & and) | or
        constexpr int and_mask = 0x1F & ~(LPR - 1);
        return __builtin_amdgcn_ds_swizzle(x, and_mask | (J << 5));
    }
}
template <int LPR, int J>
__device__ __forceinline__ float group_bcast_f(float x)
{
    return __int_as_float(group_bcast<LPR, J>(__float_as_int(x)));
}

// Broadcast of lane (group base + jb*U + JU).  One batch per tile: compile-time
// ds_swizzle.  Several batches: the batch index is a run-time (wave-uniform)
// loop counter, so ds_bpermute, or v_readlane when the group is the wave.
template <int LPR, int U, int NB, int JU>
__device__ __forceinline__ int tile_bcast(int x, int jb, int lane)
{
    if constexpr (NB == 1) {
        return group_bcast<LPR, JU>(x);
    } else if constexpr (LPR == 64) {
        return __builtin_amdgcn_readlane(x, jb * U + JU);
    } else {
        return __builtin_amdgcn_ds_bpermute(((lane & ~(LPR - 1)) + jb * U + JU) << 2, x);
    }
}
template <int LPR, int U, int NB, int JU>
__device__ __forceinline__ float tile_bcast_f(float x, int jb, int lane)
{
    return __int_as_float(tile_bcast<LPR, U, NB, JU>(__float_as_int(x), jb, lane));
}

template <int LPR>
__device__ __forceinline__ float group_sum(float x)
{
#pragma unroll
    for (int m = 1; m < LPR; m <<= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// ------------------------------------------------------------------ row access
// Row<T, RPL>: RPL consecutive columns of a factor row as fp32.  `lp` is the
// lane's base pointer (factor + its first column), `rb` the row stride in
// bytes (a compile-time constant on the vector path, so the address is one
// 64-bit shift-add).
template <typename T, int RPL> struct Row;

template <> struct Row<float, 4> {
    using Raw = float4;
    static __device__ __forceinline__ Raw load(const char* lp, uint32_t row, uint64_t rb)
    {
        return *reinterpret_cast<const float4*>(lp + (uint64_t)row * rb);
    }
    static __device__ __forceinline__ Raw zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
    static __device__ __forceinline__ void unpack(const Raw& r, float (&v)[4])
    {
        v[0] = r.x; v[1] = r.y; v[2] = r.z; v[3] = r.w;
    }
};

template <> struct Row<uint16_t, 8> {  // bfloat16 bit patterns, widened exactly
    using Raw = uint4;
    static __device__ __forceinline__ Raw load(const char* lp, uint32_t row, uint64_t rb)
    {
        return *reinterpret_cast<const uint4*>(lp + (uint64_t)row * rb);
    }
    static __device__ __forceinline__ Raw zero() { return make_uint4(0u, 0u, 0u, 0u); }
    static __device__ __forceinline__ void unpack(const Raw& r, float (&v)[8])
    {
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 * i] = __uint_as_float(w[i] << 16);
            v[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
        }
    }
};

template <> struct Row<float, 1> {
    using Raw = float;
    static __device__ __forceinline__ Raw load(const char* lp, uint32_t row, uint64_t rb)
    {
        return *reinterpret_cast<const float*>(lp + (uint64_t)row * rb);
    }
    static __device__ __forceinline__ Raw zero() { return 0.f; }
    static __device__ __forceinline__ void unpack(const Raw& r, float (&v)[1]) { v[0] = r; }
};

template <> struct Row<uint16_t, 1> {
    using Raw = uint32_t;
    static __device__ __forceinline__ Raw load(const char* lp, uint32_t row, uint64_t rb)
    {
        return *reinterpret_cast<const uint16_t*>(lp + (uint64_t)row * rb);
    }
    static __device__ __forceinline__ Raw zero() { return 0u; }
    static __device__ __forceinline__ void unpack(const Raw& r, float (&v)[1]) { v[0] = __uint_as_float(r << 16); }
};

// Output row pieces: RPL fp32 columns of row `row`, starting at column c.
template <int RPL>
__device__ __forceinline__ void store_cols(float* out, int64_t row, int64_t ld, int c, const float (&v)[RPL])
{
    float* p = out + row * ld + c;
    if constexpr (RPL % 4 == 0) {
#pragma unroll
        for (int i = 0; i < RPL; i += 4)
            *reinterpret_cast<float4*>(p + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < RPL; ++i) p[i] = v[i];
    }
}

template <int RPL>
__device__ __forceinline__ void atomic_cols(float* out, int64_t row, int64_t ld, int c, const float (&v)[RPL])
{
    float* p = out + row * ld + c;
#pragma unroll
    for (int i = 0; i < RPL; ++i) atomicAdd(p + i, v[i]);
}

template <int RPL>
__device__ __forceinline__ void zero_rows(float* out, int64_t first, int64_t last_excl, int64_t ld, int c)
{
    float z[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) z[i] = 0.f;
    for (int64_t r = first; r < last_excl; ++r) store_cols<RPL>(out, r, ld, c, z);
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int pop_chunk(int* queue, int lane)
{
    int c = 0;
    if (lane == 0) c = atomicAdd(queue, 1);
    return __builtin_amdgcn_readfirstlane(c);
}

// ----------------------------------------------------------------- init kernel
// Resets the work-queue counter (and the loss), zeroes the output rows that
// several chunks add into, and the long runs of untouched rows.
__global__ void __launch_bounds__(kBlock) init_kernel(float* out, int64_t ld, int col0, int ncols,
                                                      const int32_t* split, int64_t n_split,
                                                      const int32_t* gaps, int64_t n_gaps, int* queue,
                                                      double* loss)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (queue) *queue = 0;
        if (loss) *loss = 0.0;
    }
    if (!out) return;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int64_t total = n_split * ncols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += nthreads) {
        const int64_t r = split[i / ncols];
        out[r * ld + col0 + (i % ncols)] = 0.f;
    }
    for (int64_t gi = blockIdx.x; gi < n_gaps; gi += gridDim.x) {
        const int64_t start = gaps[2 * gi], len = gaps[2 * gi + 1];
        const int64_t n = len * ncols;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
            out[(start + i / ncols) * ld + col0 + (i % ncols)] = 0.f;
    }
}

// ------------------------------------------------------------- MTTKRP kernels
// KIND 0: MTTKRP.  KIND 1: scale * MTTKRP of the residuals val - CP model,
// recomputed per nonzero from all factor rows.
template <int NIN, int LPR, int RPL, typename T, int KIND>
__global__ void __launch_bounds__(kBlock) AMPED_OCCUPANCY mttkrp_kernel(const KParams p)
{
    constexpr int G = 64 / LPR;                       // nonzero groups per wave
    constexpr int RT = LPR * RPL;                     // columns per wave row
    constexpr int UMAX = (NIN <= 2) ? AMPED_UMAX : (AMPED_UMAX + 1) / 2;
    constexpr int MPL = (LPR < UMAX) ? UMAX / LPR : 1;  // nonzeros of metadata per lane
    constexpr int TS = LPR * MPL;                     // nonzeros per group per tile
    constexpr int U = (TS < UMAX) ? TS : UMAX;        // sub-steps per gather batch
    constexpr int NB = TS / U;                        // batches per tile (MPL == 1 if NB > 1)
    using RowT = Row<T, RPL>;
    using OwnRow = Row<float, (KIND == 1) ? RPL : 1>;
    static_assert(KIND == 0 || std::is_same<T, float>::value, "residual form is fp32 only");

    __shared__ int s_key[kWaves][2 * G];
    __shared__ int s_ext[kWaves][2 * G];
    __shared__ float s_acc[kWaves][2 * G][RT];

    // vector path: the row is exactly RT columns, so the strides are constants
    constexpr bool VEC = RPL > 1;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int g = lane / LPR;
    const int s = lane % LPR;
    const bool lane_on = VEC || (s * RPL < p.ncols);
    const int c = p.col0 + (lane_on ? s * RPL : 0);   // this lane's first column (kept in the row)
    const int64_t ld = VEC ? (int64_t)RT : p.ld;
    const uint64_t rb = (uint64_t)ld * sizeof(T);
    const uint64_t rb_own = (uint64_t)ld * sizeof(float);
    const float oscale = (KIND == 1) ? p.scale : 1.0f;
    const char* lbase[NIN];
#pragma unroll
    for (int w = 0; w < NIN; ++w) lbase[w] = static_cast<const char*>(p.fac[w]) + (int64_t)c * sizeof(T);
    const char* obase = (KIND == 1) ? reinterpret_cast<const char*>(p.own + c) : nullptr;

    for (;;) {
        const int chunk = pop_chunk(p.queue, lane);
        if (chunk >= p.n_chunks) break;
        const int64_t cs = (int64_t)chunk * p.chunk;
        const int64_t ce = min(cs + p.chunk, p.nnz);
        const int64_t Lg = ((ce - cs + G * TS - 1) / (G * TS)) * TS;
        const int64_t gs = cs + g * Lg;
        const int64_t ge = min(gs + Lg, ce);
        const bool gon = gs < ge;

        if (s == 0) {
            s_key[wv][2 * g] = -1;
            s_key[wv][2 * g + 1] = -1;
        }

        int open_key = -1;
        bool open_first = true;
        bool left_shared = false;
        float acc[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) acc[i] = 0.f;

        if (gon) {
            const int first = p.out_idx[gs];
            const int prev = gs > 0 ? p.out_idx[gs - 1] : -1;
            left_shared = (prev == first);
            if (lane_on && first - prev - 1 > 0 && first - prev - 1 < kGapInKernel)
                zero_rows<RPL>(p.out, prev + 1, first, ld, c);
            open_key = first;
        }

        bool parked = false;
        auto flush_mid = [&]() {
            // the open segment ended inside the run
            if (open_first && left_shared) {
                parked = true;
                float* dst = &s_acc[wv][2 * g][s * RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) dst[i] = acc[i];
                if (s == 0) {
                    s_key[wv][2 * g] = open_key;
                    s_ext[wv][2 * g] = (g == 0) ? 1 : 0;
                }
            } else if (lane_on) {
                float v[RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) v[i] = acc[i] * oscale;
                store_cols<RPL>(p.out, open_key, ld, c, v);
            }
        };

        // lane s of a group holds the metadata of nonzero gs + t*LPR + s; the
        // next tile's metadata is loaded while this tile's rows are in flight
        const int ntiles = (int)(Lg / TS);
        // lane s holds nonzeros base + m*LPR + s, m < MPL
        int m_key[MPL], m_idx[MPL][NIN];
        float m_val[MPL];
        auto load_meta = [&](int t, int (&key)[MPL], int (&ix)[MPL][NIN], float (&v)[MPL]) {
#pragma unroll
            for (int m = 0; m < MPL; ++m) {
                key[m] = 0;
                v[m] = 0.f;
#pragma unroll
                for (int w = 0; w < NIN; ++w) ix[m][w] = 0;
                const int64_t mp = gs + (int64_t)t * TS + m * LPR + s;
                if (gon && t < ntiles && mp < ge) {
                    key[m] = __builtin_nontemporal_load(p.out_idx + mp);
#pragma unroll
                    for (int w = 0; w < NIN; ++w) ix[m][w] = __builtin_nontemporal_load(p.in_idx[w] + mp);
                    v[m] = __builtin_nontemporal_load(p.val + mp);
                }
            }
        };
        load_meta(0, m_key, m_idx, m_val);
        for (int t = 0; t < ntiles; ++t) {
            const int64_t base = gs + (int64_t)t * TS;
            int n_key[MPL], n_idx[MPL][NIN];
            float n_val[MPL];
#pragma unroll 1
            for (int jb = 0; jb < NB; ++jb) {
                typename RowT::Raw raw[U][NIN];
                typename OwnRow::Raw own[U];
                int keys[U];
                float vals[U];
                bool valid[U];
                // issue every gather of the batch first (idle slots read row 0)
                static_for<U>([&](auto ju) {
                    constexpr int JU = decltype(ju)::value;
                    constexpr int M = (NB == 1) ? JU / LPR : 0;   // which of the lane's nonzeros
                    constexpr int JL = (NB == 1) ? JU % LPR : JU; // which lane of the group
                    valid[ju] = gon && (base + jb * U + JU < ge);
                    keys[ju] = tile_bcast<LPR, U, NB, JL>(m_key[M], jb, lane);
                    vals[ju] = tile_bcast_f<LPR, U, NB, JL>(m_val[M], jb, lane);
#pragma unroll
                    for (int w = 0; w < NIN; ++w) {
                        const int ix = tile_bcast<LPR, U, NB, JL>(m_idx[M][w], jb, lane);
                        if constexpr (VEC) raw[ju][w] = RowT::load(lbase[w], ix, rb);
                        else raw[ju][w] = lane_on ? RowT::load(lbase[w], ix, rb) : RowT::zero();
                    }
                    if constexpr (KIND == 1) {
                        if constexpr (VEC) own[ju] = OwnRow::load(obase, keys[ju], rb_own);
                        else own[ju] = lane_on ? OwnRow::load(obase, keys[ju], rb_own) : OwnRow::zero();
                    }
                });
                if (jb == 0) load_meta(t + 1, n_key, n_idx, n_val);
                static_for<U>([&](auto ju) {
                    float prod[RPL];
                    {
                        float r0[RPL];
                        RowT::unpack(raw[ju][0], r0);
#pragma unroll
                        for (int i = 0; i < RPL; ++i) prod[i] = r0[i];
                    }
#pragma unroll
                    for (int w = 1; w < NIN; ++w) {
                        float rw[RPL];
                        RowT::unpack(raw[ju][w], rw);
#pragma unroll
                        for (int i = 0; i < RPL; ++i) prod[i] *= rw[i];
                    }
                    float coef = vals[ju];
                    if constexpr (KIND == 1) {
                        float ow[RPL];
                        OwnRow::unpack(own[ju], ow);
                        float part = 0.f;
#pragma unroll
                        for (int i = 0; i < RPL; ++i) part = fmaf(prod[i], ow[i], part);
                        coef = vals[ju] - group_sum<LPR>(part);
                    }
                    if (valid[ju]) {
                        const int key = keys[ju];
                        if (key != open_key) {
                            flush_mid();
                            if (lane_on && key - open_key - 1 > 0 && key - open_key - 1 < kGapInKernel)
                                zero_rows<RPL>(p.out, open_key + 1, key, ld, c);
#pragma unroll
                            for (int i = 0; i < RPL; ++i) acc[i] = 0.f;
                            open_key = key;
                            open_first = false;
                        }
#pragma unroll
                        for (int i = 0; i < RPL; ++i) acc[i] = fmaf(coef, prod[i], acc[i]);
                    }
                });
            }
#pragma unroll
            for (int m = 0; m < MPL; ++m) {
                m_key[m] = n_key[m];
                m_val[m] = n_val[m];
#pragma unroll
                for (int w = 0; w < NIN; ++w) m_idx[m][w] = n_idx[m][w];
            }
        }

        // end of the run: the open segment
        if (gon) {
            const int nextk = ge < p.nnz ? p.out_idx[ge] : -1;
            const bool right_shared = (nextk == open_key);
            if ((open_first && left_shared) || right_shared) {
                float* dst = &s_acc[wv][2 * g + 1][s * RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) dst[i] = acc[i];
                if (s == 0) {
                    s_key[wv][2 * g + 1] = open_key;
                    s_ext[wv][2 * g + 1] = ((open_first && left_shared && g == 0) ? 1 : 0) |
                                           ((right_shared && ge == ce) ? 2 : 0);
                }
                parked = true;
            } else if (lane_on) {
                float v[RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) v[i] = acc[i] * oscale;
                store_cols<RPL>(p.out, open_key, ld, c, v);
            }
            if (ge == p.nnz && lane_on && p.rows - open_key - 1 > 0 && p.rows - open_key - 1 < kGapInKernel)
                zero_rows<RPL>(p.out, open_key + 1, p.rows, ld, c);
        }

        // combine the parked pieces of rows that cross group boundaries
        if (__builtin_amdgcn_ballot_w64(parked) != 0) {
            wave_lds_sync();
            if (g == 0) {
                int cur = -1, cur_ext = 0;
                float cacc[RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) cacc[i] = 0.f;
                auto emit = [&]() {
                    if (cur < 0 || !lane_on) return;
                    float v[RPL];
#pragma unroll
                    for (int i = 0; i < RPL; ++i) v[i] = cacc[i] * oscale;
                    if (cur_ext) atomic_cols<RPL>(p.out, cur, ld, c, v);
                    else store_cols<RPL>(p.out, cur, ld, c, v);
                };
                for (int q = 0; q < 2 * G; ++q) {
                    const int k = s_key[wv][q];
                    if (k < 0) continue;
                    const float* src = &s_acc[wv][q][s * RPL];
                    if (k != cur) {
                        emit();
                        cur = k;
                        cur_ext = s_ext[wv][q];
#pragma unroll
                        for (int i = 0; i < RPL; ++i) cacc[i] = src[i];
                    } else {
                        cur_ext |= s_ext[wv][q];
#pragma unroll
                        for (int i = 0; i < RPL; ++i) cacc[i] += src[i];
                    }
                }
                emit();
            }
            wave_lds_sync();
        }
    }
}

// ----------------------------------------------------- pipelined MTTKRP kernel
// Same work decomposition and output rules as mttkrp_kernel, with the memory
// accesses software-pipelined:
//  * the nonzero metadata of tile tau+2 is loaded (VGPRs) while tile tau is
//    processed and parked in a 2-slot LDS ring at the start of tile tau+1, so
//    its latency is hidden behind at least two batches of work;
//  * the factor-row gathers of batch q+1 are issued before batch q is
//    consumed (two register buffers), so a wave always has a batch in flight.
// A tile is TS >= 2U nonzeros per group, a batch U nonzeros per group.
template <int NIN, int LPR, int RPL, typename T, int KIND>
__global__ void __launch_bounds__(kBlock) AMPED_OCCUPANCY mttkrp_pipe_kernel(const KParams p)
{
    constexpr int G = 64 / LPR;
    constexpr int RT = LPR * RPL;
    constexpr int UMAX = (NIN <= 2) ? AMPED_UMAX : (AMPED_UMAX + 1) / 2;
    constexpr int U = UMAX;                                      // nonzeros per group per batch
    constexpr int TS = (4 * LPR > 2 * U) ? 4 * LPR : 2 * U;      // nonzeros per group per tile
    constexpr int Q4 = TS / (4 * LPR);                           // 16-byte metadata loads per lane and field
    constexpr int NB = TS / U;                                   // batches per tile (even)
    constexpr int NF = NIN + 2;                                  // key, input indices, value
    constexpr bool VEC = RPL > 1;
    // fibers: consecutive nonzeros with the same output index and the same
    // first input index share that input row; it is gathered and multiplied
    // once per fiber (the remaining product is summed over the fiber first)
    constexpr bool FIBER = (KIND == 0) && (NIN >= 2) && (AMPED_FIBER != 0);
    using RowT = Row<T, RPL>;
    using OwnRow = Row<float, (KIND == 1) ? RPL : 1>;
    static_assert(KIND == 0 || std::is_same<T, float>::value, "residual form is fp32 only");
    static_assert(NB % 2 == 0, "batches per tile must be even");

    __shared__ int s_key[kWaves][2 * G];
    __shared__ int s_ext[kWaves][2 * G];
    __shared__ float s_acc[kWaves][2 * G][RT];
    __shared__ int s_meta[kWaves][2][NF][G * TS];               // [slot][field][group*TS + j]

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int g = lane / LPR;
    const int s = lane % LPR;
    const bool lane_on = VEC || (s * RPL < p.ncols);
    const int c = p.col0 + (lane_on ? s * RPL : 0);
    const int64_t ld = VEC ? (int64_t)RT : p.ld;
    const uint64_t rb = (uint64_t)ld * sizeof(T);
    const uint64_t rb_own = (uint64_t)ld * sizeof(float);
    const float oscale = (KIND == 1) ? p.scale : 1.0f;
    const char* lbase[NIN];
#pragma unroll
    for (int w = 0; w < NIN; ++w) lbase[w] = static_cast<const char*>(p.fac[w]) + (int64_t)c * sizeof(T);
    const char* obase = (KIND == 1) ? reinterpret_cast<const char*>(p.own + c) : nullptr;

    for (;;) {
        const int chunk = pop_chunk(p.queue, lane);
        if (chunk >= p.n_chunks) break;
        const int64_t cs = (int64_t)chunk * p.chunk;
        const int64_t ce = min(cs + p.chunk, p.nnz);
        const int64_t Lg = ((ce - cs + G * TS - 1) / (G * TS)) * TS;
        const int64_t gs = cs + g * Lg;
        const int64_t ge = min(gs + Lg, ce);
        const bool gon = gs < ge;
        const int ntiles = (int)(Lg / TS);
        const int nbatch = ntiles * NB;

        if (s == 0) {
            s_key[wv][2 * g] = -1;
            s_key[wv][2 * g + 1] = -1;
        }
        int open_key = -1;
        bool open_first = true;
        bool left_shared = false;
        float acc[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) acc[i] = 0.f;
        if (gon) {
            const int first = p.out_idx[gs];
            const int prev = gs > 0 ? p.out_idx[gs - 1] : -1;
            left_shared = (prev == first);
            if (lane_on && first - prev - 1 > 0 && first - prev - 1 < kGapInKernel)
                zero_rows<RPL>(p.out, prev + 1, first, ld, c);
            open_key = first;
        }
        bool parked = false;
        auto flush_mid = [&]() {
            if (open_first && left_shared) {
                parked = true;
                float* dst = &s_acc[wv][2 * g][s * RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) dst[i] = acc[i];
                if (s == 0) {
                    s_key[wv][2 * g] = open_key;
                    s_ext[wv][2 * g] = (g == 0) ? 1 : 0;
                }
            } else if (lane_on) {
                float v[RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) v[i] = acc[i] * oscale;
                store_cols<RPL>(p.out, open_key, ld, c, v);
            }
        };

        // ---- metadata: VGPR staging -> LDS ring.  Lane s of group g holds
        // nonzeros gs + t*TS + k*4*LPR + 4s .. +3 of each field, read with one
        // 16-byte load when chunk starts are 4-aligned (the layout arrays are
        // padded by 4 entries, so such a load never leaves the allocation).
        const bool vec_meta = (p.chunk & 3) == 0;
        i32x4 vm[Q4][NF];
        auto load_meta = [&](int t) {
#pragma unroll
            for (int kq = 0; kq < Q4; ++kq) {
                const int64_t mp = gs + (int64_t)t * TS + kq * 4 * LPR + 4 * s;
                const bool on = gon && t < ntiles && mp < ge;
                if (vec_meta) {
                    const i32x4 z = {0, 0, 0, 0};
                    vm[kq][0] = on ? __builtin_nontemporal_load(reinterpret_cast<const i32x4*>(p.out_idx + mp)) : z;
#pragma unroll
                    for (int w = 0; w < NIN; ++w)
                        vm[kq][1 + w] = on ? __builtin_nontemporal_load(reinterpret_cast<const i32x4*>(p.in_idx[w] + mp)) : z;
                    vm[kq][NF - 1] = on ? __builtin_nontemporal_load(reinterpret_cast<const i32x4*>(p.val + mp)) : z;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const bool one = gon && t < ntiles && mp + e < ge;
                        vm[kq][0][e] = one ? p.out_idx[mp + e] : 0;
#pragma unroll
                        for (int w = 0; w < NIN; ++w) vm[kq][1 + w][e] = one ? p.in_idx[w][mp + e] : 0;
                        vm[kq][NF - 1][e] = one ? __float_as_int(p.val[mp + e]) : 0;
                    }
                }
            }
        };
        auto park_meta = [&](int slot) {
#pragma unroll
            for (int kq = 0; kq < Q4; ++kq)
#pragma unroll
                for (int f = 0; f < NF; ++f)
                    *reinterpret_cast<i32x4*>(&s_meta[wv][slot][f][g * TS + kq * 4 * LPR + 4 * s]) = vm[kq][f];
            wave_lds_sync();
        };
        auto meta_at = [&](int slot, int f, int j) { return s_meta[wv][slot][f][g * TS + j]; };

        typename RowT::Raw rawA[U][NIN], rawB[U][NIN];
        typename OwnRow::Raw ownA[U], ownB[U];

        // issue the gathers of batch q (idle entries read row 0)
        auto issue = [&](int q, typename RowT::Raw (&raw)[U][NIN], typename OwnRow::Raw (&own)[U], int& fmask) {
            const int t = q / NB;
            const int j0 = (q % NB) * U;
            const int slot = t & 1;
            const int64_t base = gs + (int64_t)t * TS + j0;
            fmask = 0;
            static_for<U>([&](auto ju) {
                constexpr int JU = decltype(ju)::value;
                const bool valid = gon && (base + JU < ge);
                bool fend = true;
                if constexpr (FIBER) {
                    // the next nonzero of the run is in this tile or at the start of the next
                    const bool nvalid = gon && (base + JU + 1 < ge);
                    const int nj = j0 + JU + 1;
                    const int nslot = (nj < TS) ? slot : (slot ^ 1);
                    const int nidx = (nj < TS) ? nj : 0;
                    fend = !nvalid || meta_at(nslot, 0, nidx) != meta_at(slot, 0, j0 + JU) ||
                           meta_at(nslot, 1, nidx) != meta_at(slot, 1, j0 + JU);
                    fmask |= (fend ? 1 : 0) << JU;
                }
#pragma unroll
                for (int w = 0; w < NIN; ++w) {
                    const int ix = valid ? meta_at(slot, 1 + w, j0 + JU) : 0;
                    if (FIBER && w == 0 && !fend) {
                        raw[JU][w] = RowT::zero();
                    } else {
                        if constexpr (VEC) raw[JU][w] = RowT::load(lbase[w], ix, rb);
                        else raw[JU][w] = lane_on ? RowT::load(lbase[w], ix, rb) : RowT::zero();
                    }
                }
                if constexpr (KIND == 1) {
                    const int k = valid ? meta_at(slot, 0, j0 + JU) : 0;
                    if constexpr (VEC) own[JU] = OwnRow::load(obase, k, rb_own);
                    else own[JU] = lane_on ? OwnRow::load(obase, k, rb_own) : OwnRow::zero();
                }
            });
        };

        // consume batch q from its buffers: Hadamard, scale, running row sum
        float facc[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) facc[i] = 0.f;
        auto consume = [&](int q, typename RowT::Raw (&raw)[U][NIN], typename OwnRow::Raw (&own)[U], int fmask) {
            const int t = q / NB;
            const int j0 = (q % NB) * U;
            const int slot = t & 1;
            const int64_t base = gs + (int64_t)t * TS + j0;
            static_for<U>([&](auto ju) {
                constexpr int JU = decltype(ju)::value;
                const bool valid = gon && (base + JU < ge);
                const int key = meta_at(slot, 0, j0 + JU);
                const float val = __int_as_float(meta_at(slot, NF - 1, j0 + JU));
                if constexpr (FIBER) {
                    // facc += val * prod_{w>=1} rows; at a fiber end acc += facc * row_0
                    float prod[RPL];
                    RowT::unpack(raw[JU][1], prod);
#pragma unroll
                    for (int w = 2; w < NIN; ++w) {
                        float rw[RPL];
                        RowT::unpack(raw[JU][w], rw);
#pragma unroll
                        for (int i = 0; i < RPL; ++i) prod[i] *= rw[i];
                    }
                    if (valid) {
                        if (key != open_key) {
                            flush_mid();
                            if (lane_on && key - open_key - 1 > 0 && key - open_key - 1 < kGapInKernel)
                                zero_rows<RPL>(p.out, open_key + 1, key, ld, c);
#pragma unroll
                            for (int i = 0; i < RPL; ++i) acc[i] = 0.f;
                            open_key = key;
                            open_first = false;
                        }
#pragma unroll
                        for (int i = 0; i < RPL; ++i) facc[i] = fmaf(val, prod[i], facc[i]);
                        if ((fmask >> JU) & 1) {
                            float r0[RPL];
                            RowT::unpack(raw[JU][0], r0);
#pragma unroll
                            for (int i = 0; i < RPL; ++i) {
                                acc[i] = fmaf(facc[i], r0[i], acc[i]);
                                facc[i] = 0.f;
                            }
                        }
                    }
                    return;
                }
                float prod[RPL];
                {
                    float r0[RPL];
                    RowT::unpack(raw[JU][0], r0);
#pragma unroll
                    for (int i = 0; i < RPL; ++i) prod[i] = r0[i];
                }
#pragma unroll
                for (int w = 1; w < NIN; ++w) {
                    float rw[RPL];
                    RowT::unpack(raw[JU][w], rw);
#pragma unroll
                    for (int i = 0; i < RPL; ++i) prod[i] *= rw[i];
                }
                float coef = val;
                if constexpr (KIND == 1) {
                    float ow[RPL];
                    OwnRow::unpack(own[JU], ow);
                    float part = 0.f;
#pragma unroll
                    for (int i = 0; i < RPL; ++i) part = fmaf(prod[i], ow[i], part);
                    coef = val - group_sum<LPR>(part);
                }
                if (valid) {
                    if (key != open_key) {
                        flush_mid();
                        if (lane_on && key - open_key - 1 > 0 && key - open_key - 1 < kGapInKernel)
                            zero_rows<RPL>(p.out, open_key + 1, key, ld, c);
#pragma unroll
                        for (int i = 0; i < RPL; ++i) acc[i] = 0.f;
                        open_key = key;
                        open_first = false;
                    }
#pragma unroll
                    for (int i = 0; i < RPL; ++i) acc[i] = fmaf(coef, prod[i], acc[i]);
                }
            });
        };

        if (nbatch > 0) {
            int fA = 0, fB = 0;
            load_meta(0);
            park_meta(0);
            load_meta(1);
            park_meta(1);  // the fiber test of tile 0 looks at the first entry of tile 1
            load_meta(2);
            issue(0, rawA, ownA, fA);
#pragma unroll 1
            for (int q = 0; q < nbatch; q += 2) {
                if ((q % NB) == 0 && q > 0) {
                    // start of tile t = q/NB (t >= 1): tile t+1 goes to the ring, tile t+2 is loaded
                    const int t = q / NB;
                    park_meta((t + 1) & 1);
                    load_meta(t + 2);
                }
                issue(q + 1, rawB, ownB, fB);
                consume(q, rawA, ownA, fA);
                if (q + 2 < nbatch) issue(q + 2, rawA, ownA, fA);
                consume(q + 1, rawB, ownB, fB);
            }
        }

        // end of the run: the open segment
        if (gon) {
            const int nextk = ge < p.nnz ? p.out_idx[ge] : -1;
            const bool right_shared = (nextk == open_key);
            if ((open_first && left_shared) || right_shared) {
                float* dst = &s_acc[wv][2 * g + 1][s * RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) dst[i] = acc[i];
                if (s == 0) {
                    s_key[wv][2 * g + 1] = open_key;
                    s_ext[wv][2 * g + 1] = ((open_first && left_shared && g == 0) ? 1 : 0) |
                                           ((right_shared && ge == ce) ? 2 : 0);
                }
                parked = true;
            } else if (lane_on) {
                float v[RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) v[i] = acc[i] * oscale;
                store_cols<RPL>(p.out, open_key, ld, c, v);
            }
            if (ge == p.nnz && lane_on && p.rows - open_key - 1 > 0 && p.rows - open_key - 1 < kGapInKernel)
                zero_rows<RPL>(p.out, open_key + 1, p.rows, ld, c);
        }

        if (__builtin_amdgcn_ballot_w64(parked) != 0) {
            wave_lds_sync();
            if (g == 0) {
                int cur = -1, cur_ext = 0;
                float cacc[RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) cacc[i] = 0.f;
                auto emit = [&]() {
                    if (cur < 0 || !lane_on) return;
                    float v[RPL];
#pragma unroll
                    for (int i = 0; i < RPL; ++i) v[i] = cacc[i] * oscale;
                    if (cur_ext) atomic_cols<RPL>(p.out, cur, ld, c, v);
                    else store_cols<RPL>(p.out, cur, ld, c, v);
                };
                for (int qq = 0; qq < 2 * G; ++qq) {
                    const int k = s_key[wv][qq];
                    if (k < 0) continue;
                    const float* src = &s_acc[wv][qq][s * RPL];
                    if (k != cur) {
                        emit();
                        cur = k;
                        cur_ext = s_ext[wv][qq];
#pragma unroll
                        for (int i = 0; i < RPL; ++i) cacc[i] = src[i];
                    } else {
                        cur_ext |= s_ext[wv][qq];
#pragma unroll
                        for (int i = 0; i < RPL; ++i) cacc[i] += src[i];
                    }
                }
                emit();
            }
        }
        wave_lds_sync();
    }
}

// ------------------------------------------------------------------ CP loss
// Sum over nonzeros of (val - sum_r prod_w A_w[i_w, r])^2: per-entry work in
// fp32, each squared residual added in fp64 by the group's first lane, one
// fp64 atomic per wave.
template <int NIN, int LPR, int RPL>
__global__ void __launch_bounds__(kBlock) AMPED_OCCUPANCY cp_loss_kernel(const KParams p)
{
    constexpr int G = 64 / LPR;
    constexpr int RT = LPR * RPL;
    constexpr int UMAX = (NIN <= 2) ? AMPED_UMAX : (AMPED_UMAX + 1) / 2;
    constexpr int MPL = (LPR < UMAX) ? UMAX / LPR : 1;  // nonzeros of metadata per lane
    constexpr int TS = LPR * MPL;                     // nonzeros per group per tile
    constexpr int U = (TS < UMAX) ? TS : UMAX;        // sub-steps per gather batch
    constexpr int NB = TS / U;                        // batches per tile (MPL == 1 if NB > 1)
    constexpr bool VEC = RPL > 1;
    using RowT = Row<float, RPL>;

    const int lane = threadIdx.x & 63;
    const int g = lane / LPR;
    const int s = lane % LPR;
    const bool lane_on = VEC || (s * RPL < p.ncols);
    const int c = p.col0 + (lane_on ? s * RPL : 0);
    const uint64_t rb = (uint64_t)(VEC ? (int64_t)RT : p.ld) * sizeof(float);
    const char* lbase[NIN + 1];
#pragma unroll
    for (int w = 0; w < NIN; ++w) lbase[w] = static_cast<const char*>(p.fac[w]) + (int64_t)c * sizeof(float);
    lbase[NIN] = reinterpret_cast<const char*>(p.own + c);
    double lsum = 0.0;

    for (;;) {
        const int chunk = pop_chunk(p.queue, lane);
        if (chunk >= p.n_chunks) break;
        const int64_t cs = (int64_t)chunk * p.chunk;
        const int64_t ce = min(cs + p.chunk, p.nnz);
        const int64_t Lg = ((ce - cs + G * TS - 1) / (G * TS)) * TS;
        const int64_t gs = cs + g * Lg;
        const int64_t ge = min(gs + Lg, ce);
        const bool gon = gs < ge;
        const int ntiles = (int)(Lg / TS);
        // lane s holds nonzeros base + m*LPR + s, m < MPL
        int m_key[MPL], m_idx[MPL][NIN];
        float m_val[MPL];
        auto load_meta = [&](int t, int (&key)[MPL], int (&ix)[MPL][NIN], float (&v)[MPL]) {
#pragma unroll
            for (int m = 0; m < MPL; ++m) {
                key[m] = 0;
                v[m] = 0.f;
#pragma unroll
                for (int w = 0; w < NIN; ++w) ix[m][w] = 0;
                const int64_t mp = gs + (int64_t)t * TS + m * LPR + s;
                if (gon && t < ntiles && mp < ge) {
                    key[m] = __builtin_nontemporal_load(p.out_idx + mp);
#pragma unroll
                    for (int w = 0; w < NIN; ++w) ix[m][w] = __builtin_nontemporal_load(p.in_idx[w] + mp);
                    v[m] = __builtin_nontemporal_load(p.val + mp);
                }
            }
        };
        load_meta(0, m_key, m_idx, m_val);
        for (int t = 0; t < ntiles; ++t) {
            const int64_t base = gs + (int64_t)t * TS;
            int n_key[MPL], n_idx[MPL][NIN];
            float n_val[MPL];
#pragma unroll 1
            for (int jb = 0; jb < NB; ++jb) {
                typename RowT::Raw raw[U][NIN + 1];
                float vals[U];
                bool valid[U];
                static_for<U>([&](auto ju) {
                    constexpr int JU = decltype(ju)::value;
                    constexpr int M = (NB == 1) ? JU / LPR : 0;
                    constexpr int JL = (NB == 1) ? JU % LPR : JU;
                    valid[ju] = gon && (base + jb * U + JU < ge);
                    vals[ju] = tile_bcast_f<LPR, U, NB, JL>(m_val[M], jb, lane);
                    const int kk = tile_bcast<LPR, U, NB, JL>(m_key[M], jb, lane);
                    if constexpr (VEC) raw[ju][NIN] = RowT::load(lbase[NIN], kk, rb);
                    else raw[ju][NIN] = lane_on ? RowT::load(lbase[NIN], kk, rb) : RowT::zero();
#pragma unroll
                    for (int w = 0; w < NIN; ++w) {
                        const int ix = tile_bcast<LPR, U, NB, JL>(m_idx[M][w], jb, lane);
                        if constexpr (VEC) raw[ju][w] = RowT::load(lbase[w], ix, rb);
                        else raw[ju][w] = lane_on ? RowT::load(lbase[w], ix, rb) : RowT::zero();
                    }
                });
                if (jb == 0) load_meta(t + 1, n_key, n_idx, n_val);
                static_for<U>([&](auto ju) {
                    float prod[RPL];
                    RowT::unpack(raw[ju][NIN], prod);
#pragma unroll
                    for (int w = 0; w < NIN; ++w) {
                        float rw[RPL];
                        RowT::unpack(raw[ju][w], rw);
#pragma unroll
                        for (int i = 0; i < RPL; ++i) prod[i] *= rw[i];
                    }
                    float part = 0.f;
#pragma unroll
                    for (int i = 0; i < RPL; ++i) part += prod[i];
                    const float e = vals[ju] - group_sum<LPR>(part);
                    if (valid[ju] && s == 0) lsum = fma((double)e, (double)e, lsum);
                });
            }
#pragma unroll
            for (int m = 0; m < MPL; ++m) {
                m_key[m] = n_key[m];
                m_val[m] = n_val[m];
#pragma unroll
                for (int w = 0; w < NIN; ++w) m_idx[m][w] = n_idx[m][w];
            }
        }
    }
    // wave sum in fp64, one atomic per wave
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) lsum += __shfl_xor(lsum, m, 64);
    if (lane == 0 && lsum != 0.0) atomicAdd(p.loss, lsum);
}

// ------------------------------------------------------------------ dispatch
using KernelFn = void (*)(const KParams);

// Vector instances: fp32 ranks 16/32/64/128 and bf16 ranks 32/64/128 for up
// to 4 input modes; every other case takes the scalar column-tile path.
constexpr int kMaxVecNin = 4;

#ifndef AMPED_PIPELINE
#define AMPED_PIPELINE 0
#endif
#if AMPED_PIPELINE
#define MTTKRP_KERNEL mttkrp_pipe_kernel
#else
#define MTTKRP_KERNEL mttkrp_kernel
#endif

template <int NIN, typename T, int KIND>
KernelFn pick_vec(int lpr)
{
    constexpr int RPL = 16 / sizeof(T);
    if constexpr (NIN > kMaxVecNin) {
        return nullptr;
    } else {
        switch (lpr) {
        case 4: return MTTKRP_KERNEL<NIN, 4, RPL, T, KIND>;
        case 8: return MTTKRP_KERNEL<NIN, 8, RPL, T, KIND>;
        case 16: return MTTKRP_KERNEL<NIN, 16, RPL, T, KIND>;
        case 32:
            if constexpr (std::is_same<T, float>::value) return MTTKRP_KERNEL<NIN, 32, RPL, T, KIND>;
            else return nullptr;
        default: return nullptr;
        }
    }
}

template <int NIN>
KernelFn pick_mttkrp_nin(FactorType ft, Kind kind, int lpr, bool scalar)
{
    if (kind == Kind::Mttkrp) {
        if (ft == FactorType::F32)
            return scalar ? MTTKRP_KERNEL<NIN, 64, 1, float, 0> : pick_vec<NIN, float, 0>(lpr);
        return scalar ? MTTKRP_KERNEL<NIN, 64, 1, uint16_t, 0> : pick_vec<NIN, uint16_t, 0>(lpr);
    }
    if (ft != FactorType::F32) return nullptr;
    return scalar ? MTTKRP_KERNEL<NIN, 64, 1, float, 1> : pick_vec<NIN, float, 1>(lpr);
}

KernelFn pick_mttkrp(int nin, FactorType ft, Kind kind, int lpr, bool scalar)
{
    switch (nin) {
    case 1: return pick_mttkrp_nin<1>(ft, kind, lpr, scalar);
    case 2: return pick_mttkrp_nin<2>(ft, kind, lpr, scalar);
    case 3: return pick_mttkrp_nin<3>(ft, kind, lpr, scalar);
    case 4: return pick_mttkrp_nin<4>(ft, kind, lpr, scalar);
    case 5: return pick_mttkrp_nin<5>(ft, kind, lpr, scalar);
    case 6: return pick_mttkrp_nin<6>(ft, kind, lpr, scalar);
    case 7: return pick_mttkrp_nin<7>(ft, kind, lpr, scalar);
    default: return nullptr;
    }
}

template <int NIN>
KernelFn pick_loss_nin(int lpr, bool scalar)
{
    if (scalar) return cp_loss_kernel<NIN, 64, 1>;
    if constexpr (NIN > kMaxVecNin) {
        return nullptr;
    } else {
        switch (lpr) {
        case 4: return cp_loss_kernel<NIN, 4, 4>;
        case 8: return cp_loss_kernel<NIN, 8, 4>;
        case 16: return cp_loss_kernel<NIN, 16, 4>;
        case 32: return cp_loss_kernel<NIN, 32, 4>;
        default: return nullptr;
        }
    }
}

KernelFn pick_loss(int nin, int lpr, bool scalar)
{
    switch (nin) {
    case 1: return pick_loss_nin<1>(lpr, scalar);
    case 2: return pick_loss_nin<2>(lpr, scalar);
    case 3: return pick_loss_nin<3>(lpr, scalar);
    case 4: return pick_loss_nin<4>(lpr, scalar);
    case 5: return pick_loss_nin<5>(lpr, scalar);
    case 6: return pick_loss_nin<6>(lpr, scalar);
    case 7: return pick_loss_nin<7>(lpr, scalar);
    default: return nullptr;
    }
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

// Persistent grid size: every CU filled to the kernel's occupancy.
int persistent_grid(KernelFn fn)
{
    static std::mutex mu;
    static std::unordered_map<const void*, int> per_cu;
    static std::unordered_map<int, int> cus;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    auto cit = cus.find(dev);
    if (cit == cus.end()) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cit = cus.emplace(dev, n).first;
    }
    auto it = per_cu.find(reinterpret_cast<const void*>(fn));
    if (it == per_cu.end()) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn), kBlock, 0) !=
                hipSuccess ||
            nb < 1)
            nb = 1;
        it = per_cu.emplace(reinterpret_cast<const void*>(fn), nb).first;
    }
    return it->second * cit->second;
}

hipError_t launch_init(const ModeDev& m, float* out, int64_t ld, int col0, int ncols, double* loss,
                       hipStream_t st)
{
    const int64_t work = std::max<int64_t>(m.n_split * ncols, m.n_gaps * kBlock);
    int grid = (int)std::min<int64_t>(std::max<int64_t>(1, (work + kBlock - 1) / kBlock), 2048);
    hipLaunchKernelGGL(init_kernel, dim3(grid), dim3(kBlock), 0, st, out, ld, col0, ncols, m.split_rows,
                       out ? m.n_split : 0, m.gaps, out ? m.n_gaps : 0, m.queue, loss);
    return hipGetLastError();
}

KParams base_params(const ModeDev& m)
{
    KParams k{};
    k.out_idx = m.out_idx;
    for (int w = 0; w < kMaxIn; ++w) k.in_idx[w] = m.in_idx[w];
    k.val = m.val;
    k.queue = m.queue;
    k.nnz = m.nnz;
    k.chunk = m.chunk;
    k.n_chunks = m.n_chunks;
    k.rows = m.rows;
    return k;
}

// dst[p] = src[perm[p]] for 32-bit words (layout build).
__global__ void __launch_bounds__(kBlock) permute_kernel(uint32_t* dst, const uint32_t* src, const int32_t* perm,
                                                         int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) dst[p] = src[perm[p]];
}

}  // namespace

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
    KernelFn fn = lpr ? pick_mttkrp(a.nin, a.ftype, a.kind, lpr, false) : nullptr;
    const bool scalar = (fn == nullptr);
    // the fused residual form needs the whole row in one launch (rank <= 64
    // on the scalar path)
    if (scalar && a.kind == Kind::ResidualGrad && a.rank > 64) return hipErrorNotSupported;
    if (scalar) fn = pick_mttkrp(a.nin, a.ftype, a.kind, 64, true);
    if (!fn) return hipErrorNotSupported;
    KParams k = base_params(m);
    for (int w = 0; w < a.nin; ++w) k.fac[w] = a.in_factors[w];
    k.own = a.own_factor;
    k.out = a.out;
    k.ld = a.rank;
    k.scale = a.scale;
    const int grid = persistent_grid(fn);
    if (grid <= 0) return hipErrorInvalidDevice;
    const int tile = scalar ? 64 : a.rank;
    for (int col0 = 0; col0 < a.rank; col0 += tile) {
        const int ncols = std::min(tile, a.rank - col0);
        hipError_t e = launch_init(m, a.out, a.rank, col0, ncols, nullptr, a.stream);
        if (e != hipSuccess) return e;
        if (m.n_chunks == 0) continue;
        k.col0 = col0;
        k.ncols = ncols;
        void* args[] = {&k};
        e = hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(grid), dim3(kBlock), args, 0, a.stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_cp_loss(const LossArgs& a)
{
    const ModeDev& m = *a.m;
    const int lpr = vector_lpr(a.rank, 4);
    KernelFn fn = lpr ? pick_loss(a.order - 1, lpr, false) : nullptr;
    const bool scalar = (fn == nullptr);
    if (scalar && a.rank > 64) return hipErrorNotSupported;
    if (scalar) fn = pick_loss(a.order - 1, 64, true);
    if (!fn) return hipErrorNotSupported;
    KParams k = base_params(m);
    for (int w = 0; w < a.order - 1; ++w) k.fac[w] = a.in_factors[w];
    k.own = a.own_factor;
    k.loss = a.loss;
    k.ld = a.rank;
    k.col0 = 0;
    k.ncols = a.rank;
    hipError_t e = launch_init(m, nullptr, 0, 0, 0, a.loss, a.stream);
    if (e != hipSuccess) return e;
    if (m.n_chunks == 0) return hipSuccess;
    const int grid = persistent_grid(fn);
    if (grid <= 0) return hipErrorInvalidDevice;
    void* args[] = {&k};
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(grid), dim3(kBlock), args, 0, a.stream);
}

}  // namespace amped
