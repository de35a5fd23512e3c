#pragma once
// Device code shared by the gfx950 kernel translation units: sparse MTTKRP (Eq. 1, Sec. 2.1), its bfloat16-factor
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
//    consecutive columns of a factor row (16 bytes; 8 for bf16 rows of 32
//    bytes, and of 64 bytes when at most two factors are gathered), so a group
//    loads a whole row with one coalesced access.  Group g walks its own contiguous run of
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
//  * MTTKRP keeps the most-used rows of each input factor in LDS (hot-row
//    cache); their gathers issue no memory request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>

#include "internal.h"

namespace amped {
namespace dev {

constexpr int kBlock = 256;  // init and permute kernels
// MTTKRP kernel blocks: the waves of a block share only the hot-row cache,
// so MTTKRP (which uses it) runs 512-thread blocks, one per CU beside a large
// cache, and the residual and loss forms (whose extra own-row registers leave
// them short of waves otherwise) 256-thread blocks without it.
#ifndef AMPED_BLOCK
#define AMPED_BLOCK 512
#endif
#ifndef AMPED_BLOCK_OWN
#define AMPED_BLOCK_OWN 256
#endif
__host__ __device__ constexpr int mttkrp_block(int kind) { return kind == 0 ? AMPED_BLOCK : AMPED_BLOCK_OWN; }
// The residual and loss forms keep hot rows in LDS too (else MTTKRP only).
#ifndef AMPED_HOT_OWN
#define AMPED_HOT_OWN 0
#endif
__host__ __device__ constexpr bool hot_cache_kind(int kind) { return kind == 0 || AMPED_HOT_OWN != 0; }
// Compile-time knobs, off by default (both measured slower): non-temporal
// output-row stores, and the cache-policy bits of factor-row gathers.
#ifndef AMPED_OUT_NT
#define AMPED_OUT_NT 0
#endif
#ifndef AMPED_GATHER_AUX
#define AMPED_GATHER_AUX 0
#endif
// Diagnostic build: every wave of the MTTKRP-shaped kernels records how many
// chunks and nonzeros it took from the work queue and when it took its first
// chunk and exited (constant-rate wall clock), for the load-balance report.
#ifndef AMPED_QUEUE_STATS
#define AMPED_QUEUE_STATS 0
#endif
constexpr int kMaxIn = kMaxOrder - 1;

// Tuning knobs (compile-time): nonzeros per group whose gathers are issued
// together (MTTKRP, then the residual gradient, with up to 2 input modes; the
// loss and higher orders use the third value), and the waves per SIMD the
// register allocation must allow (0 = compiler's choice).
#ifndef AMPED_UMAX
#define AMPED_UMAX 4
#endif
#ifndef AMPED_UMAX_GRAD
#define AMPED_UMAX_GRAD 4
#endif
#ifndef AMPED_UMAX_OWN
#define AMPED_UMAX_OWN 2
#endif
#ifndef AMPED_UMAX_NIN
#define AMPED_UMAX_NIN 2   // most input modes that still get AMPED_UMAX
#endif
#ifndef AMPED_MIN_WAVES
#define AMPED_MIN_WAVES 0
#endif
// Spread each tile's metadata loads over its batch pairs (see the tile loop).
#ifndef AMPED_META_SPREAD
#define AMPED_META_SPREAD 1
#endif
#if AMPED_MIN_WAVES > 0
#define AMPED_OCCUPANCY __attribute__((amdgpu_waves_per_eu(AMPED_MIN_WAVES)))
#else
#define AMPED_OCCUPANCY
#endif

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

struct KParams {
    const int32_t* out_idx;
    const int32_t* in_idx[kMaxIn];
    const float* val;
    const void* fac[kMaxIn];
    const float* own;
    float* out;
    double* loss;
    unsigned* queue;  // n_stripes counters
    int n_stripes;    // contiguous chunk stripes, one counter each (1..kQueueSlots)
    int64_t nnz, chunk, n_chunks, rows;
    int64_t ld;     // row stride of factors and output, in elements
    int col0;       // first column handled by this launch
    int ncols;      // columns handled by this launch
    float scale;
    uint32_t fbytes[kMaxIn];  // input factor sizes in bytes (buffer addressing)
    uint32_t own_bytes;
    const void* zero_row;     // 16 zero bytes: what padding entries read on the 64-bit path
    float* sink;              // 64 * 8 floats that absorb stores which must not land
    int prev_key;             // output index just before position 0 of these arrays (-1: none)
    int next_key;             // output index just after position nnz - 1 (-1: none)
    const int32_t* hot[kMaxIn];  // per input: direct-mapped table of hot_k rows kept in LDS
    int hot_k;                // LDS row-cache slots per input (power of two; 0 = none)
#if AMPED_QUEUE_STATS
    unsigned long long* qstats;  // per wave: chunks, nonzeros, first-pop and exit times
#endif
};

// Dynamic LDS of the MTTKRP kernel: 16 zero bytes, then (vector path, K > 0)
// the tags [NIN][K] and rows [NIN][K][row bytes] of the hot-row cache.
__host__ __device__ constexpr size_t hot_tag_offset() { return 16; }
__host__ __device__ constexpr size_t hot_row_offset(int nin, int k) { return (16 + (size_t)nin * k * 4 + 15) & ~(size_t)15; }
__host__ __device__ constexpr size_t hot_lds_bytes(int nin, int k, int row_bytes)
{
    return k > 0 ? hot_row_offset(nin, k) + (size_t)nin * k * row_bytes : 16;
}

// Raw buffer resource over [base, base + bytes): word 3 is the gfx9-family
// default for untyped dword access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

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

template <int LPR>
__device__ __forceinline__ float group_sum(float x)
{
#pragma unroll
    for (int m = 1; m < LPR; m <<= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// ------------------------------------------------------------------ row access
// Row<T, RPL>: RPL consecutive columns of a factor row as fp32, read from a
// 64-bit address (load_ptr) or a buffer resource and 32-bit byte offset
// (load_buf, vector forms only).
template <typename T, int RPL> struct Row;


template <> struct Row<float, 4> {
    using Raw = float4;
    // bitwise OR with the same lane's 16 bytes of an LDS row (one side is 0)
    static __device__ __forceinline__ Raw merge_lds(const Raw& a, const char* lds)
    {
        const u32x4 b = *reinterpret_cast<const u32x4*>(lds);
        return make_float4(__uint_as_float(__float_as_uint(a.x) | b.x), __uint_as_float(__float_as_uint(a.y) | b.y),
                           __uint_as_float(__float_as_uint(a.z) | b.z), __uint_as_float(__float_as_uint(a.w) | b.w));
    }
    static __device__ __forceinline__ Raw load_buf(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, AMPED_GATHER_AUX);
        return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
    }
    static __device__ __forceinline__ Raw load_ptr(const char* a) { return *reinterpret_cast<const float4*>(a); }
    static __device__ __forceinline__ void unpack(const Raw& r, float (&v)[4])
    {
        v[0] = r.x; v[1] = r.y; v[2] = r.z; v[3] = r.w;
    }
};

template <> struct Row<uint16_t, 8> {  // bfloat16 bit patterns, widened exactly
    using Raw = uint4;
    static __device__ __forceinline__ Raw merge_lds(const Raw& a, const char* lds)
    {
        const u32x4 b = *reinterpret_cast<const u32x4*>(lds);
        return make_uint4(a.x | b.x, a.y | b.y, a.z | b.z, a.w | b.w);
    }
    static __device__ __forceinline__ Raw load_buf(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, AMPED_GATHER_AUX);
        return make_uint4(v.x, v.y, v.z, v.w);
    }
    static __device__ __forceinline__ Raw load_ptr(const char* a) { return *reinterpret_cast<const uint4*>(a); }
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

template <> struct Row<uint16_t, 4> {  // 4 bfloat16 per lane (rows of up to 64 bytes)
    using Raw = uint2;
    static __device__ __forceinline__ Raw merge_lds(const Raw& a, const char* lds)
    {
        const u32x2 b = *reinterpret_cast<const u32x2*>(lds);
        return make_uint2(a.x | b.x, a.y | b.y);
    }
    static __device__ __forceinline__ Raw load_buf(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, AMPED_GATHER_AUX);
        return make_uint2(v.x, v.y);
    }
    static __device__ __forceinline__ Raw load_ptr(const char* a) { return *reinterpret_cast<const uint2*>(a); }
    static __device__ __forceinline__ void unpack(const Raw& r, float (&v)[4])
    {
        v[0] = __uint_as_float(r.x << 16);
        v[1] = __uint_as_float(r.x & 0xFFFF0000u);
        v[2] = __uint_as_float(r.y << 16);
        v[3] = __uint_as_float(r.y & 0xFFFF0000u);
    }
};

template <> struct Row<float, 1> {
    using Raw = float;
    static __device__ __forceinline__ Raw load_buf(__amdgpu_buffer_rsrc_t, uint32_t) { return 0.f; }
    static __device__ __forceinline__ Raw load_ptr(const char* a) { return *reinterpret_cast<const float*>(a); }
    static __device__ __forceinline__ void unpack(const Raw& r, float (&v)[1]) { v[0] = r; }
};

template <> struct Row<uint16_t, 1> {
    using Raw = uint32_t;
    static __device__ __forceinline__ Raw load_buf(__amdgpu_buffer_rsrc_t, uint32_t) { return 0u; }
    static __device__ __forceinline__ Raw load_ptr(const char* a) { return *reinterpret_cast<const uint16_t*>(a); }
    static __device__ __forceinline__ void unpack(const Raw& r, float (&v)[1]) { v[0] = __uint_as_float(r << 16); }
};

// Output row pieces: RPL fp32 columns of row `row`, starting at column c.
template <int RPL>
__device__ __forceinline__ void store_vec(float* p, const float (&v)[RPL]);
template <int RPL>
__device__ __forceinline__ void store_cols(float* out, int64_t row, int64_t ld, int c, const float (&v)[RPL])
{
    store_vec<RPL>(out + row * ld + c, v);
}

template <int RPL>
__device__ __forceinline__ void atomic_cols(float* out, int64_t row, int64_t ld, int c, const float (&v)[RPL])
{
    float* p = out + row * ld + c;
#pragma unroll
    for (int i = 0; i < RPL; ++i) atomicAdd(p + i, v[i]);
}

// RPL fp32 values of an output row to a lane's own address.
template <int RPL>
__device__ __forceinline__ void store_vec(float* p, const float (&v)[RPL])
{
    if constexpr (RPL % 4 == 0) {
#pragma unroll
        for (int i = 0; i < RPL; i += 4) {
            const f32x4 x = {v[i], v[i + 1], v[i + 2], v[i + 3]};
            if constexpr (AMPED_OUT_NT != 0) __builtin_nontemporal_store(x, reinterpret_cast<f32x4*>(p + i));
            else *reinterpret_cast<f32x4*>(p + i) = x;
        }
    } else {
#pragma unroll
        for (int i = 0; i < RPL; ++i) p[i] = v[i];
    }
}
template <int RPL>
__device__ __forceinline__ void lds_store(float* p, const float (&v)[RPL])
{
    if constexpr (RPL % 4 == 0) {
#pragma unroll
        for (int i = 0; i < RPL; i += 4)
            *reinterpret_cast<float4*>(p + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < RPL; ++i) p[i] = v[i];
    }
}

// U consecutive ints of an LDS ring row (16-byte aligned when U % 4 == 0,
// 8-byte aligned when U == 2) with the widest reads that fit.
template <int U>
__device__ __forceinline__ void lds_vec(const int* p, int (&v)[U])
{
    if constexpr (U % 4 == 0) {
#pragma unroll
        for (int i = 0; i < U; i += 4) {
            const i32x4 x = *reinterpret_cast<const i32x4*>(p + i);
            v[i] = x.x; v[i + 1] = x.y; v[i + 2] = x.z; v[i + 3] = x.w;
        }
    } else if constexpr (U == 2) {
        const int2 x = *reinterpret_cast<const int2*>(p);
        v[0] = x.x; v[1] = x.y;
    } else {
#pragma unroll
        for (int i = 0; i < U; ++i) v[i] = p[i];
    }
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work queue.  The chunks are split into S contiguous stripes, each with its
// own counter.  A wave starts on stripe `home` and moves on to the next stripe
// when one runs dry, so with one stripe per XCD the consecutive chunks of a
// stripe (neighbouring output rows; for a heavy row, neighbouring input
// indices) are taken by one XCD's CUs while any chunk is left on its stripe,
// and no CU idles while any chunk is left anywhere.  With S = 1 this is one
// global counter.  A wave reads each counter at most once past the end of its
// stripe, so a counter never exceeds the stripe's chunks plus the waves of the
// grid (below 2^32: chunks < 2^31), and it is compared as unsigned.
struct ChunkQueue {
    unsigned* q;
    int64_t n_chunks;
    int S, home, tried = 0;
    int64_t b0 = 0, b1 = 0;   // current stripe's chunk range

    __device__ __forceinline__ ChunkQueue(unsigned* q_, int64_t n, int stripes, int home_)
        : q(q_), n_chunks(n), S(stripes), home(home_)
    {
        set_stripe();
    }
    __device__ __forceinline__ void set_stripe()
    {
        const int x = (home + tried) % S;
        b0 = (int64_t)x * n_chunks / S;
        b1 = (int64_t)(x + 1) * n_chunks / S;
    }
    // next chunk, or -1 when every stripe is exhausted (wave-uniform)
    __device__ __forceinline__ int64_t pop(int lane)
    {
        while (tried < S) {
            unsigned c = 0;
            if (lane == 0) c = atomicAdd(q + (home + tried) % S, 1u);
            c = (unsigned)__builtin_amdgcn_readfirstlane((int)c);
            if ((int64_t)c < b1 - b0) return b0 + (int64_t)c;
            if (++tried < S) set_stripe();
        }
        return -1;
    }
};

// --------------------------------------------------------------- MTTKRP kernel
// KIND 0: MTTKRP.  KIND 1: scale * MTTKRP of the residuals val - CP model,
// recomputed per nonzero from all factor rows.  KIND 2: the sparse CP loss,
// sum over nonzeros of (val - CP model)^2 (per-entry work in fp32, each
// squared residual added in fp64, one fp64 atomic per wave; no output
// matrix).  KIND 3: KIND 1 and KIND 2 in one pass (every mode's layout holds
// every nonzero, so the residuals the gradient computes give the loss too).
//
// Memory accesses are software-pipelined:
//  * the nonzero metadata of tile tau+2 is loaded (VGPRs) while tile tau is
//    processed and parked in a 2-slot LDS ring at the start of tile tau+1, so
//    its latency is hidden behind at least two batches of work;
//  * the factor-row gathers of batch q+1 are issued before batch q is
//    consumed (two register buffers), so a wave always has a batch in flight.
// A tile is TS >= 2U nonzeros per group, a batch U nonzeros per group.
//
// The inner loop has no per-nonzero bounds test: ring entries past the end of
// a group's run are padding that carries the run's last output index, a zero
// value and the row index -1, whose gather returns zeros (past the end of the
// buffer resource, or redirected to a zero row on the 64-bit path).  Padding
// therefore adds exact zeros to the open row and never starts a new one.
template <int NIN, int LPR, int RPL, typename T, int KIND, bool BUF>
__global__ void __launch_bounds__(mttkrp_block(KIND)) AMPED_OCCUPANCY mttkrp_kernel(const KParams p)
{
    constexpr int kMttkrpBlock = mttkrp_block(KIND);
    constexpr int kWaves = kMttkrpBlock / 64;
    constexpr int G = 64 / LPR;
    constexpr int RT = LPR * RPL;
    // nonzeros per group per batch: the loss and high orders keep fewer rows
    // in flight per batch
    constexpr int U = (KIND != 2 && NIN <= AMPED_UMAX_NIN) ? (KIND == 0 ? AMPED_UMAX : AMPED_UMAX_GRAD)
                                                          : AMPED_UMAX_OWN;
    constexpr bool GRAD = KIND == 1 || KIND == 3;                // residual gradient: output scaled by p.scale
    constexpr bool LOSS = KIND == 2 || KIND == 3;                // squared residuals summed into p.loss
    constexpr int TS = (4 * LPR > 2 * U) ? 4 * LPR : 2 * U;      // nonzeros per group per tile
    constexpr int Q4 = TS / (4 * LPR);                           // 16-byte metadata loads per lane and field
    constexpr int NB = TS / U;                                   // batches per tile (even)
    constexpr int NF = NIN + 2;                                  // key, input indices, value
    constexpr int FS = G * TS;                                   // ring entries per field
    constexpr bool VEC = RPL > 1;
    using RowT = Row<T, RPL>;
    constexpr bool OWN = KIND >= 1;                              // the output mode's row is read too
    constexpr bool OUT = KIND != 2;                              // an output matrix is written
    using OwnRow = Row<float, OWN ? RPL : 1>;
    constexpr int kMetaNT = 2;                                   // non-temporal cache policy
    static_assert(KIND == 0 || std::is_same<T, float>::value, "residual and loss forms are fp32 only");
    static_assert(NB % 2 == 0, "batches per tile must be even");
    static_assert(TS % 4 == 0 && (U == 1 || U == 2 || U % 4 == 0), "ring rows must be vector aligned");
    static_assert(!BUF || VEC, "buffer addressing is for the vector path");

    __shared__ int s_key[kWaves][2 * G];
    __shared__ int s_ext[kWaves][2 * G];
    __shared__ __align__(16) float s_acc[kWaves][2 * G][RT];    // slot 2g+1 is also the in-loop park sink
    __shared__ __align__(16) int s_meta[kWaves][2][NF][FS];     // [slot][field][group*TS + j]

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int g = lane / LPR;
    const int s = lane % LPR;
    const bool lane_on = VEC || (s * RPL < p.ncols);
    const int c = p.col0 + (lane_on ? s * RPL : 0);
    const int64_t ld = VEC ? (int64_t)RT : p.ld;
    const uint64_t rb = (uint64_t)ld * sizeof(T);
    const uint64_t rb_own = (uint64_t)ld * sizeof(float);
    const float oscale = GRAD ? p.scale : 1.0f;
    const char* lbase[NIN];
#pragma unroll
    for (int w = 0; w < NIN; ++w) lbase[w] = static_cast<const char*>(p.fac[w]) + (int64_t)c * sizeof(T);
    const char* obase = OWN ? reinterpret_cast<const char*>(p.own + c) : nullptr;
    const char* zrow = static_cast<const char*>(p.zero_row);
    float* const gsink = p.sink + s * RPL;
    double lsum = 0.0;  // LOSS: sum of squared residuals (each group's value in all its LPR lanes)
    // BUF: every factor is below 4 GiB, so rows are read with buffer loads
    // addressed by a 32-bit byte offset (row * row_bytes + column bytes)
    __amdgpu_buffer_rsrc_t rsrc[NIN];
    __amdgpu_buffer_rsrc_t rsrc_own;
    const uint32_t cb = (uint32_t)c * (uint32_t)sizeof(T);
    const uint32_t cb_own = (uint32_t)c * (uint32_t)sizeof(float);
    if constexpr (BUF) {
#pragma unroll
        for (int w = 0; w < NIN; ++w) rsrc[w] = make_rsrc(p.fac[w], p.fbytes[w]);
        if constexpr (OWN) rsrc_own = make_rsrc(p.own, p.own_bytes);
    }
    // Hot-row cache (vector path): the K rows of each input factor named by
    // the direct-mapped table p.hot[w] are copied to LDS once per block; ring
    // entries that name a cached row are rewritten to -2 - slot when parked.
    extern __shared__ __align__(16) char s_dyn[];
    constexpr int RB = RT * (int)sizeof(T);  // row bytes on the vector path
    const int K = (VEC && hot_cache_kind(KIND)) ? p.hot_k : 0;
    const int* const htag = reinterpret_cast<const int*>(s_dyn + hot_tag_offset());
    const uint32_t hrow = (uint32_t)hot_row_offset(NIN, K);  // byte offset of the cached rows
    {
        if (threadIdx.x < 4) reinterpret_cast<int*>(s_dyn)[threadIdx.x] = 0;
        if constexpr (VEC && hot_cache_kind(KIND)) {
            if (K > 0) {
                int* tag = reinterpret_cast<int*>(s_dyn + hot_tag_offset());
#pragma unroll
                for (int w = 0; w < NIN; ++w) {
                    for (int i = threadIdx.x; i < K; i += kMttkrpBlock) tag[w * K + i] = p.hot[w][i];
                    constexpr int PR = RB / 16;   // 16-byte pieces per row
                    for (int i = threadIdx.x; i < K * PR; i += kMttkrpBlock) {
                        const int slot = i / PR, piece = i % PR;
                        const int row = p.hot[w][slot];
                        u32x4 v = {0u, 0u, 0u, 0u};
                        if (row >= 0)
                            v = *reinterpret_cast<const u32x4*>(static_cast<const char*>(p.fac[w]) +
                                                                 (uint64_t)row * RB + piece * 16);
                        *reinterpret_cast<u32x4*>(s_dyn + hrow + ((size_t)w * K + slot) * RB + piece * 16) = v;
                    }
                }
            }
        }
        __syncthreads();
    }
    // one factor-row gather: row >= 0 from memory, -1 (padding) zeros, <= -2
    // cache slot -2 - row from LDS (its memory read then returns zeros: past
    // the buffer's end, or the zero row on the 64-bit path)
    auto gather = [&](int w, int ix) -> typename RowT::Raw {
        typename RowT::Raw r;
        if constexpr (BUF) r = RowT::load_buf(rsrc[w], (uint32_t)max(ix, -1) * (uint32_t)rb + cb);
        else r = RowT::load_ptr(ix < 0 ? zrow : lbase[w] + (uint64_t)(uint32_t)ix * rb);
        if constexpr (VEC && hot_cache_kind(KIND)) {
            constexpr uint32_t LB = RPL * sizeof(T);   // bytes per lane
            const uint32_t la = ix <= -2 ? hrow + (uint32_t)(w * K + (-2 - ix)) * RB + (uint32_t)s * LB : 0u;
            r = RowT::merge_lds(r, s_dyn + la);
        }
        return r;
    };
    auto gather_own = [&](int k) -> typename OwnRow::Raw {
        if constexpr (BUF) return OwnRow::load_buf(rsrc_own, (uint32_t)k * (uint32_t)rb_own + cb_own);
        else return OwnRow::load_ptr(k < 0 ? zrow : obase + (uint64_t)(uint32_t)k * rb_own);
    };
    const bool vec_meta = (p.chunk & 3) == 0;

#if AMPED_QUEUE_STATS
    unsigned long long st_chunks = 0, st_nnz = 0, st_first = 0;
#endif
    ChunkQueue cq(p.queue, p.n_chunks, p.n_stripes, (int)(blockIdx.x % (unsigned)p.n_stripes));
    for (;;) {
        const int64_t chunk = cq.pop(lane);
        if (chunk < 0) break;
        const int64_t cs = chunk * p.chunk;
        const int clen = (int)(min(cs + p.chunk, p.nnz) - cs);
#if AMPED_QUEUE_STATS
        if (st_chunks == 0) st_first = (unsigned long long)wall_clock64();
        ++st_chunks;
        st_nnz += (unsigned long long)clen;
#endif
        const int Lg = ((clen + FS - 1) / FS) * TS;            // run length per group, whole tiles
        const int goff = g * Lg;                                // group's first position in the chunk
        const int len = max(0, min(Lg, clen - goff));           // nonzeros in the group's run
        const bool gon = len > 0;
        const int ntiles = Lg / TS;
        const int nbatch = ntiles * NB;
        const int64_t gs = cs + goff;
        const int64_t ge = gs + len;
        // metadata of this chunk as buffers over [cs, cs + clen rounded up to
        // 4); reads past that return zeros, so no load needs a bounds branch
        const uint32_t mbytes = (uint32_t)((clen + 3) & ~3) * 4u;
        __amdgpu_buffer_rsrc_t mr[NF];
        mr[0] = make_rsrc(p.out_idx + cs, mbytes);
#pragma unroll
        for (int w = 0; w < NIN; ++w) mr[1 + w] = make_rsrc(p.in_idx[w] + cs, mbytes);
        mr[NF - 1] = make_rsrc(p.val + cs, mbytes);

        int open_key = -1, last_key = -1;
        int first_open = 1;  // the open row is the run's first
        int lsh = 0;         // the run's first row continues from the previous position
        float acc[RPL];
        float cur_own[RPL];  // own row of the entry consumed last (forms that read it)
        int own_key = -1;
#pragma unroll
        for (int i = 0; i < RPL; ++i) acc[i] = cur_own[i] = 0.f;
        if constexpr (OUT) {
            if (gon) {
                const int first = p.out_idx[gs];
                const int prev = gs > 0 ? p.out_idx[gs - 1] : p.prev_key;
                last_key = p.out_idx[ge - 1];
                lsh = (prev == first) ? 1 : 0;
                open_key = first;
            }
            // slot 2g: the run's first row when it continues from the left
            // (bit 0: from the previous chunk); slot 2g+1: the run's last row
            if (s == 0) {
                s_key[wv][2 * g] = lsh ? open_key : -1;
                s_ext[wv][2 * g] = (g == 0) ? 1 : 0;
                s_key[wv][2 * g + 1] = -1;
            }
        }

        // ---- metadata: VGPR staging -> LDS ring.  Lane s of group g holds
        // nonzeros gs + t*TS + k*4*LPR + 4s .. +3 of each field, read with one
        // 16-byte load when chunk starts are 4-aligned.
        i32x4 vm[Q4][NF];
        auto load_meta = [&](int t) {
            if (t < ntiles) {
#pragma unroll
                for (int kq = 0; kq < Q4; ++kq) {
                    const uint32_t off = (uint32_t)(goff + t * TS + kq * 4 * LPR + 4 * s) * 4u;
                    if (vec_meta) {
#pragma unroll
                        for (int f = 0; f < NF; ++f) {
                            const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(mr[f], (int)off, 0, kMetaNT);
                            vm[kq][f] = i32x4{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
                        }
                    } else {
#pragma unroll
                        for (int f = 0; f < NF; ++f)
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                vm[kq][f][e] = (int)__builtin_amdgcn_raw_buffer_load_b32(mr[f], (int)(off + 4 * e), 0,
                                                                                         kMetaNT);
                    }
                }
            } else {
#pragma unroll
                for (int kq = 0; kq < Q4; ++kq)
#pragma unroll
                    for (int f = 0; f < NF; ++f) vm[kq][f] = i32x4{0, 0, 0, 0};
            }
        };
        // Items [L0, L1) of tile t's metadata (item l = 16-byte load kq = l / NF
        // of field l % NF), issued whatever t is: past the last tile the offset
        // is pushed out of the buffer (2^30 >= any chunk's metadata bytes), so
        // the loads return zeros and cost no memory traffic.
        auto load_meta_part = [&](int t, auto l0, auto l1) {
            constexpr int L0 = decltype(l0)::value, L1 = decltype(l1)::value;
            const uint32_t bias = t < ntiles ? 0u : (1u << 30);
            static_for<L1 - L0>([&](auto li) {
                constexpr int l = L0 + decltype(li)::value;
                constexpr int kq = l / NF, f = l % NF;
                const uint32_t off = (uint32_t)(goff + t * TS + kq * 4 * LPR + 4 * s) * 4u + bias;
                if (vec_meta) {
                    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(mr[f], (int)off, 0, kMetaNT);
                    vm[kq][f] = i32x4{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        vm[kq][f][e] = (int)__builtin_amdgcn_raw_buffer_load_b32(mr[f], (int)(off + 4 * e), 0, kMetaNT);
                }
            });
        };
        // tile t to ring slot t & 1, entries past the end of the run padded
        // here (a tile after its loads were issued, so they have landed)
        auto park_meta = [&](int t) {
#pragma unroll
            for (int kq = 0; kq < Q4; ++kq) {
                const int rel = t * TS + kq * 4 * LPR + 4 * s;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const bool pad = rel + e >= len;
                    vm[kq][0][e] = pad ? last_key : vm[kq][0][e];
#pragma unroll
                    for (int w = 0; w < NIN; ++w) vm[kq][1 + w][e] = pad ? -1 : vm[kq][1 + w][e];
                    vm[kq][NF - 1][e] = pad ? 0 : vm[kq][NF - 1][e];
                }
                if constexpr (VEC && hot_cache_kind(KIND)) {
                    if (K > 0) {
                        // rows held in the LDS cache become -2 - slot (tags
                        // are rows or -2, so padding -1 never matches)
#pragma unroll
                        for (int w = 0; w < NIN; ++w)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int ix = vm[kq][1 + w][e];
                                const int slot = ix & (K - 1);
                                vm[kq][1 + w][e] = (htag[w * K + slot] == ix) ? -2 - slot : ix;
                            }
                    }
                }
#pragma unroll
                for (int f = 0; f < NF; ++f)
                    *reinterpret_cast<i32x4*>(&s_meta[wv][t & 1][f][g * TS + kq * 4 * LPR + 4 * s]) = vm[kq][f];
            }
            wave_lds_sync();
        };

        typename RowT::Raw rawA[U][NIN], rawB[U][NIN];
        typename OwnRow::Raw ownA[U], ownB[U];

        // issue the gathers of batch q
        auto issue = [&](int q, typename RowT::Raw (&raw)[U][NIN], typename OwnRow::Raw (&own)[U]) {
            const int t = q / NB;
            const int j0 = (q % NB) * U;
            const int* mrow = &s_meta[wv][t & 1][0][g * TS + j0];
            int ix[NIN][U];
#pragma unroll
            for (int w = 0; w < NIN; ++w) lds_vec<U>(mrow + (1 + w) * FS, ix[w]);
            int kk[U];
            int kprev = 0;   // key of the entry before the batch (same tile)
            if constexpr (OWN) {
                lds_vec<U>(mrow, kk);
                kprev = mrow[j0 > 0 ? -1 : 0];
            }
#pragma unroll
            for (int ju = 0; ju < U; ++ju) {
#pragma unroll
                for (int w = 0; w < NIN; ++w) raw[ju][w] = gather(w, ix[w][ju]);
                if constexpr (OWN) {
                    // the own row is read where the key changes (and at a
                    // tile's first entry); elsewhere consume reuses the row
                    // it holds.  Lanes that need none load at -1 (zeros), and
                    // when no group of the wave needs one the load instruction
                    // is skipped altogether (a wave-uniform branch, so the
                    // address unit does no work for it)
                    const bool same = j0 + ju > 0 && kk[ju] == (ju == 0 ? kprev : kk[ju > 0 ? ju - 1 : 0]);
                    const bool need = !(ix[0][ju] == -1 || same);   // -1: padding
                    if (__builtin_amdgcn_ballot_w64(need) != 0) own[ju] = gather_own(need ? kk[ju] : -1);
                    else own[ju] = typename OwnRow::Raw{};
                }
            }
        };

        // a finished row: stored, or parked in LDS when it is the run's first
        // row and continues from the left (the store then goes to a sink).
        // Unneeded parks go to slot 2g+1, which is only filled at the run's end.
        auto flush = [&]() {
            const bool pk = (first_open & lsh) != 0;
            float* lp = &s_acc[wv][2 * g + (pk ? 0 : 1)][s * RPL];
            lds_store<RPL>(lp, acc);
            float v[RPL];
#pragma unroll
            for (int i = 0; i < RPL; ++i) v[i] = acc[i] * oscale;
            float* gp = (pk || !lane_on) ? gsink : p.out + (int64_t)open_key * ld + c;
            store_vec<RPL>(gp, v);
        };

        // consume batch q from its buffers: Hadamard, scale, running row sum
        auto consume = [&](int q, typename RowT::Raw (&raw)[U][NIN], typename OwnRow::Raw (&own)[U]) {
            const int t = q / NB;
            const int j0 = (q % NB) * U;
            const int* mrow = &s_meta[wv][t & 1][0][g * TS + j0];
            int key[U], vbits[U];
            if constexpr (OUT || OWN) lds_vec<U>(mrow, key);
            lds_vec<U>(mrow + (NF - 1) * FS, vbits);
#pragma unroll
            for (int ju = 0; ju < U; ++ju) {
                const float val = __int_as_float(vbits[ju]);
                float prod[RPL];
                RowT::unpack(raw[ju][0], prod);
#pragma unroll
                for (int w = 1; w < NIN; ++w) {
                    float rw[RPL];
                    RowT::unpack(raw[ju][w], rw);
#pragma unroll
                    for (int i = 0; i < RPL; ++i) prod[i] *= rw[i];
                }
                float coef = val;
                if constexpr (OWN) {
                    // same rule as in issue: a fresh row where the key changes
                    // or the tile starts, else the row of the previous entry
                    const bool fresh = j0 + ju == 0 || key[ju] != own_key;
                    float ow[RPL];
                    OwnRow::unpack(own[ju], ow);
#pragma unroll
                    for (int i = 0; i < RPL; ++i) cur_own[i] = fresh ? ow[i] : cur_own[i];
                    own_key = key[ju];
                    float part = 0.f;
#pragma unroll
                    for (int i = 0; i < RPL; ++i) part = fmaf(prod[i], cur_own[i], part);
                    if constexpr (!VEC) part = lane_on ? part : 0.f;
                    coef = val - group_sum<LPR>(part);
                }
                if constexpr (LOSS) lsum = fma((double)coef, (double)coef, lsum);
                if constexpr (OUT) {
                    if (key[ju] != open_key) {
                        flush();
#pragma unroll
                        for (int i = 0; i < RPL; ++i) acc[i] = 0.f;
                        open_key = key[ju];
                        first_open = 0;
                    }
#pragma unroll
                    for (int i = 0; i < RPL; ++i) acc[i] = fmaf(coef, prod[i], acc[i]);
                }
            }
        };

        // With at most 8 batch pairs per tile, the tile is unrolled and the
        // loads of tile t+2's metadata are spread over its batch pairs at
        // fixed places, so every pass of the tile loop issues the same loads
        // and the compiler's load-counter waits are exact; otherwise tile
        // t+2 is loaded at once at the start of tile t.
        constexpr int IT = NB / 2;
        constexpr bool SPREAD = AMPED_META_SPREAD != 0 && IT <= 8;
        if (SPREAD && nbatch > 0) {
            constexpr int NL = Q4 * NF;
            load_meta(0);
            park_meta(0);
            load_meta(1);
            issue(0, rawA, ownA);
#pragma unroll 1
            for (int t = 0; t < ntiles; ++t) {
                park_meta(t + 1);
                static_for<IT>([&](auto kk) {
                    constexpr int K = decltype(kk)::value;
                    const int q = t * NB + 2 * K;
                    issue(q + 1, rawB, ownB);
                    load_meta_part(t + 2, std::integral_constant<int, K * NL / IT>{},
                                   std::integral_constant<int, (K + 1) * NL / IT>{});
                    consume(q, rawA, ownA);
                    issue(q + 2, rawA, ownA);   // past the last batch: padding only
                    consume(q + 1, rawB, ownB);
                });
            }
        } else if (nbatch > 0) {
            load_meta(0);
            park_meta(0);
            load_meta(1);
            issue(0, rawA, ownA);
#pragma unroll 1
            for (int q = 0; q < nbatch; q += 2) {
                // start of tile t: tile t+1 goes to the ring, tile t+2 is
                // loaded after the next batch's gathers (loads complete in
                // order, so consuming batch q then does not wait for it)
                const bool tile_start = (q % NB) == 0;
                if (tile_start) park_meta(q / NB + 1);
                issue(q + 1, rawB, ownB);
                if (tile_start) load_meta(q / NB + 2);
                consume(q, rawA, ownA);
                // unconditional, so the wait before the next consume counts
                // the same loads on every pass; past the last batch the ring
                // slot holds padding only (its gathers read nothing)
                issue(q + 2, rawA, ownA);
                consume(q + 1, rawB, ownB);
            }
        }

        if constexpr (!OUT) continue;

        // end of the run: the open row
        bool parked = false;
        if (gon) {
            const int nextk = ge < p.nnz ? p.out_idx[ge] : p.next_key;
            const bool right_shared = (nextk == open_key);
            const bool left_open = first_open && lsh;  // the run is one row, continued from the left
            if (left_open && s == 0) s_key[wv][2 * g] = -1;
            if (left_open || right_shared) {
                float* dst = &s_acc[wv][2 * g + 1][s * RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) dst[i] = acc[i];
                if (s == 0) {
                    s_key[wv][2 * g + 1] = open_key;
                    s_ext[wv][2 * g + 1] = ((left_open && g == 0) ? 1 : 0) | ((right_shared && ge == cs + clen) ? 2 : 0);
                }
            } else if (lane_on) {
                float v[RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) v[i] = acc[i] * oscale;
                store_cols<RPL>(p.out, open_key, ld, c, v);
            }
            parked = lsh || right_shared;
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
#if AMPED_QUEUE_STATS
    if (lane == 0 && p.qstats) {
        unsigned long long* r = p.qstats + ((size_t)blockIdx.x * kWaves + wv) * 4;
        r[0] = st_chunks;
        r[1] = st_nnz;
        r[2] = st_first;
        r[3] = (unsigned long long)wall_clock64();
    }
#endif
    if constexpr (LOSS) {
        // wave sum in fp64, one atomic per wave.  The first log2(LPR) steps add
        // equal values (every lane of a group holds the group's sum), so they
        // are exact doublings undone by the final 1/LPR.
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) lsum += __shfl_xor(lsum, m, 64);
        lsum *= 1.0 / LPR;
        if (lane == 0 && lsum != 0.0) atomicAdd(p.loss, lsum);
    }
}

using KernelFn = void (*)(const KParams);

// Vector instances: fp32 ranks 16/32/64/128 and bf16 ranks 32/64/128 for up
// to 4 input modes; every other case takes the scalar column-tile path.
constexpr int kMaxVecNin = 4;

// Kernel pickers, one translation unit each (compiled in parallel).
KernelFn pick_mttkrp_f32(int nin, int lpr, bool scalar, bool buf);
KernelFn pick_mttkrp_bf16(int nin, int lpr, bool scalar, bool buf);
KernelFn pick_grad(int nin, int lpr, bool scalar, bool buf);
KernelFn pick_loss(int nin, int lpr, bool scalar, bool buf);
KernelFn pick_grad_loss(int nin, int lpr, bool scalar, bool buf);

// The instance each picker returns: lpr counts 16-byte lanes per row (the
// vector path), scalar selects the column-tile path.  bfloat16 rows of up to
// 64 bytes (rank <= 32) use 8 bytes per lane, so a wave still covers 8 rows
// per gather at rank 32 (16-byte lanes would make 16 narrow groups), except
// 64-byte rows with three or more gathered factors (below).
#ifndef AMPED_BF16_NARROW
#define AMPED_BF16_NARROW 1
#endif
template <int NIN, typename T, int KIND, bool BUF>
KernelFn pick_vec(int lpr)
{
    constexpr int RPL = 16 / sizeof(T);
    constexpr bool narrow = AMPED_BF16_NARROW && std::is_same<T, uint16_t>::value;
    if constexpr (NIN > kMaxVecNin) {
        return nullptr;
    } else {
        if constexpr (narrow) {
            // with three or more gathered factors, 64-byte rows take 16-byte
            // lanes again (16 rows per gather instruction): the order-4
            // tensors measured faster so, in every mode, the order-3 ones
            // slower
            if (lpr == 2 || (lpr == 4 && NIN <= 2)) {
                switch (lpr) {
                case 2: return mttkrp_kernel<NIN, 4, 4, T, KIND, BUF>;
                case 4: return mttkrp_kernel<NIN, 8, 4, T, KIND, BUF>;
                default: return nullptr;
                }
            }
        }
        switch (lpr) {
        case 4: return mttkrp_kernel<NIN, 4, RPL, T, KIND, BUF>;
        case 8: return mttkrp_kernel<NIN, 8, RPL, T, KIND, BUF>;
        case 16: return mttkrp_kernel<NIN, 16, RPL, T, KIND, BUF>;
        case 32:
            if constexpr (std::is_same<T, float>::value) return mttkrp_kernel<NIN, 32, RPL, T, KIND, BUF>;
            else return nullptr;
        default: return nullptr;
        }
    }
}

template <int NIN, typename T, int KIND>
KernelFn pick_nin(int lpr, bool scalar, bool buf)
{
    if (scalar) return mttkrp_kernel<NIN, 64, 1, T, KIND, false>;
    return buf ? pick_vec<NIN, T, KIND, true>(lpr) : pick_vec<NIN, T, KIND, false>(lpr);
}

template <typename T, int KIND>
KernelFn pick_any(int nin, int lpr, bool scalar, bool buf)
{
    switch (nin) {
    case 1: return pick_nin<1, T, KIND>(lpr, scalar, buf);
    case 2: return pick_nin<2, T, KIND>(lpr, scalar, buf);
    case 3: return pick_nin<3, T, KIND>(lpr, scalar, buf);
    case 4: return pick_nin<4, T, KIND>(lpr, scalar, buf);
    case 5: return pick_nin<5, T, KIND>(lpr, scalar, buf);
    case 6: return pick_nin<6, T, KIND>(lpr, scalar, buf);
    case 7: return pick_nin<7, T, KIND>(lpr, scalar, buf);
    default: return nullptr;
    }
}

}  // namespace dev
}  // namespace amped
