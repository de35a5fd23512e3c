// gfx950 kernels for one CP-ALS sweep around the sparse MTTKRP (CPD by
// alternating least squares, Sec. 2.1; the mode loop of Alg. 1).  After the
// MTTKRP of mode d (M = X_(d) times the Khatri-Rao product of the others):
//
//   V   = Hadamard over w != d of G_w,  G_w = A_w^T A_w          (R x R)
//   A_d = M V^{-1}, then unit-norm columns with the norms in lambda
//
// Nothing per row is read twice more than needed: with S = M^T M,
// P = V^{-1} S V^{-1} is the Gram matrix of the unnormalised update, so
// lambda_r = sqrt(P_rr), the new G_d = D^{-1} P D^{-1} (D = diag(lambda)) and
// A_d = M W with W = V^{-1} D^{-1} come from R x R algebra; the big matrices
// pass through memory once each for S and once for A_d = M W.
//
// Kernels:
//  * gram_partial: A^T A of a rows x R fp32 matrix on the matrix cores.  Each
//    wave takes a slab of rows and one group of up to four 32 x 32 output tiles;
//    v_mfma_f32_32x32x2f32 consumes two rows per instruction, with lane l
//    supplying A[row0 + l/32][tile*32 + l%32] as both operands (the K index of
//    the product is the row).  Per-slab fp32 partials are summed in fp64 by
//    gram_reduce, in slab order (deterministic).
//  * als_small: one block, fp64: V, V^{-1} (Gauss-Jordan), P, lambda,
//    the new G_d, W and, after the last mode, the fit.
//  * als_solve: A_d = M W, a persistent grid over tiles of rows (256 at
//    R <= 32) staged through LDS beside W; the next tile's rows are loaded
//    into registers while the current one is computed.
//  * tensor_norm2: ||X||^2 over the mode-0 layout, exact duplicates (adjacent
//    there) summed before squaring.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "internal.h"

namespace amped {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kGramMaxPairs = 4;   // 32x32 output tiles per wave (4 x 16 accumulators)

// x[t] for a run-time t < T, without indexing a register array
template <int T>
__device__ __forceinline__ float pick(const float (&x)[T], int t)
{
    float r = x[0];
#pragma unroll
    for (int j = 1; j < T; ++j) r = (t == j) ? x[j] : r;
    return r;
}

// Upper-triangle tile pair p of T x T tiles (G is symmetric): row-major over
// tm <= tn.
__host__ __device__ constexpr int tri_tm(int T, int p)
{
    int tm = 0;
    while (p >= T - tm) {
        p -= T - tm;
        ++tm;
    }
    return tm;
}
__host__ __device__ constexpr int tri_tn(int T, int p)
{
    int tm = 0;
    while (p >= T - tm) {
        p -= T - tm;
        ++tm;
    }
    return tm + p;
}

// T = number of 32-column tiles (R <= 32 T).  Grid (slabs, tile groups);
// four waves per block each take a quarter of the slab's rows and keep up to
// kGramMaxPairs 32x32 tiles in MFMA accumulators, with kGramBatch row pairs of
// loads in flight before their MFMAs.  The four waves' tiles are then summed
// through LDS in wave order (deterministic) into the slab's partial.
constexpr int kGramBatch = 8;
template <int T>
__global__ void __launch_bounds__(256) gram_partial(const float* A, int64_t rows, int R, int64_t slab_rows,
                                                    float* partial)
{
    constexpr int NP = T * (T + 1) / 2;                               // upper-triangle tiles
    constexpr int NPB = NP < kGramMaxPairs ? NP : kGramMaxPairs;   // tiles per block
    constexpr int B = T <= 2 ? kGramBatch : kGramBatch / 2;          // row pairs per load batch
    __shared__ float s_t[4][NPB][32 * 32];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b0 = (int64_t)blockIdx.x * slab_rows;
    const int64_t b1 = std::min<int64_t>(b0 + slab_rows, rows);
    const int64_t q = ((slab_rows + 3) / 4 + 1) & ~(int64_t)1;   // even rows per wave, 4 q >= slab_rows
    const int64_t r0 = std::min<int64_t>(b0 + wave * q, b1);
    const int64_t r1 = std::min<int64_t>(r0 + q, b1);
    const int p0 = blockIdx.y * kGramMaxPairs;
    const int np = std::min(kGramMaxPairs, NP - p0);
    f32x16 acc[NPB];
#pragma unroll
    for (int j = 0; j < NPB; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[j][v] = 0.f;
    const int col = lane & 31;
    const int kk = lane >> 5;
    // batches of B row pairs, double-buffered: batch k+1 is loaded while
    // batch k feeds the MFMAs
    auto load = [&](float (&x)[B][T], int64_t i) {
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int64_t row = i + 2 * u + kk;
            const bool rv = row < r1;
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const int c = t * 32 + col;
                x[u][t] = (rv && c < R) ? A[row * R + c] : 0.f;
            }
        }
    };
    auto fma_batch = [&](const float (&x)[B][T]) {
#pragma unroll
        for (int u = 0; u < B; ++u)
#pragma unroll
            for (int j = 0; j < NPB; ++j) {
                if (j < np) {
                    const int p = p0 + j;
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(pick<T>(x[u], tri_tm(T, p)),
                                                                  pick<T>(x[u], tri_tn(T, p)), acc[j], 0, 0, 0);
                }
            }
    };
    float xa[B][T], xb[B][T];
    if (r0 < r1) load(xa, r0);
    for (int64_t i = r0; i < r1; i += 4 * B) {
        load(xb, i + 2 * B);      // rows past r1 read as zeros
        fma_batch(xa);
        if (i + 4 * B < r1) load(xa, i + 4 * B);
        fma_batch(xb);
    }
    // lane l holds output column l%32; value v sits in row 8(v/4) + 4(l/32) + v%4
#pragma unroll
    for (int j = 0; j < NPB; ++j) {
        if (j >= np) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v) s_t[wave][j][(8 * (v >> 2) + 4 * kk + (v & 3)) * 32 + col] = acc[j][v];
    }
    __syncthreads();
    float* out = partial + (int64_t)blockIdx.x * R * R;
    for (int e = threadIdx.x; e < np * 1024; e += 256) {
        const int j = e >> 10, m = (e >> 5) & 31, n = e & 31;
        const float sum = ((s_t[0][j][e & 1023] + s_t[1][j][e & 1023]) + s_t[2][j][e & 1023]) + s_t[3][j][e & 1023];
        const int p = p0 + j;
        const int r = tri_tm(T, p) * 32 + m, c = tri_tn(T, p) * 32 + n;
        if (r < R && c < R) {
            out[r * R + c] = sum;
            out[c * R + r] = sum;   // the mirrored tile (the same entry on the diagonal tiles)
        }
    }
}

// G[e] = sum over slabs of partial[slab][e] in fp64.  A block takes 32
// consecutive entries; its 8 slab lanes add every 8th slab, then the 8 sums
// are added in lane order (deterministic).
__global__ void __launch_bounds__(256) gram_reduce(const float* partial, int64_t nslab, int R, double* G)
{
    __shared__ double s[8][32];
    const int e32 = threadIdx.x & 31, sl = threadIdx.x >> 5;
    const int e = blockIdx.x * 32 + e32;
    const int RR = R * R;
    double acc = 0.0;
    if (e < RR) {
        // 8 loads in flight, added in slab order
        int64_t k = sl;
        for (; k + 56 < nslab; k += 64) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = partial[(k + 8 * u) * RR + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += (double)v[u];
        }
        for (; k < nslab; k += 8) acc += (double)partial[k * RR + e];
    }
    s[sl][e32] = acc;
    __syncthreads();
    if (sl == 0 && e < RR) {
        double t = 0.0;
        for (int j = 0; j < 8; ++j) t += s[j][e32];
        G[e] = t;
    }
}

// Largest 1-norm condition number of V for which the update's product M W
// keeps fp32 sums (als_solve).  The sum over k of M[i, k] W[k, r] cancels by
// up to about sqrt(kappa) when V is ill-conditioned (nearly collinear factor
// columns); fp32 sums then lose that many ulps, so above this bound the sums
// are taken in fp64.  At kappa = 1e4 the fp32 rounding of M W stays below the
// fp32 error of M itself (about 1e-6 relative).
constexpr double kSolveFp32MaxCond = 1e4;

// R x R fp64 algebra of one mode update, one block of 256 threads.  Works
// in 4 R x R doubles: LDS when they fit (dynamic, in_lds), else the global
// scratch.  G: [N][R][R] (G[d] is replaced).
__global__ void __launch_bounds__(256) als_small(double* G, const double* S, int N, int d, int R, double* scratch,
                                                 double* W, int* wide, double* lambda, int last,
                                                 const double* xnorm2, double* fit, int in_lds)
{
    extern __shared__ __align__(16) double s_small[];
    if (in_lds) scratch = s_small;
    const int tid = threadIdx.x;
    const int RR = R * R;
    double* V = scratch;
    double* L = scratch + RR;
    double* Vi = scratch + 2 * RR;
    double* T = scratch + 3 * RR;
    for (int e = tid; e < RR; e += 256) {
        double v = 1.0;
        for (int w = 0; w < N; ++w)
            if (w != d) v *= G[(int64_t)w * RR + e];
        V[e] = v;
        L[e] = 0.0;
    }
    __syncthreads();
    // V^{-1} by Gauss-Jordan elimination without pivoting (V is symmetric
    // positive semi-definite): L holds the reduced V, Vi starts as I.  A pivot
    // that is not positive (V singular, e.g. a zero factor column) is replaced
    // by a tiny one, so that row and column of V^{-1} stay apart from the rest.
    double vmax = 0.0;
    for (int k = 0; k < R; ++k) vmax = fmax(vmax, fabs(V[k * R + k]));
    const double tiny = (vmax > 0.0 ? vmax : 1.0) * 1e-30;
    __shared__ double fcol[128];
    for (int e = tid; e < RR; e += 256) {
        L[e] = V[e];
        Vi[e] = (e / R == e % R) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < R; ++k) {
        // pivot row k scaled by 1/pivot; the column-k multipliers saved first
        const double pv = L[k * R + k];
        const double inv = 1.0 / (pv > tiny ? pv : tiny);
        for (int i = tid; i < R; i += 256) fcol[i] = L[i * R + k];
        __syncthreads();
        for (int j = tid; j < R; j += 256) {
            L[k * R + j] *= inv;
            Vi[k * R + j] *= inv;
        }
        __syncthreads();
        for (int e = tid; e < RR; e += 256) {
            const int i = e / R, j = e % R;
            if (i == k) continue;
            const double f = fcol[i];
            L[e] -= f * L[k * R + j];
            Vi[e] -= f * Vi[k * R + j];
        }
        __syncthreads();
    }
    // The 1-norm condition number kappa = ||V||_1 ||V^{-1}||_1 picks the
    // precision of the update's product M W (als_solve): fp32 sums while kappa
    // <= kSolveFp32MaxCond, fp64 sums above (or when kappa is not finite).
    if (tid < 64) {
        double a = 0.0, b = 0.0;
        for (int j = tid; j < R; j += 64) {
            double sa = 0.0, sb = 0.0;
            for (int i = 0; i < R; ++i) {
                sa += fabs(V[i * R + j]);
                sb += fabs(Vi[i * R + j]);
            }
            a = fmax(a, sa);
            b = fmax(b, sb);
        }
        for (int m = 1; m < 64; m <<= 1) {
            a = fmax(a, __shfl_xor(a, m, 64));
            b = fmax(b, __shfl_xor(b, m, 64));
        }
        const double kappa = a * b;
        if (tid == 0) *wide = (kappa <= kSolveFp32MaxCond) ? 0 : 1;   // NaN: fp64
    }
    __syncthreads();
    // S into V's slot (V is no longer needed), then T = S V^{-1}
    for (int e = tid; e < RR; e += 256) V[e] = S[e];
    __syncthreads();
    for (int e = tid; e < RR; e += 256) {
        const int i = e / R, j = e % R;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += V[i * R + k] * Vi[k * R + j];
        T[e] = s;
    }
    __syncthreads();
    // P = V^{-1} T (V^{-1} is symmetric) into V; lambda = sqrt(diag P)
    for (int e = tid; e < RR; e += 256) {
        const int i = e / R, j = e % R;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += Vi[k * R + i] * T[k * R + j];
        V[e] = s;
    }
    __syncthreads();
    for (int r = tid; r < R; r += 256) {
        const double p = V[r * R + r];
        lambda[r] = p > 0.0 ? sqrt(p) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < RR; e += 256) {
        const int i = e / R, j = e % R;
        const double li = lambda[i], lj = lambda[j];
        G[(int64_t)d * RR + e] = (li > 0.0 && lj > 0.0) ? V[e] / (li * lj) : 0.0;
        W[e] = lj > 0.0 ? Vi[e] / lj : 0.0;
    }
    __syncthreads();
    if (last) {
        // <X, Xhat> = sum_r lambda_r (S W)_rr = trace(S V^{-1}) over columns
        // with lambda_r > 0; ||Xhat||^2 = lambda^T (Hadamard of all G) lambda.
        // Per-thread sums over a fixed slice, then a fixed-order block sum.
        __shared__ double part[256];
        double xh = 0.0;
        for (int e = tid; e < RR; e += 256) {
            const int i = e / R, j = e % R;
            double h = 1.0;
            for (int w = 0; w < N; ++w) h *= G[(int64_t)w * RR + e];
            xh += lambda[i] * lambda[j] * h;
        }
        part[tid] = xh;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (tid < off) part[tid] += part[tid + off];
            __syncthreads();
        }
        if (tid == 0) {
            double inner = 0.0;
            for (int r = 0; r < R; ++r)
                if (lambda[r] > 0.0) inner += T[r * R + r];
            const double x2 = *xnorm2;
            const double res = x2 - 2.0 * inner + part[0];
            *fit = x2 > 0.0 ? 1.0 - sqrt(res > 0.0 ? res : 0.0) / sqrt(x2) : 0.0;
        }
    }
}

// A = M W for a rows x R fp32 matrix M and an R x R fp64 matrix W.  W =
// V^{-1} D^{-1} has large entries of opposite sign when V is ill-conditioned
// (nearly collinear factor columns), and the sum over k then cancels: when
// als_small flagged V (*wide != 0) the products and sums are fp64 and A is
// rounded to fp32 once, otherwise W is rounded to fp32 and the sums are fp32.
// A block of 256 threads stages RB rows of M (row stride R + 1 in LDS, so the
// rows a wave reads fall in different banks) and W; thread (g, c8) computes
// RPT rows and 8 columns from registers.
template <int RPT, typename Acc>
__device__ __forceinline__ void solve_tile(const Acc* sW, int RW, const float* sM, int R, int i0, int nr, int c8,
                                           float* A, int64_t r0)
{
    Acc acc[RPT][8];
#pragma unroll
    for (int j = 0; j < RPT; ++j)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[j][c] = Acc(0);
    for (int k = 0; k < R; ++k) {
        Acc w[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) w[c] = sW[k * RW + 8 * c8 + c];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const Acc m = (i0 + j < nr) ? (Acc)sM[(i0 + j) * (R + 1) + k] : Acc(0);
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[j][c] = fma(m, w[c], acc[j][c]);
        }
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        if (i0 + j >= nr) continue;
        float* out = A + (r0 + i0 + j) * R + 8 * c8;
        if ((R & 7) == 0) {   // 32-byte aligned run of 8 columns
            *reinterpret_cast<float4*>(out) = make_float4((float)acc[j][0], (float)acc[j][1], (float)acc[j][2],
                                                          (float)acc[j][3]);
            *reinterpret_cast<float4*>(out + 4) = make_float4((float)acc[j][4], (float)acc[j][5], (float)acc[j][6],
                                                              (float)acc[j][7]);
        } else {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (8 * c8 + c < R) out[c] = (float)acc[j][c];
        }
    }
}

// Persistent: block b takes tiles b, b + grid, ... of RB rows.  W goes to LDS
// once per block.  With R % 4 == 0 each thread holds its part of the next
// tile's rows of M (up to 8 float4) in registers, loaded before the current
// tile is computed, so the loads overlap the arithmetic and the stores.
template <int RPT>
__global__ void __launch_bounds__(256) als_solve(const float* M, const double* W, const int* wide_flag, float* A,
                                                 int64_t rows, int R, int RB, int64_t ntiles)
{
    extern __shared__ __align__(16) double s_solve[];
    const int C8 = (R + 7) / 8;                 // column groups of 8
    const int RW = 8 * C8;                      // padded row length of W
    const bool wide = *wide_flag != 0;          // the same for every thread
    double* sW = s_solve;                       // [R][RW] fp64, or fp32 in the first half
    float* sWf = reinterpret_cast<float*>(s_solve);
    float* sM = reinterpret_cast<float*>(s_solve + R * RW);   // [RB][R + 1]
    const int tid = threadIdx.x;
    for (int e = tid; e < R * RW; e += 256) {
        const int k = e / RW, c = e % RW;
        const double w = c < R ? W[k * R + c] : 0.0;
        if (wide) sW[e] = w;
        else sWf[e] = (float)w;
    }
    const bool vec = (R & 3) == 0;
    const float4* M4 = reinterpret_cast<const float4*>(M);
    float4 v[8];   // RB * R / 4 <= 8 * 256 (launch_als_solve)
    auto fetch = [&](int64_t t) {
        const int64_t r0 = t * RB;
        const int n4 = t < ntiles ? (int)(std::min<int64_t>(RB, rows - r0) * R / 4) : 0;
        const float4* src = M4 + (t < ntiles ? r0 * (R / 4) : 0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = u * 256 + tid;
            v[u] = e < n4 ? src[e] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    if (vec) fetch(blockIdx.x);
    const int g = tid / C8, c8 = tid % C8;
    const int i0 = RPT * g;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t r0 = t * RB;
        const int nr = (int)std::min<int64_t>(RB, rows - r0);
        __syncthreads();   // W staged; the previous tile's reads of sM done
        if (vec) {
            const int n4 = nr * R / 4;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = u * 256 + tid;
                if (e < n4) {
                    const int i = (4 * e) / R, k = (4 * e) % R;
                    float* d = &sM[i * (R + 1) + k];
                    d[0] = v[u].x; d[1] = v[u].y; d[2] = v[u].z; d[3] = v[u].w;
                }
            }
        } else {
            for (int e = tid; e < nr * R; e += 256) sM[(e / R) * (R + 1) + e % R] = M[r0 * R + e];
        }
        __syncthreads();
        if (vec) fetch(t + gridDim.x);
        if (i0 < nr) {
            if (wide) solve_tile<RPT, double>(sW, RW, sM, R, i0, nr, c8, A, r0);
            else solve_tile<RPT, float>(sWf, RW, sM, R, i0, nr, c8, A, r0);
        }
    }
}

// ||X||^2 over a layout whose exact duplicates are adjacent (mode 0's).
struct InIdx {
    const int32_t* p[kMaxOrder - 1];
};

__global__ void __launch_bounds__(256) tensor_norm2(const int32_t* out_idx, InIdx in_idx, int nin,
                                                    const float* val, int64_t nnz, double* result)
{
    __shared__ double part[4];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double s = 0.0;
    auto same = [&](int64_t a, int64_t b) {
        if (out_idx[a] != out_idx[b]) return false;
        for (int w = 0; w < nin; ++w)
            if (in_idx.p[w][a] != in_idx.p[w][b]) return false;
        return true;
    };
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride) {
        if (p > 0 && same(p - 1, p)) continue;
        double v = val[p];
        for (int64_t q = p + 1; q < nnz && same(p, q); ++q) v += val[q];
        s += v * v;
    }
    for (int m = 1; m < 64; m <<= 1) s += __shfl_xor(s, m, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(result, part[0] + part[1] + part[2] + part[3]);
}

}  // namespace

int64_t gram_slabs(int64_t rows)
{
    // about 8192 rows per slab; above 256 slabs a multiple of 256, so every
    // CU of the 256 gets the same number of slabs
    int64_t n = (rows + 8191) / 8192;
    if (n > 256) n = (n + 255) / 256 * 256;
    return std::max<int64_t>(1, std::min<int64_t>(n, 2048));
}

hipError_t launch_gram(const float* A, int64_t rows, int R, float* partial, double* G, hipStream_t st,
                       int64_t nslab)
{
    if (R < 1 || R > 128) return hipErrorInvalidValue;
    if (nslab <= 0) nslab = gram_slabs(rows);
    int64_t slab_rows = (rows + nslab - 1) / nslab;
    slab_rows += slab_rows & 1;
    const int T = (R + 31) / 32;
    const int groups = (T * (T + 1) / 2 + kGramMaxPairs - 1) / kGramMaxPairs;
    dim3 grid((unsigned)nslab, (unsigned)groups);
    switch (T) {
    case 1: hipLaunchKernelGGL(gram_partial<1>, grid, dim3(256), 0, st, A, rows, R, slab_rows, partial); break;
    case 2: hipLaunchKernelGGL(gram_partial<2>, grid, dim3(256), 0, st, A, rows, R, slab_rows, partial); break;
    case 3: hipLaunchKernelGGL(gram_partial<3>, grid, dim3(256), 0, st, A, rows, R, slab_rows, partial); break;
    default: hipLaunchKernelGGL(gram_partial<4>, grid, dim3(256), 0, st, A, rows, R, slab_rows, partial); break;
    }
    hipLaunchKernelGGL(gram_reduce, dim3((R * R + 31) / 32), dim3(256), 0, st, partial, nslab, R, G);
    return hipGetLastError();
}

// ------------------------------------------------ Gram without allocation
// The partial sums of amped_gram_noalloc live in this fixed device array
// instead of memory allocated per call: kGramScratchFloats floats (32 MiB) on
// every device the library runs on, held until the process ends.  Every call
// on a device shares its array; gram_partial overwrites every entry the
// reduction reads, so nothing has to be cleared between calls, and calls that
// overlap on one device race on it.
constexpr int64_t kGramScratchFloats = int64_t(8) << 20;
static __device__ __align__(256) float scratch[kGramScratchFloats];

namespace {
// Device address of `scratch` per device, looked up once per device with that
// device current (the host-side name is not a device address).
constexpr int kMaxDevices = 64;
float* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

int64_t gram_noalloc_slabs(int64_t rows, int R)
{
    const int64_t fit = kGramScratchFloats / ((int64_t)R * R);
    return std::min(gram_slabs(rows), fit);
}

hipError_t launch_gram_noalloc(const float* A, int64_t rows, int R, double* G, hipStream_t st)
{
    if (R < 1 || R > 128 || rows < 1) return hipErrorInvalidValue;
    const int64_t nslab = gram_noalloc_slabs(rows, R);
    if (nslab < 1 || nslab * (int64_t)R * R > kGramScratchFloats) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    float* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            if (!p) return hipErrorInvalidSymbol;
            g_scratch_ptr[dev] = static_cast<float*>(p);
        }
        ptr = g_scratch_ptr[dev];
    }
    return launch_gram(A, rows, R, ptr, G, st, nslab);
}

hipError_t launch_als_small(double* G, const double* S, int N, int d, int R, double* scratch, double* W, int* wide,
                            double* lambda, bool last, const double* xnorm2, double* fit, hipStream_t st)
{
    const size_t bytes = (size_t)4 * R * R * sizeof(double);
    const bool in_lds = bytes <= (size_t)128 * 1024;
    hipLaunchKernelGGL(als_small, dim3(1), dim3(256), in_lds ? bytes : 0, st, G, S, N, d, R, scratch, W, wide,
                       lambda, last ? 1 : 0, xnorm2, fit, in_lds ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_als_solve(const float* M, const double* W, const int* wide, float* A, int64_t rows, int R,
                            hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    const int C8 = (R + 7) / 8;
    // rows per thread: 4, or 2 above R = 64 so that the fp64 W (R x 8 C8
    // doubles) and the staged rows of M fit one block's LDS
    const int rpt = R > 64 ? 2 : 4;
    const int RB = rpt * (256 / C8);    // rows per block
    const size_t lds = (size_t)R * 8 * C8 * sizeof(double) + (size_t)RB * (R + 1) * sizeof(float);
    if ((int64_t)RB * R > 8 * 256 * 4) return hipErrorInvalidValue;   // the kernel holds 8 float4 per thread
    const int64_t ntiles = (rows + RB - 1) / RB;
    // persistent grid: as many blocks as fit on the GPU at once
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = rpt == 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, als_solve<4>, 256, lds)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, als_solve<2>, 256, lds);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(ntiles, (int64_t)std::max(per_cu, 1) * cus)));
    if (rpt == 4) hipLaunchKernelGGL(als_solve<4>, grid, dim3(256), lds, st, M, W, wide, A, rows, R, RB, ntiles);
    else hipLaunchKernelGGL(als_solve<2>, grid, dim3(256), lds, st, M, W, wide, A, rows, R, RB, ntiles);
    return hipGetLastError();
}

hipError_t launch_tensor_norm2(const ModeDev& m, int nin, double* result, bool accumulate, hipStream_t st)
{
    hipError_t e = accumulate ? hipSuccess : hipMemsetAsync(result, 0, sizeof(double), st);
    if (e != hipSuccess || m.nnz == 0) return e;
    InIdx ii{};
    for (int w = 0; w < nin; ++w) ii.p[w] = m.in_idx[w];
    const int grid = (int)std::min<int64_t>((m.nnz + 255) / 256, 4096);
    hipLaunchKernelGGL(tensor_norm2, dim3(grid), dim3(256), 0, st, m.out_idx, ii, nin, m.val, m.nnz, result);
    return hipGetLastError();
}

}  // namespace amped
