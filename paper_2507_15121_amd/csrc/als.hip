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
//  * als_small: one block, fp64: V, its Cholesky factor, V^{-1}, P, lambda,
//    the new G_d, W (fp32) and, after the last mode, the fit.
//  * als_solve: A_d = M W, 64 rows per block staged through LDS with W.
//  * tensor_norm2: ||X||^2 over the mode-0 layout, exact duplicates (adjacent
//    there) summed before squaring.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

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

// T = number of 32-column tiles (R <= 32 T).  Grid (slabs, tile groups), one
// wave per block.
template <int T>
__global__ void __launch_bounds__(64) gram_partial(const float* A, int64_t rows, int R, int64_t slab_rows,
                                                   float* partial)
{
    constexpr int NP = T * T;
    const int lane = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * slab_rows;
    const int64_t r1 = std::min<int64_t>(r0 + slab_rows, rows);
    const int p0 = blockIdx.y * kGramMaxPairs;
    const int np = std::min(kGramMaxPairs, NP - p0);
    f32x16 acc[kGramMaxPairs];
#pragma unroll
    for (int q = 0; q < kGramMaxPairs; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[q][v] = 0.f;
    const int col = lane & 31;
    const int kk = lane >> 5;
    for (int64_t i = r0; i < r1; i += 2) {
        const int64_t row = i + kk;
        const bool rv = row < r1;
        float x[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int c = t * 32 + col;
            x[t] = (rv && c < R) ? A[row * R + c] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < kGramMaxPairs; ++q) {
            if (q < np) {
                const int p = p0 + q;
                acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(pick<T>(x, p / T), pick<T>(x, p % T), acc[q], 0, 0,
                                                              0);
            }
        }
    }
    // lane l holds output column l%32; value v sits in row 8(v/4) + 4(l/32) + v%4
    float* out = partial + (int64_t)blockIdx.x * R * R;
#pragma unroll
    for (int q = 0; q < kGramMaxPairs; ++q) {
        if (q >= np) continue;
        const int p = p0 + q;
        const int tm = p / T, tn = p % T;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int m = 8 * (v >> 2) + 4 * kk + (v & 3);
            const int r = tm * 32 + m, c = tn * 32 + col;
            if (r < R && c < R) out[r * R + c] = acc[q][v];
        }
    }
}

__global__ void __launch_bounds__(256) gram_reduce(const float* partial, int64_t nslab, int R, double* G)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= R * R) return;
    double s = 0.0;
    for (int64_t k = 0; k < nslab; ++k) s += (double)partial[k * R * R + e];
    G[e] = s;
}

// R x R fp64 algebra of one mode update, one block of 256 threads.
// scratch: 4 R x R doubles.  G: [N][R][R] (G[d] is replaced).
__global__ void __launch_bounds__(256) als_small(double* G, const double* S, int N, int d, int R, double* scratch,
                                                 float* W, double* lambda, int last, const double* xnorm2,
                                                 double* fit)
{
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
    // Cholesky V = L L^T, column by column; a pivot that is not positive
    // (V singular, e.g. a zero factor column) is replaced by a tiny one
    double vmax = 0.0;
    for (int k = 0; k < R; ++k) vmax = fmax(vmax, fabs(V[k * R + k]));
    const double tiny = (vmax > 0.0 ? vmax : 1.0) * 1e-30;
    __shared__ double piv;
    for (int k = 0; k < R; ++k) {
        if (tid == 0) {
            double s = V[k * R + k];
            for (int j = 0; j < k; ++j) s -= L[k * R + j] * L[k * R + j];
            piv = sqrt(s > tiny ? s : tiny);
            L[k * R + k] = piv;
        }
        __syncthreads();
        for (int i = k + 1 + tid; i < R; i += 256) {
            double s = V[i * R + k];
            for (int j = 0; j < k; ++j) s -= L[i * R + j] * L[k * R + j];
            L[i * R + k] = s / piv;
        }
        __syncthreads();
    }
    // V^{-1}: column c solves L y = e_c, then L^T x = y (in place)
    for (int c = tid; c < R; c += 256) {
        for (int i = 0; i < R; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int j = 0; j < i; ++j) s -= L[i * R + j] * Vi[j * R + c];
            Vi[i * R + c] = s / L[i * R + i];
        }
        for (int i = R - 1; i >= 0; --i) {
            double s = Vi[i * R + c];
            for (int j = i + 1; j < R; ++j) s -= L[j * R + i] * Vi[j * R + c];
            Vi[i * R + c] = s / L[i * R + i];
        }
    }
    __syncthreads();
    // T = S V^{-1}
    for (int e = tid; e < RR; e += 256) {
        const int i = e / R, j = e % R;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += S[i * R + k] * Vi[k * R + j];
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
        W[e] = lj > 0.0 ? (float)(Vi[e] / lj) : 0.f;
    }
    __syncthreads();
    if (last && tid == 0) {
        // <X, Xhat> = sum_r lambda_r (S W)_rr = trace(S V^{-1}) over columns
        // with lambda_r > 0; ||Xhat||^2 = lambda^T (Hadamard of all G) lambda
        double inner = 0.0;
        for (int r = 0; r < R; ++r)
            if (lambda[r] > 0.0) inner += T[r * R + r];
        double xh = 0.0;
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < R; ++j) {
                double h = 1.0;
                for (int w = 0; w < N; ++w) h *= G[(int64_t)w * RR + i * R + j];
                xh += lambda[i] * lambda[j] * h;
            }
        const double x2 = *xnorm2;
        const double res = x2 - 2.0 * inner + xh;
        *fit = x2 > 0.0 ? 1.0 - sqrt(res > 0.0 ? res : 0.0) / sqrt(x2) : 0.0;
    }
}

// A = M W for rows x R fp32 matrices (row-major), W R x R; 64 rows per block.
constexpr int kSolveRows = 64;
__global__ void __launch_bounds__(256) als_solve(const float* M, const float* W, float* A, int64_t rows, int R)
{
    extern __shared__ float s_solve[];
    float* sW = s_solve;             // [R][R]
    float* sM = s_solve + R * R;     // [kSolveRows][R]
    const int tid = threadIdx.x;
    for (int e = tid; e < R * R; e += 256) sW[e] = W[e];
    const int64_t r0 = (int64_t)blockIdx.x * kSolveRows;
    const int nr = (int)std::min<int64_t>(kSolveRows, rows - r0);
    for (int e = tid; e < nr * R; e += 256) sM[e] = M[r0 * R + e];
    __syncthreads();
    for (int e = tid; e < nr * R; e += 256) {
        const int i = e / R, c = e % R;
        float s = 0.f;
        for (int k = 0; k < R; ++k) s = fmaf(sM[i * R + k], sW[k * R + c], s);
        A[r0 * R + e] = s;
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
    return std::max<int64_t>(1, std::min<int64_t>((rows + 4095) / 4096, 2048));
}

hipError_t launch_gram(const float* A, int64_t rows, int R, float* partial, double* G, hipStream_t st)
{
    if (R < 1 || R > 128) return hipErrorInvalidValue;
    const int64_t nslab = gram_slabs(rows);
    int64_t slab_rows = (rows + nslab - 1) / nslab;
    slab_rows += slab_rows & 1;
    const int T = (R + 31) / 32;
    const int groups = (T * T + kGramMaxPairs - 1) / kGramMaxPairs;
    dim3 grid((unsigned)nslab, (unsigned)groups);
    switch (T) {
    case 1: hipLaunchKernelGGL(gram_partial<1>, grid, dim3(64), 0, st, A, rows, R, slab_rows, partial); break;
    case 2: hipLaunchKernelGGL(gram_partial<2>, grid, dim3(64), 0, st, A, rows, R, slab_rows, partial); break;
    case 3: hipLaunchKernelGGL(gram_partial<3>, grid, dim3(64), 0, st, A, rows, R, slab_rows, partial); break;
    default: hipLaunchKernelGGL(gram_partial<4>, grid, dim3(64), 0, st, A, rows, R, slab_rows, partial); break;
    }
    hipLaunchKernelGGL(gram_reduce, dim3((R * R + 255) / 256), dim3(256), 0, st, partial, nslab, R, G);
    return hipGetLastError();
}

hipError_t launch_als_small(double* G, const double* S, int N, int d, int R, double* scratch, float* W,
                            double* lambda, bool last, const double* xnorm2, double* fit, hipStream_t st)
{
    hipLaunchKernelGGL(als_small, dim3(1), dim3(256), 0, st, G, S, N, d, R, scratch, W, lambda, last ? 1 : 0,
                       xnorm2, fit);
    return hipGetLastError();
}

hipError_t launch_als_solve(const float* M, const float* W, float* A, int64_t rows, int R, hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    const size_t lds = (size_t)(R * R + kSolveRows * R) * sizeof(float);
    hipLaunchKernelGGL(als_solve, dim3((unsigned)((rows + kSolveRows - 1) / kSolveRows)), dim3(256), lds, st, M, W, A,
                       rows, R);
    return hipGetLastError();
}

hipError_t launch_tensor_norm2(const ModeDev& m, int nin, double* result, hipStream_t st)
{
    hipError_t e = hipMemsetAsync(result, 0, sizeof(double), st);
    if (e != hipSuccess || m.nnz == 0) return e;
    InIdx ii{};
    for (int w = 0; w < nin; ++w) ii.p[w] = m.in_idx[w];
    const int grid = (int)std::min<int64_t>((m.nnz + 255) / 256, 4096);
    hipLaunchKernelGGL(tensor_norm2, dim3(grid), dim3(256), 0, st, m.out_idx, ii, nin, m.val, m.nnz, result);
    return hipGetLastError();
}

}  // namespace amped
