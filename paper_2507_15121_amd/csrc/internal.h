// Internal interfaces shared by the C-ABI layer, the host layout builder and
// the HIP kernel launchers.  Not installed; not part of the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

namespace amped {

constexpr int kMaxOrder = 8;
constexpr int64_t kDefaultChunk = 4096;
// Largest chunk: a chunk's metadata arrays stay below 2^30 bytes, so 32-bit
// buffer offsets into them (with an out-of-range bias) never wrap.
constexpr int64_t kMaxChunk = int64_t(1) << 28;
// Hot-row tables: for every power of two K <= kHotMax, a direct-mapped table
// of K slots; slot s names the row r with r % K == s that the most nonzeros
// use in this mode (kHotEmpty if no row maps to s).  The tables of all K are
// stored back to back, the one for K at offset K - 1.
constexpr int kHotMax = 1024;
constexpr int kHotTableLen = 2 * kHotMax - 1;
constexpr int32_t kHotEmpty = -2;
// Scratch floats each tensor keeps for stores that must not land (64 lanes x 8).
constexpr int kSinkFloats = 512;
// The init kernel zeroes untouched output rows: runs at least this long as
// (start, length) ranges, shorter runs row by row from the zero-row list.
// A range is one workgroup's work, so longer runs are cut into ranges of
// about kGapPiece rows (each at least kLongGap): an untouched run of millions
// of rows (say, the unused tail of an index space) is then spread over the
// whole grid instead of one workgroup.
constexpr int kLongGap = 16;
constexpr int kGapPiece = 2048;
// Work-queue counters per layout: the chunks are split into at most this many
// contiguous stripes, each with its own counter (one stripe per XCD).
constexpr int kQueueSlots = 8;

// ----------------------------------------------------------------- host layout
struct HostModeLayout {
    std::vector<int32_t> perm;        // position -> input nonzero
    std::vector<uint8_t> flags;       // per chunk: bit0 head continues, bit1 tail continues
    std::vector<int32_t> zero_rows;   // rows shared by two or more chunks, then untouched rows of short runs
    std::vector<int32_t> gaps;        // (start, length) pairs of long untouched-row runs
    std::vector<int32_t> hot;         // hot-row tables of this mode's rows [kHotTableLen]
    int64_t touched = 0;              // distinct output indices
};

// Position order of the input sorted lexicographically by (i_0, ..., i_{N-1}),
// stable; an empty vector means the input already is in that order.
std::vector<int32_t> lex_order(int order, const int64_t* dims, int64_t nnz, const int32_t* idx);

// Stable order by i_mode of `base` (identity when base is empty).
void mode_order(const int64_t* dims, int64_t nnz, const int32_t* idx, const std::vector<int32_t>& base,
                int mode, std::vector<int32_t>& perm);

// Chunk flags, zero-row list, long gaps, hot-row tables and touched count of a
// mode order.
void mode_tables(const int64_t* dims, int64_t nnz, const int32_t* idx, int mode, int64_t chunk,
                 HostModeLayout& lay);

// The same tables from the mode's sorted output-index column keys[nnz].
void mode_tables_sorted(const int32_t* keys, int64_t nnz, int64_t rows, int64_t chunk, HostModeLayout& lay);

// True when the COO is already in lexicographic order of (i_0, ..., i_{N-1}).
bool is_lexicographic(int order, int64_t nnz, const int32_t* idx);

// Device layout build: a stable LSD radix sort of n (key, value) pairs by the
// low key_bits bits of the keys, 8 bits per pass, ping-ponging between
// (keys, vals) and (keys_alt, vals_alt); *result_in_alt says where the sorted
// pairs are.  scratch holds sort_scratch_words(n) 32-bit words.
int64_t sort_scratch_words(int64_t n);
hipError_t launch_stable_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt,
                                    uint32_t* scratch, int64_t n, int key_bits, bool* result_in_alt,
                                    hipStream_t st);
// a[i] = i for i < n.
hipError_t launch_iota(int32_t* a, int64_t n, hipStream_t st);

// Gather idx[w][perm[p]] for p in [p0, p1) into dst.
void gather_i32(const int32_t* src, const int32_t* perm, int64_t p0, int64_t p1, int32_t* dst);
void gather_f32(const float* src, const int32_t* perm, int64_t p0, int64_t p1, float* dst);

// -------------------------------------------------------------- device layout
struct ModeDev {
    const int32_t* out_idx = nullptr;              // [nnz]
    const int32_t* in_idx[kMaxOrder - 1] = {};     // other modes ascending, each [nnz]
    const float* val = nullptr;                    // [nnz]
    const int32_t* zero_rows = nullptr;            // [n_zero]
    const int32_t* gaps = nullptr;                 // [2 * n_gaps]
    int64_t nnz = 0, chunk = 0, n_chunks = 0, rows = 0, n_zero = 0, n_gaps = 0;
    unsigned* queue = nullptr;                     // kQueueSlots device work-queue counters
    const int32_t* hot = nullptr;                  // hot-row tables of this mode [kHotTableLen]
    const void* zero_row = nullptr;                // 16 zero bytes
    float* sink = nullptr;                         // kSinkFloats floats of write-only scratch
    // A shard of a longer layout (whole chunks of it): the output indices just
    // before and after the shard, -1 at the layout's ends.  Rows that cross a
    // shard edge cross a chunk edge, so they are in the zero-row list and every
    // shard adds into them.
    int prev_key = -1, next_key = -1;
};

enum class FactorType { F32 = 0, BF16 = 1 };
// ResidualGradLoss: the residual gradient that also sums the squared
// residuals into `loss` (the sparse CP loss) in the same pass.
enum class Kind { Mttkrp = 0, ResidualGrad = 1, ResidualGradLoss = 3 };

struct LaunchArgs {
    const ModeDev* m = nullptr;
    int nin = 0;                                   // number of input modes (order - 1)
    int rank = 0;
    FactorType ftype = FactorType::F32;
    Kind kind = Kind::Mttkrp;
    const void* in_factors[kMaxOrder - 1] = {};    // input-mode factors, modes ascending
    int64_t in_rows[kMaxOrder - 1] = {};           // their row counts
    const int32_t* in_hot[kMaxOrder - 1] = {};     // their hot-row tables
    const float* own_factor = nullptr;             // factor of the output mode (ResidualGrad)
    float scale = 1.0f;                            // ResidualGrad output scale
    float* out = nullptr;
    double* loss = nullptr;                        // ResidualGradLoss: fp64 loss
    bool loss_accumulate = false;                  // add to *loss instead of resetting it
    hipStream_t stream = nullptr;
};

// Enqueue init + MTTKRP (or fused residual gradient).  Returns hipSuccess or the
// launch error.
hipError_t launch_mttkrp(const LaunchArgs& a);

// Enqueue the CP loss over the given layout (any mode's layout holds every
// nonzero once).  all_factors are in mode order with the layout's output mode
// first resolved by the caller: own_factor = factor of the layout's mode.
struct LossArgs {
    const ModeDev* m = nullptr;
    int order = 0;
    int rank = 0;
    const float* own_factor = nullptr;
    const float* in_factors[kMaxOrder - 1] = {};
    int64_t in_rows[kMaxOrder - 1] = {};
    const int32_t* in_hot[kMaxOrder - 1] = {};
    double* loss = nullptr;
    bool accumulate = false;                       // add to *loss instead of resetting it
    hipStream_t stream = nullptr;
};
hipError_t launch_cp_loss(const LossArgs& a);

#if AMPED_QUEUE_STATS
// Diagnostic build: copy the per-wave work-queue records of the last
// MTTKRP-shaped launch (4 words each: chunks, nonzeros, first-pop time, exit
// time) after synchronising the device.
hipError_t queue_stats_copy(unsigned long long* host, int64_t max_records, int64_t* n_records, int* waves_per_block);
#endif

// CP-ALS building blocks (csrc/als.hip).  G = A^T A (fp64) of a rows x R fp32
// matrix, R <= 128, via gram_slabs(rows) x R x R fp32 partials.
int64_t gram_slabs(int64_t rows);
hipError_t launch_gram(const float* A, int64_t rows, int R, float* partial, double* G, hipStream_t st,
                       int64_t nslab = 0);
// The same with the partial sums in the library's fixed device array (no
// allocation): at most gram_noalloc_slabs(rows, R) <= gram_slabs(rows) slabs,
// so that they fit its 32 MiB.
int64_t gram_noalloc_slabs(int64_t rows, int R);
hipError_t launch_gram_noalloc(const float* A, int64_t rows, int R, double* G, hipStream_t st);
// The R x R algebra of the mode-d update (scratch: 4 R x R doubles); G is
// [N][R][R] and G[d] is replaced by the Gram matrix of the new factor.
hipError_t launch_als_small(double* G, const double* S, int N, int d, int R, double* scratch, double* W, int* wide,
                            double* lambda, bool last, const double* xnorm2, double* fit, hipStream_t st);
// A = M W: M and A rows x R fp32, W R x R fp64; the sums in fp64 when als_small
// set *wide (V ill-conditioned), else in fp32.
hipError_t launch_als_solve(const float* M, const double* W, const int* wide, float* A, int64_t rows, int R,
                            hipStream_t st);
// ||X||^2 over a layout whose exact duplicates are adjacent (accumulate: add
// to *result; no run of duplicates may cross the layout's ends then).
hipError_t launch_tensor_norm2(const ModeDev& m, int nin, double* result, bool accumulate, hipStream_t st);

// dst[p] = src[perm[p]] for p < n, 32-bit words, on the device.
hipError_t launch_permute32(void* dst, const void* src, const int32_t* perm, int64_t n, hipStream_t st);

}  // namespace amped
