/*
 * amped.h -- C ABI of the MI355X (gfx950) sparse MTTKRP library.
 *
 * The operation is MTTKRP on a sparse tensor along every mode (Eq. 1 in
 * Sec. 2.1 of Wijeratne, Kannan and Prasanna, "AMPED: Accelerating MTTKRP for
 * Billion-Scale Sparse Tensor Decomposition on Multiple GPUs", ICPP'25):
 *
 *     Y_d[i, r] = sum over nonzeros k with i_d(k) = i of
 *                 val(k) * prod_{w != d} A_w[i_w(k), r]
 *
 * i.e. the elementwise computation ("EC", Sec. 3) summed into a zeroed
 * output.  Beside it: the same computation with bfloat16 factor matrices and
 * fp32 accumulation, and the sparse CP least-squares loss over the nonzeros
 * with its gradient (CP model of Sec. 2.1), whose backward is MTTKRP on the
 * residuals fused with the residual computation.
 *
 * Conventions that hold for every call:
 *  - Every function returns an amped_status; on a non-OK status nothing was
 *    enqueued and amped_last_error() returns a message (thread-local, valid
 *    until the next call on the same thread).  No C++ exception crosses the
 *    ABI.
 *  - Index arrays are int32 in the [order][nnz] layout (mode-major, the same
 *    layout as torch's COO indices), values are fp32.
 *  - Factor matrices and outputs are caller-owned DEVICE buffers, row-major,
 *    row stride = rank elements, 16-byte aligned.  They must stay alive until
 *    the stream's work completes; the library never frees or keeps them.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Launches are asynchronous; device faults surface at the caller's next
 *    synchronisation.
 *  - A tensor handle is immutable after creation and binds the HIP device that
 *    was current at creation.  It owns a small device work queue per mode, so
 *    calls that use the same handle AND the same mode (or two cp_loss calls)
 *    must be ordered on one stream; calls on different modes may overlap,
 *    except on a handle with host-resident layouts (options.host_layout),
 *    whose calls share its shard buffers and must all be ordered on one
 *    stream.  amped_cp_als_sweep calls on one handle must not overlap.
 *  - Limits: 2 <= order <= 8; 1 <= dims[w] <= 2^31-1; 0 <= nnz <= 2^31-1;
 *    1 <= rank <= 4096.
 */
#ifndef AMPED_H
#define AMPED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amped_tensor_s *amped_tensor_t;

typedef enum {
    AMPED_OK = 0,
    AMPED_ERR_INVALID = 1,     /* null pointer, bad order/mode/rank/size, misalignment   */
    AMPED_ERR_RANGE = 2,       /* an index outside [0, dims[w]) at creation              */
    AMPED_ERR_NOMEM = 3,       /* host or device allocation failed, or byte cap exceeded */
    AMPED_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed             */
    AMPED_ERR_UNSUPPORTED = 5  /* no usable gfx950 device, or a case not implemented     */
} amped_status;

/* Creation options; pass NULL for the defaults. */
typedef struct {
    int64_t chunk_nnz;        /* CH: nonzeros per work-queue chunk, <= 2^28; 0 = 4096.  Part of
                                 the layout contract (chunk k holds positions
                                 [k*CH, min((k+1)*CH, nnz)) of a mode's order).        */
    int64_t device_byte_cap;  /* 0 = no cap; otherwise creation fails with NOMEM,
                                 before touching the device, if the layouts would
                                 need more device bytes than this.                     */
    int32_t keep_perm;        /* 1 = keep each mode's permutation (on the device, or
                                 in host memory with host_layout) so
                                 amped_tensor_layout can return it.                    */
    int32_t host_layout;      /* 1 = keep the per-mode layouts in pinned host memory
                                 (built by the host order builder) and stream them to
                                 the device in shards on every call: for tensors whose
                                 layouts do not fit in device memory (out-of-core
                                 shard streaming, Sec. 4.8).  The device then holds
                                 two shard buffers and the per-mode row lists only.
                                 Results equal those of a device-resident tensor up
                                 to fp32 summation order.  0 = device-resident.      */
    int64_t shard_nnz;        /* host_layout: nonzeros per streamed shard, rounded up
                                 to whole chunks; 0 = 2^25.  Ignored otherwise.       */
} amped_options;

/*
 * Build the per-mode layouts of a COO tensor and copy them to the current HIP
 * device.  The paper keeps one copy of the tensor per output mode with all
 * nonzeros of an output index together (Sec. 3, "Tensor Partitioning"; Sec.
 * 3.1 tensor sharding) and splits it into equal-size inter-shard partitions
 * (Sec. 3.1/3.2); here, for every mode d, the nonzeros are put in the order
 * of the key (i_d, then the other indices in ascending mode order), exact
 * duplicates keeping their input order, and that order is cut into chunks of
 * CH nonzeros that the kernels take from a work queue.
 *
 *   order    number of modes N (2..8)
 *   dims     host, [order] mode sizes
 *   nnz      number of stored entries (duplicates allowed; they add up)
 *   indices  host, int32 [order][nnz]; need not be sorted
 *   values   host, fp32 [nnz]
 *   opts     host, nullable
 *   out      host, receives the handle (set to NULL on failure)
 *
 * The orders are computed on the device (stable radix sorts; the same order
 * amped_layout_host computes on the host), or on the host with host_layout.
 * The caller's host arrays are only read during the call.  Errors: INVALID for bad arguments, RANGE for an index
 * outside its mode, NOMEM, HIP, UNSUPPORTED (no device).
 */
amped_status amped_tensor_create(int order, const int64_t *dims, int64_t nnz,
                                 const int32_t *indices, const float *values,
                                 const amped_options *opts, amped_tensor_t *out);

/*
 * Release a tensor: the N per-mode copies of the tensor that the paper keeps
 * for the N output modes (Sec. 3, "Tensor Partitioning"; Table 1, copies of
 * the tensor) and the handle's work queues and row lists.  Synchronises the
 * handle's device first, then frees everything the handle owns; the caller's
 * factors and outputs are untouched.  NULL is a no-op.  Errors: HIP if the
 * synchronisation reports an earlier device fault (the handle is freed anyway).
 */
amped_status amped_tensor_destroy(amped_tensor_t t);

/*
 * Shape and layout facts of a tensor (all outputs host and nullable):
 *   order; dims[order]; nnz;
 *   chunk_nnz (CH) and n_chunks = ceil(nnz / CH): the size and number of the
 *     equal-size partitions each mode's copy is cut into (Sec. 3.1/3.2,
 *     inter-shard partitioning);
 *   touched[order] = distinct output indices per mode, i.e. the rows of the
 *     mode's MTTKRP output that some nonzero updates (Sec. 3.1: all nonzeros
 *     of one output index sit in one partition run);
 *   device_bytes = device memory the handle owns.
 * Errors: INVALID for a NULL tensor.
 */
amped_status amped_tensor_info(amped_tensor_t t, int *order, int64_t *dims, int64_t *nnz,
                               int64_t *chunk_nnz, int64_t *n_chunks, int64_t *touched,
                               int64_t *device_bytes);

/*
 * Copy mode `mode`'s layout -- the mode's copy of the tensor with all
 * nonzeros of one output index together (Sec. 3.1, tensor sharding), in the
 * key order described at amped_tensor_create, cut into equal-size partitions
 * (Sec. 3.1/3.2) -- from the device, or from the pinned host copy with
 * host_layout, to host arrays (introspection and tests; synchronous).
 * Errors: INVALID for a NULL tensor, a bad mode, or perm requested without
 * keep_perm; HIP if a copy fails.  All outputs are nullable:
 *   perm        int32 [nnz]   position -> input nonzero (needs keep_perm=1,
 *                             else INVALID when requested)
 *   out_idx     int32 [nnz]   i_mode in layout order (non-decreasing)
 *   in_idx      int32 [order-1][nnz]  the other indices, modes ascending
 *   values      fp32  [nnz]
 *   chunk_flags uint8 [n_chunks]  bit0: chunk's first output index continues
 *               from the previous chunk; bit1: its last one continues into the
 *               next chunk.
 */
amped_status amped_tensor_layout(amped_tensor_t t, int mode, int32_t *perm, int32_t *out_idx,
                                 int32_t *in_idx, float *values, uint8_t *chunk_flags);

/*
 * The same per-mode order and chunk flags, computed on the host only (no
 * device involved): the host preprocessing that builds a mode's partitioned
 * copy of the tensor (Sec. 3.1/3.2; its cost is the preprocessing time of
 * Sec. 5.7).  It is the builder amped_tensor_create uses with host_layout,
 * and its order is the one the device builder produces.
 *   indices     host, int32 [order][nnz], need not be sorted
 *   perm        host, int32 [nnz], position -> input nonzero (nullable)
 *   chunk_flags host, uint8 [ceil(nnz/chunk_nnz)] (nullable)
 * Errors: INVALID for bad arguments or chunk_nnz < 1, RANGE for an index
 * outside its mode, NOMEM.
 */
amped_status amped_layout_host(int order, const int64_t *dims, int64_t nnz,
                               const int32_t *indices, int mode, int64_t chunk_nnz,
                               int32_t *perm, uint8_t *chunk_flags);

/*
 * MTTKRP along `mode` (Eq. 1, Sec. 2.1; one GPU's share of Alg. 1's mode
 * loop, Sec. 4.6): out[i, r] = sum_{k: i_mode(k)=i} val(k) prod_{w!=mode}
 * factors[w][i_w(k), r], computed in fp32.
 *
 *   factors  host array of `order` DEVICE pointers, factors[w] is dims[w] x rank
 *            fp32 row-major; factors[mode] is not read (may be NULL)
 *   out      DEVICE, dims[mode] x rank fp32, fully overwritten (rows with no
 *            nonzero become 0); must not alias a factor
 *   stream   hipStream_t or NULL
 *
 * Errors (synchronous, nothing enqueued): INVALID for a bad mode/rank, a NULL
 * or misaligned pointer; HIP if a launch fails.
 *
 * The most-used rows of each input factor (from the layout's index counts)
 * are read from an on-chip copy made at launch; results are identical either
 * way.  The environment variable AMPED_HOT_MAX, read once per process, caps
 * the rows kept per factor (0 turns the copy off).  Also applies to
 * amped_mttkrp_bf16.
 */
amped_status amped_mttkrp(amped_tensor_t t, int mode, int rank, const float *const *factors,
                          float *out, void *stream);

/*
 * MTTKRP with bfloat16 factor matrices: factors[w] holds dims[w] x rank bf16
 * bit patterns (uint16, row-major, 16-byte aligned).  Each factor value is
 * widened exactly to fp32; products, accumulation and the fp32 output are as
 * in amped_mttkrp.  Index arithmetic and segment boundaries are unchanged.
 */
amped_status amped_mttkrp_bf16(amped_tensor_t t, int mode, int rank,
                               const uint16_t *const *factors, float *out, void *stream);

/*
 * Sparse CP loss at the stored entries (CP model of Sec. 2.1):
 *   *loss = sum_k (val(k) - sum_r prod_w factors[w][i_w(k), r])^2
 * Per-entry work in fp32, the sum over entries accumulated in fp64.
 *   factors  host array of `order` DEVICE fp32 pointers (all read)
 *   loss     DEVICE, one double, overwritten
 */
amped_status amped_cp_loss(amped_tensor_t t, int rank, const float *const *factors,
                           double *loss, void *stream);

/*
 * Gradient of the loss above with respect to factors[mode], times -scale/2:
 *   grad[i, r] = scale * sum_{k: i_mode(k)=i} e(k) prod_{w!=mode} factors[w][i_w(k), r]
 * with e(k) = val(k) - sum_r prod_w factors[w][i_w(k), r] recomputed on the
 * fly in the same kernel (nothing per entry is stored).  With
 * scale = -2 * dL_out the result is dL_out * dLoss/dfactors[mode].
 *   grad  DEVICE, dims[mode] x rank fp32, fully overwritten; must not alias a factor
 */
amped_status amped_cp_grad(amped_tensor_t t, int mode, int rank, const float *const *factors,
                           float scale, float *grad, void *stream);

/*
 * amped_cp_grad and amped_cp_loss in one pass over the layout of `mode` (the
 * CP model of Sec. 2.1 and the gradient of its loss): every mode's layout
 * holds every stored entry, so the residuals e(k) the gradient recomputes
 * also give the loss.  A training step that needs the loss and every
 * factor's gradient then reads the tensor N times instead of N + 1.
 *   grad   as in amped_cp_grad (the same bits)
 *   loss   DEVICE, one double, overwritten with sum_k e(k)^2 (fp64 sum of
 *          fp32 per-entry residuals; the entries are added in the order of
 *          this mode's layout, so the last bits may differ from amped_cp_loss)
 * Errors as in amped_cp_grad; INVALID also for a NULL loss.
 */
amped_status amped_cp_loss_grad(amped_tensor_t t, int mode, int rank, const float *const *factors,
                                float scale, float *grad, double *loss, void *stream);

/*
 * Gram matrix G = A^T A of a dense matrix, the R x R building block of the
 * CP-ALS update (V = Hadamard product of the other factors' Gram matrices).
 * Products on the matrix cores in fp32, per-slab partial sums added in fp64
 * in a fixed order (deterministic).
 *   A     DEVICE, rows x rank fp32 row-major (rows >= 1, 1 <= rank <= 128)
 *   G     DEVICE, rank x rank fp64 row-major, overwritten
 * Stream-ordered temporary memory (hipMallocAsync) holds the partial sums.
 */
amped_status amped_gram(const float *A, int64_t rows, int rank, double *G, void *stream);

/*
 * amped_gram without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, and harnesses
 * that forbid hipMalloc.  The result is amped_gram's (bit for bit up to rank
 * 64; for larger ranks with many rows the rows are split into fewer slabs, so
 * the fp64 sum of the fp32 slab partials may differ in the last bits).
 *   A, rows, rank, G, stream  as in amped_gram
 * The per-slab partial sums go to a fixed 32 MiB device array that the
 * library keeps on every device it runs on until the process ends (no
 * hipMalloc, hipFree or allocating call).  Every call on one device uses the
 * same array and overwrites every entry it reads, so calls that overlap on
 * one device (on different streams, or from different threads) race and must
 * be ordered by the caller.  The first call on a device looks up the array's
 * device address.  Errors: INVALID for a NULL pointer, rows < 1, or a rank
 * outside [1, 128] (larger ranks' partial sums exceed the array); UNSUPPORTED
 * for a device that is not gfx950; HIP for a failed launch.
 */
amped_status amped_gram_noalloc(const float *A, int64_t rows, int rank, double *G, void *stream);

/*
 * One CP-ALS sweep (CPD by alternating least squares, Sec. 2.1; the mode
 * loop of Alg. 1 with the standard least-squares update after each MTTKRP):
 * for d = 0..N-1
 *   M = MTTKRP_d(factors)                        (amped_mttkrp)
 *   V = Hadamard over w != d of factors[w]^T factors[w]
 *   factors[d] = M V^{-1} with unit 2-norm columns; lambda = the column norms
 *                (a zero column stays zero with lambda 0)
 * and after the last mode the fit 1 - ||X - Xhat|| / ||X|| of the CP model
 * Xhat = sum_r lambda_r a_r o b_r o ... to the full tensor (entries not
 * stored are zeros; exact duplicates add up).  The R x R algebra runs in
 * fp64 (V^{-1} by Gauss-Jordan elimination; a non-positive pivot is replaced
 * by a tiny one), the row-sized products in fp32.  The fit comes from
 * ||X||^2 - 2<X, Xhat> + ||Xhat||^2, so with fp32 products its absolute error
 * is about 1e-6 / (1 - fit), at most about 2e-3 as the fit nears 1.
 *   factors  host array of `order` DEVICE pointers, each dims[w] x rank fp32,
 *            16-byte aligned; read, and factors[d] overwritten in mode order
 *   lambda   DEVICE, rank doubles (16-byte aligned), overwritten
 *   fit      DEVICE, one double, overwritten
 *   flags    AMPED_ALS_REUSE_GRAMS: the factors are exactly those the
 *            previous sweep on this tensor, at this rank, left; the Gram
 *            matrices it kept are used instead of being recomputed (INVALID
 *            if there is no such sweep).  0 otherwise.
 * 1 <= rank <= 128.  The tensor keeps a workspace for the rank of its last
 * sweep (max_d dims[d] x rank floats plus small R x R arrays); sweeps on one
 * tensor must not overlap.  With host_layout, the one-time ||X||^2 pass is
 * streamed as well, in shards cut between runs of equal coordinates; a run
 * longer than a shard returns UNSUPPORTED.
 */
#define AMPED_ALS_REUSE_GRAMS 1u
amped_status amped_cp_als_sweep(amped_tensor_t t, int rank, float *const *factors, double *lambda,
                                double *fit, unsigned flags, void *stream);

/*
 * Message for the last non-OK status on this thread ("" if none).  Not an
 * operation of the paper: the error channel of every call above (the paper's
 * Alg. 1-3 define no failure behaviour).  The string is owned by the library
 * and valid until the next call on the same thread.
 */
const char *amped_last_error(void);

/* Library version string (static storage).  Not an operation of the paper. */
const char *amped_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AMPED_H */
