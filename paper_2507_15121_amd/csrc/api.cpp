// C ABI of the sparse MTTKRP library (declared in include/amped.h): argument
// checks, handle lifetime, the per-mode layout build (host order, device
// gather) and the kernel launches.
#include <hip/hip_runtime_api.h>
#include <omp.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "amped.h"
#if AMPED_QUEUE_STATS
#include "amped_diag.h"
#endif
#include "internal.h"

using amped::HostModeLayout;
using amped::kMaxOrder;
using amped::kSinkFloats;
using amped::ModeDev;

namespace {

thread_local std::string g_err;

amped_status fail(amped_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

amped_status hip_fail(hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(AMPED_ERR_NOMEM, "%s: out of device memory (%s)", what, hipGetErrorString(e));
    if (e == hipErrorNotSupported) return fail(AMPED_ERR_UNSUPPORTED, "%s: case not supported", what);
    return fail(AMPED_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = (prev == dev) || hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (ok && prev >= 0) (void)hipSetDevice(prev);
    }
};

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

struct amped_tensor_s {
    int order = 0;
    int64_t dims[kMaxOrder] = {};
    int64_t nnz = 0, chunk = 0, n_chunks = 0;
    int device = 0;
    bool keep_perm = false;
    int64_t device_bytes = 0;
    std::vector<void*> allocs;
    ModeDev mode[kMaxOrder];
    ModeDev loss_dev;                       // mode-0 layout with its own queue
    int32_t* perm[kMaxOrder] = {};
    std::vector<uint8_t> flags[kMaxOrder];
    int64_t touched[kMaxOrder] = {};
    // Host-resident layouts (options.host_layout): each mode's arrays in
    // pinned host memory, streamed to two device staging buffers per call.
    bool host_layout = false;
    int64_t stage_len = 0;  // nonzeros per shard (whole chunks)
    struct HostMode {
        int32_t* out_idx = nullptr;
        int32_t* in_idx[kMaxOrder - 1] = {};
        float* val = nullptr;
    } hmode[kMaxOrder];
    std::vector<void*> pinned;
    std::vector<int32_t> hperm[kMaxOrder];  // kept permutations (keep_perm)
    void* stage[2] = {};                    // (order + 1) arrays of stage_len + 4 entries each
    hipStream_t copy_stream = nullptr;
    hipEvent_t copied[2] = {}, consumed[2] = {}, call_start = nullptr;
    // CP-ALS workspace, allocated by the first sweep of a rank
    struct AlsWork {
        int rank = 0;
        float* M = nullptr;        // MTTKRP output, max_d I_d x R
        double* G = nullptr;       // [N][R][R] Gram matrices
        double* S = nullptr;       // R x R, M^T M
        float* partial = nullptr;  // Gram partials
        double* scratch = nullptr; // 4 R x R
        double* W = nullptr;       // R x R, V^{-1} D^{-1}
        int* wide = nullptr;       // set by als_small: the product M W sums in fp64
        double* xnorm2 = nullptr;  // ||X||^2 (computed once)
        bool have_xnorm2 = false;
        bool have_grams = false;   // G matches the factors the last sweep wrote
    } als;

    hipError_t alloc(void** p, size_t bytes)
    {
        *p = nullptr;
        if (bytes == 0) return hipSuccess;
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) {
            allocs.push_back(*p);
            device_bytes += (int64_t)bytes;
        }
        return e;
    }
    void release(void* p)
    {
        for (auto& a : allocs)
            if (a == p) {
                (void)hipFree(a);
                a = nullptr;
            }
    }
    hipError_t host_alloc(void** p, size_t bytes)
    {
        *p = nullptr;
        if (bytes == 0) return hipSuccess;
        hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
        if (e == hipSuccess) pinned.push_back(*p);
        return e;
    }
    void free_all()
    {
        for (void* a : allocs)
            if (a) (void)hipFree(a);
        allocs.clear();
        for (void* a : pinned) (void)hipHostFree(a);
        pinned.clear();
        for (hipEvent_t& ev : {std::ref(copied[0]), std::ref(copied[1]), std::ref(consumed[0]), std::ref(consumed[1]),
                               std::ref(call_start)})
            if (ev) {
                (void)hipEventDestroy(ev);
                ev = nullptr;
            }
        if (copy_stream) {
            (void)hipStreamDestroy(copy_stream);
            copy_stream = nullptr;
        }
    }
};

namespace {

// Bits needed to hold the values 0..n (0 for n <= 0).
int bits_for(int64_t n)
{
    int b = 0;
    while (b < 63 && n > 0 && (n >> b)) ++b;
    return b;
}

amped_status validate_coo(int order, const int64_t* dims, int64_t nnz, const int32_t* indices, const float* values)
{
    if (order < 2 || order > kMaxOrder) return fail(AMPED_ERR_INVALID, "order %d outside [2, %d]", order, kMaxOrder);
    if (!dims) return fail(AMPED_ERR_INVALID, "dims is NULL");
    for (int w = 0; w < order; ++w)
        if (dims[w] < 1 || dims[w] > 0x7FFFFFFF)
            return fail(AMPED_ERR_INVALID, "dims[%d] = %lld outside [1, 2^31-1]", w, (long long)dims[w]);
    if (nnz < 0 || nnz > 0x7FFFFFFF) return fail(AMPED_ERR_INVALID, "nnz = %lld outside [0, 2^31-1]", (long long)nnz);
    if (nnz > 0 && (!indices || !values)) return fail(AMPED_ERR_INVALID, "indices or values is NULL");
    for (int w = 0; w < order; ++w) {
        const int32_t* col = indices + (int64_t)w * nnz;
        const int64_t dim = dims[w];
        int64_t bad = nnz;
#pragma omp parallel for reduction(min : bad) schedule(static)
        for (int64_t k = 0; k < nnz; ++k)
            if (col[k] < 0 || col[k] >= dim) bad = std::min(bad, k);
        if (bad < nnz)
            return fail(AMPED_ERR_RANGE, "indices[%d][%lld] = %d outside [0, %lld)", w, (long long)bad, col[bad],
                        (long long)dim);
    }
    return AMPED_OK;
}

amped_status check_device(int* dev)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(AMPED_ERR_UNSUPPORTED, "no HIP device");
    if (hipGetDevice(dev) != hipSuccess) return fail(AMPED_ERR_UNSUPPORTED, "no current HIP device");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, *dev) != hipSuccess)
        return fail(AMPED_ERR_UNSUPPORTED, "cannot query device %d", *dev);
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(AMPED_ERR_UNSUPPORTED, "device %d is %s, this library is built for gfx950", *dev, prop.gcnArchName);
    return AMPED_OK;
}

#define HIP_OR_FAIL(call, what)                          \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) {                          \
            st = hip_fail(e_, what);                     \
            goto cleanup;                                \
        }                                                \
    } while (0)

// A mode's row lists (zero rows, hot-row tables, long gaps) to the device,
// and its sizes.
amped_status upload_tables(amped_tensor_s* t, ModeDev& m, int d, const HostModeLayout& lay, void* queues, void* aux)
{
    amped_status st = AMPED_OK;
    void* p = nullptr;
    if (!lay.zero_rows.empty()) {
        HIP_OR_FAIL(t->alloc(&p, lay.zero_rows.size() * 4), "hipMalloc(zero rows)");
        HIP_OR_FAIL(hipMemcpy(p, lay.zero_rows.data(), lay.zero_rows.size() * 4, hipMemcpyHostToDevice),
                    "hipMemcpy(zero rows)");
        m.zero_rows = static_cast<int32_t*>(p);
    }
    HIP_OR_FAIL(t->alloc(&p, lay.hot.size() * 4), "hipMalloc(hot rows)");
    HIP_OR_FAIL(hipMemcpy(p, lay.hot.data(), lay.hot.size() * 4, hipMemcpyHostToDevice), "hipMemcpy(hot rows)");
    m.hot = static_cast<int32_t*>(p);
    if (!lay.gaps.empty()) {
        HIP_OR_FAIL(t->alloc(&p, lay.gaps.size() * 4), "hipMalloc(gaps)");
        HIP_OR_FAIL(hipMemcpy(p, lay.gaps.data(), lay.gaps.size() * 4, hipMemcpyHostToDevice), "hipMemcpy(gaps)");
        m.gaps = static_cast<int32_t*>(p);
    }
    m.nnz = t->nnz;
    m.chunk = t->chunk;
    m.n_chunks = t->n_chunks;
    m.rows = t->dims[d];
    m.n_zero = (int64_t)lay.zero_rows.size();
    m.zero_row = aux;
    m.sink = static_cast<float*>(aux) + 4;
    m.n_gaps = (int64_t)lay.gaps.size() / 2;
    m.queue = static_cast<unsigned*>(queues) + (size_t)d * amped::kQueueSlots;
    t->flags[d] = lay.flags;
    t->touched[d] = lay.touched;
cleanup:
    return st;
}

// Host-resident layouts: the host order builder sorts every mode, the layout
// arrays are gathered into pinned host memory, and the device receives the
// row lists, two shard staging buffers, a copy stream and its events.
amped_status build_host_layout(amped_tensor_s* t, const int32_t* indices, const float* values)
{
    const int order = t->order;
    const int64_t nnz = t->nnz;
    amped_status st = AMPED_OK;
    void* queues = nullptr;
    void* aux = nullptr;
    void* p = nullptr;
    HIP_OR_FAIL(t->alloc(&queues, (size_t)(order + 1) * amped::kQueueSlots * sizeof(unsigned)), "hipMalloc(queues)");
    HIP_OR_FAIL(hipMemset(queues, 0, (size_t)(order + 1) * amped::kQueueSlots * sizeof(unsigned)), "hipMemset(queues)");
    HIP_OR_FAIL(t->alloc(&aux, (size_t)(4 + kSinkFloats) * sizeof(float)), "hipMalloc(aux)");
    HIP_OR_FAIL(hipMemset(aux, 0, (size_t)(4 + kSinkFloats) * sizeof(float)), "hipMemset(aux)");
    for (int b = 0; b < 2; ++b) {
        HIP_OR_FAIL(t->alloc(&t->stage[b], (size_t)(order + 1) * (t->stage_len + 4) * 4), "hipMalloc(staging)");
        HIP_OR_FAIL(hipMemset(t->stage[b], 0, (size_t)(order + 1) * (t->stage_len + 4) * 4), "hipMemset(staging)");
        HIP_OR_FAIL(hipEventCreateWithFlags(&t->copied[b], hipEventDisableTiming), "hipEventCreate");
        HIP_OR_FAIL(hipEventCreateWithFlags(&t->consumed[b], hipEventDisableTiming), "hipEventCreate");
    }
    HIP_OR_FAIL(hipEventCreateWithFlags(&t->call_start, hipEventDisableTiming), "hipEventCreate");
    HIP_OR_FAIL(hipStreamCreateWithFlags(&t->copy_stream, hipStreamNonBlocking), "hipStreamCreate");
    try {
        const std::vector<int32_t> lex = amped::lex_order(order, t->dims, nnz, indices);
        const size_t padded = ((size_t)nnz + 4) * 4;
        for (int d = 0; d < order; ++d) {
            HostModeLayout lay;
            amped::mode_order(t->dims, nnz, indices, lex, d, lay.perm);
            amped::mode_tables(t->dims, nnz, indices, d, t->chunk, lay);
            auto& h = t->hmode[d];
            HIP_OR_FAIL(t->host_alloc(&p, padded), "hipHostMalloc(out_idx)");
            h.out_idx = static_cast<int32_t*>(p);
            amped::gather_i32(indices + (int64_t)d * nnz, lay.perm.data(), 0, nnz, h.out_idx);
            int j = 0;
            for (int w = 0; w < order; ++w) {
                if (w == d) continue;
                HIP_OR_FAIL(t->host_alloc(&p, padded), "hipHostMalloc(in_idx)");
                h.in_idx[j] = static_cast<int32_t*>(p);
                amped::gather_i32(indices + (int64_t)w * nnz, lay.perm.data(), 0, nnz, h.in_idx[j++]);
            }
            HIP_OR_FAIL(t->host_alloc(&p, padded), "hipHostMalloc(values)");
            h.val = static_cast<float*>(p);
            amped::gather_f32(values, lay.perm.data(), 0, nnz, h.val);
            for (int k = 0; k < 4; ++k) {
                h.out_idx[nnz + k] = 0;
                for (int jj = 0; jj < order - 1; ++jj) h.in_idx[jj][nnz + k] = 0;
                h.val[nnz + k] = 0.f;
            }
            st = upload_tables(t, t->mode[d], d, lay, queues, aux);
            if (st != AMPED_OK) return st;
            if (t->keep_perm) t->hperm[d] = std::move(lay.perm);
        }
    } catch (const std::bad_alloc&) {
        return fail(AMPED_ERR_NOMEM, "host allocation failed");
    }
    t->loss_dev = t->mode[0];
    t->loss_dev.queue = static_cast<unsigned*>(queues) + (size_t)order * amped::kQueueSlots;
cleanup:
    return st;
}

// Streams mode d's host-resident layout through the device: shard i goes to
// staging buffer i % 2 on the copy stream, stream s waits for it, runs
// fn(shard, i) and marks the buffer free again, so the copy of shard i+1
// overlaps the kernels of shard i.  cut(start) is a shard's end (at most
// stage_len nonzeros past start).  The shard's ModeDev points at the staging
// arrays, carries the output indices on both sides of it, and only the
// first shard's init zeroes rows.
template <typename Cut, typename Fn>
amped_status stream_shards(amped_tensor_s* t, int d, const ModeDev& base, hipStream_t s, Cut&& cut, Fn&& fn)
{
    const int order = t->order;
    const int64_t nnz = t->nnz;
    const auto& h = t->hmode[d];
    if (nnz == 0) return fn(base, 0);
    hipError_t e;
    // the staging buffers may still be read by earlier work on s
    if ((e = hipEventRecord(t->call_start, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(t->copy_stream, t->call_start, 0)) != hipSuccess)
        return hip_fail(e, "hipStreamWaitEvent");
    const size_t stride = (size_t)t->stage_len + 4;
    int i = 0;
    for (int64_t start = 0; start < nnz; ++i) {
        const int64_t end = cut(start);
        if (end <= start || end - start > t->stage_len)
            return fail(AMPED_ERR_UNSUPPORTED, "a run of equal coordinates is longer than a shard (%lld nonzeros)",
                        (long long)t->stage_len);
        const int64_t len = end - start;
        const int b = i & 1;
        if (i >= 2 && (e = hipStreamWaitEvent(t->copy_stream, t->consumed[b], 0)) != hipSuccess)
            return hip_fail(e, "hipStreamWaitEvent");
        int32_t* sb = static_cast<int32_t*>(t->stage[b]);
        ModeDev m = base;
        auto put = [&](int slot, const void* src) {
            return hipMemcpyAsync(sb + slot * stride, static_cast<const int32_t*>(src) + start, (size_t)len * 4,
                                  hipMemcpyHostToDevice, t->copy_stream);
        };
        if ((e = put(0, h.out_idx)) != hipSuccess) return hip_fail(e, "hipMemcpyAsync(shard)");
        m.out_idx = sb;
        for (int j = 0; j < order - 1; ++j) {
            if ((e = put(1 + j, h.in_idx[j])) != hipSuccess) return hip_fail(e, "hipMemcpyAsync(shard)");
            m.in_idx[j] = sb + (1 + j) * stride;
        }
        if ((e = put(order, h.val)) != hipSuccess) return hip_fail(e, "hipMemcpyAsync(shard)");
        m.val = reinterpret_cast<const float*>(sb + order * stride);
        if ((e = hipEventRecord(t->copied[b], t->copy_stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = hipStreamWaitEvent(s, t->copied[b], 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        m.nnz = len;
        m.n_chunks = (len + t->chunk - 1) / t->chunk;
        m.prev_key = start > 0 ? h.out_idx[start - 1] : -1;
        m.next_key = end < nnz ? h.out_idx[end] : -1;
        if (i > 0) {
            m.n_zero = 0;
            m.n_gaps = 0;
        }
        amped_status st = fn(m, i);
        if (st != AMPED_OK) return st;
        if ((e = hipEventRecord(t->consumed[b], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        start = end;
    }
    return AMPED_OK;
}

// Shard ends for the MTTKRP-shaped kernels: whole chunks, stage_len each.
struct ChunkCut {
    int64_t nnz, len;
    int64_t operator()(int64_t start) const { return std::min(start + len, nnz); }
};

}  // namespace

extern "C" {

const char* amped_last_error(void) { return g_err.c_str(); }

const char* amped_version(void) { return "amped 0.1.0 (gfx950)"; }

amped_status amped_layout_host(int order, const int64_t* dims, int64_t nnz, const int32_t* indices, int mode,
                               int64_t chunk_nnz, int32_t* perm, uint8_t* chunk_flags)
{
    g_err.clear();
    static const float dummy = 0.f;
    amped_status st = validate_coo(order, dims, nnz, indices, nnz ? &dummy : nullptr);
    if (st != AMPED_OK) return st;
    if (mode < 0 || mode >= order) return fail(AMPED_ERR_INVALID, "mode %d outside [0, %d)", mode, order);
    if (chunk_nnz < 1) return fail(AMPED_ERR_INVALID, "chunk_nnz must be >= 1");
    try {
        std::vector<int32_t> lex = amped::lex_order(order, dims, nnz, indices);
        HostModeLayout lay;
        amped::mode_order(dims, nnz, indices, lex, mode, lay.perm);
        amped::mode_tables(dims, nnz, indices, mode, chunk_nnz, lay);
        if (perm && nnz) std::memcpy(perm, lay.perm.data(), (size_t)nnz * sizeof(int32_t));
        if (chunk_flags && !lay.flags.empty()) std::memcpy(chunk_flags, lay.flags.data(), lay.flags.size());
    } catch (const std::bad_alloc&) {
        return fail(AMPED_ERR_NOMEM, "host allocation failed");
    }
    return AMPED_OK;
}

amped_status amped_tensor_create(int order, const int64_t* dims, int64_t nnz, const int32_t* indices,
                                 const float* values, const amped_options* opts, amped_tensor_t* out)
{
    g_err.clear();
    if (!out) return fail(AMPED_ERR_INVALID, "out is NULL");
    *out = nullptr;
    amped_status st = validate_coo(order, dims, nnz, indices, values);
    if (st != AMPED_OK) return st;
    int64_t chunk = amped::kDefaultChunk, cap = 0, shard_opt = 0;
    bool keep_perm = false, host_layout = false;
    if (opts) {
        if (opts->host_layout != 0 && opts->host_layout != 1)
            return fail(AMPED_ERR_INVALID, "host_layout must be 0 or 1");
        host_layout = opts->host_layout == 1;
        if (opts->shard_nnz < 0) return fail(AMPED_ERR_INVALID, "shard_nnz < 0");
        shard_opt = opts->shard_nnz;
        if (opts->chunk_nnz < 0 || opts->chunk_nnz > amped::kMaxChunk)
            return fail(AMPED_ERR_INVALID, "chunk_nnz %lld outside [0, 2^28]", (long long)opts->chunk_nnz);
        if (opts->chunk_nnz > 0) chunk = opts->chunk_nnz;
        if (opts->device_byte_cap < 0) return fail(AMPED_ERR_INVALID, "device_byte_cap < 0");
        cap = opts->device_byte_cap;
        if (opts->keep_perm != 0 && opts->keep_perm != 1) return fail(AMPED_ERR_INVALID, "keep_perm must be 0 or 1");
        keep_perm = opts->keep_perm == 1;
    }
    // peak device bytes: the N layouts, the kept permutations, and during the
    // build the raw COO plus one permutation; per mode at most one int per row
    // for the zero-row list and long gaps, and the hot-row tables
    const int64_t layout_bytes = (int64_t)order * (order + 1) * 4 * (nnz + 4);
    int64_t row_bytes = 0;
    for (int d = 0; d < order; ++d) row_bytes += 4 * dims[d] + 4 * amped::kHotTableLen;
    // device sort: lexicographic order, key and value ping-pong buffers, scratch
    const int64_t sort_bytes = 16 * nnz + 4 * amped::sort_scratch_words(nnz);
    // host-resident layouts: two shard buffers of whole chunks instead
    const int64_t n_chunks = (nnz + chunk - 1) / chunk;
    const int64_t shard_chunks =
        std::max<int64_t>(1, std::min(((shard_opt > 0 ? shard_opt : (int64_t)1 << 25) + chunk - 1) / chunk,
                                      std::max<int64_t>(n_chunks, 1)));
    const int64_t stage_len = shard_chunks * chunk;
    if (host_layout && stage_len > 0x7FFFFFFF - 4)
        return fail(AMPED_ERR_INVALID, "shard of %lld nonzeros too large", (long long)stage_len);
    const int64_t peak =
        host_layout ? 2 * (int64_t)(order + 1) * 4 * (stage_len + 4) + row_bytes + 4096
                    : layout_bytes + (keep_perm ? (int64_t)order * 4 * nnz : 0) + (int64_t)(order + 1) * 4 * nnz +
                          4 * nnz + (int64_t)order * ((nnz + chunk - 1) / chunk + 64) * 8 + row_bytes + sort_bytes + 4096;
    if (cap > 0 && peak > cap)
        return fail(AMPED_ERR_NOMEM, "layouts need up to %lld device bytes, cap is %lld", (long long)peak,
                    (long long)cap);
    int dev = 0;
    st = check_device(&dev);
    if (st != AMPED_OK) return st;

    amped_tensor_s* t = new (std::nothrow) amped_tensor_s();
    if (!t) return fail(AMPED_ERR_NOMEM, "host allocation failed");
    t->order = order;
    for (int w = 0; w < order; ++w) t->dims[w] = dims[w];
    t->nnz = nnz;
    t->chunk = chunk;
    t->n_chunks = (nnz + chunk - 1) / chunk;
    t->device = dev;
    t->keep_perm = keep_perm;
    if (host_layout) {
        t->host_layout = true;
        t->stage_len = stage_len;
        st = build_host_layout(t, indices, values);
        if (st != AMPED_OK) {
            (void)hipDeviceSynchronize();
            t->free_all();
            delete t;
            return st;
        }
        *out = t;
        return AMPED_OK;
    }

    hipStream_t stream = nullptr;
    void* d_cols[kMaxOrder] = {};
    void* d_vals = nullptr;
    void* d_tmp_perm = nullptr;
    void* d_queues = nullptr;
    void* d_aux = nullptr;
    // device sort buffers (freed at the end of the build)
    void* d_lex = nullptr;
    void* d_key_a = nullptr;
    void* d_key_b = nullptr;
    void* d_val_b = nullptr;
    void* d_scratch = nullptr;
    try {
        // The order of each mode is built on the device: the lexicographic
        // order (when the input is not already in it) by stable radix sorts
        // over the modes, last mode first; then per mode a stable radix sort
        // of that order by i_d, whose sorted keys are the out_idx column.  The
        // chunk flags and row lists come from those keys on the host.
        const bool lexi = amped::is_lexicographic(order, nnz, indices);
        std::vector<int32_t> keys_h((size_t)nnz);
        HIP_OR_FAIL(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking), "hipStreamCreate");
        for (int w = 0; w < order; ++w) {
            HIP_OR_FAIL(t->alloc(&d_cols[w], (size_t)nnz * 4), "hipMalloc(coo)");
            if (nnz)
                HIP_OR_FAIL(hipMemcpy(d_cols[w], indices + (int64_t)w * nnz, (size_t)nnz * 4, hipMemcpyHostToDevice),
                            "hipMemcpy(coo)");
        }
        HIP_OR_FAIL(t->alloc(&d_vals, (size_t)nnz * 4), "hipMalloc(values)");
        if (nnz) HIP_OR_FAIL(hipMemcpy(d_vals, values, (size_t)nnz * 4, hipMemcpyHostToDevice), "hipMemcpy(values)");
        if (!keep_perm) HIP_OR_FAIL(t->alloc(&d_tmp_perm, (size_t)nnz * 4), "hipMalloc(perm)");
        HIP_OR_FAIL(t->alloc(&d_queues, (size_t)(order + 1) * amped::kQueueSlots * sizeof(unsigned)),
                    "hipMalloc(queues)");
        HIP_OR_FAIL(hipMemset(d_queues, 0, (size_t)(order + 1) * amped::kQueueSlots * sizeof(unsigned)),
                    "hipMemset(queues)");
        // 16 zero bytes followed by the store sink
        HIP_OR_FAIL(t->alloc(&d_aux, (size_t)(4 + kSinkFloats) * sizeof(float)), "hipMalloc(aux)");
        HIP_OR_FAIL(hipMemset(d_aux, 0, (size_t)(4 + kSinkFloats) * sizeof(float)), "hipMemset(aux)");
        HIP_OR_FAIL(t->alloc(&d_key_b, (size_t)nnz * 4), "hipMalloc(sort)");
        HIP_OR_FAIL(t->alloc(&d_val_b, (size_t)nnz * 4), "hipMalloc(sort)");
        HIP_OR_FAIL(t->alloc(&d_scratch, (size_t)amped::sort_scratch_words(nnz) * 4), "hipMalloc(sort)");
        auto sort_pairs = [&](void* keys, void* vals, int64_t dim) -> hipError_t {
            bool alt = false;
            hipError_t e = amped::launch_stable_sort_pairs(
                static_cast<uint32_t*>(keys), static_cast<int32_t*>(vals), static_cast<uint32_t*>(d_key_b),
                static_cast<int32_t*>(d_val_b), static_cast<uint32_t*>(d_scratch), nnz, bits_for(dim - 1), &alt,
                stream);
            if (e != hipSuccess || !alt) return e;
            e = hipMemcpyAsync(keys, d_key_b, (size_t)nnz * 4, hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return e;
            return hipMemcpyAsync(vals, d_val_b, (size_t)nnz * 4, hipMemcpyDeviceToDevice, stream);
        };
        if (!lexi) {
            HIP_OR_FAIL(t->alloc(&d_lex, (size_t)nnz * 4), "hipMalloc(sort)");
            HIP_OR_FAIL(t->alloc(&d_key_a, (size_t)nnz * 4), "hipMalloc(sort)");
            HIP_OR_FAIL(amped::launch_iota(static_cast<int32_t*>(d_lex), nnz, stream), "iota");
            for (int w = order - 1; w >= 0; --w) {
                HIP_OR_FAIL(amped::launch_permute32(d_key_a, d_cols[w], static_cast<int32_t*>(d_lex), nnz, stream),
                            "permute");
                HIP_OR_FAIL(sort_pairs(d_key_a, d_lex, dims[w]), "radix sort");
            }
        }

        for (int d = 0; d < order; ++d) {
            HostModeLayout lay;
            void* d_perm = d_tmp_perm;
            if (keep_perm) {
                HIP_OR_FAIL(t->alloc(&d_perm, (size_t)nnz * 4), "hipMalloc(perm)");
                t->perm[d] = static_cast<int32_t*>(d_perm);
            }
            if (lexi) HIP_OR_FAIL(amped::launch_iota(static_cast<int32_t*>(d_perm), nnz, stream), "iota");
            else if (nnz)
                HIP_OR_FAIL(hipMemcpyAsync(d_perm, d_lex, (size_t)nnz * 4, hipMemcpyDeviceToDevice, stream), "copy");
            ModeDev& m = t->mode[d];
            void* p = nullptr;
            // layout arrays carry 4 padding entries so 16-byte loads of the
            // last nonzeros stay inside the allocation
            const size_t padded = ((size_t)nnz + 4) * 4;
            HIP_OR_FAIL(t->alloc(&p, nnz ? padded : 0), "hipMalloc(out_idx)");
            HIP_OR_FAIL(amped::launch_permute32(p, d_cols[d], static_cast<int32_t*>(d_perm), nnz, stream), "permute");
            // the lexicographic order already is mode 0's order
            if (d > 0) HIP_OR_FAIL(sort_pairs(p, d_perm, dims[d]), "radix sort");
            m.out_idx = static_cast<int32_t*>(p);
            if (nnz)
                HIP_OR_FAIL(hipMemcpyAsync(keys_h.data(), p, (size_t)nnz * 4, hipMemcpyDeviceToHost, stream),
                            "hipMemcpy(keys)");
            int j = 0;
            for (int w = 0; w < order; ++w) {
                if (w == d) continue;
                HIP_OR_FAIL(t->alloc(&p, nnz ? padded : 0), "hipMalloc(in_idx)");
                HIP_OR_FAIL(amped::launch_permute32(p, d_cols[w], static_cast<int32_t*>(d_perm), nnz, stream),
                            "permute");
                m.in_idx[j++] = static_cast<int32_t*>(p);
            }
            HIP_OR_FAIL(t->alloc(&p, nnz ? padded : 0), "hipMalloc(values)");
            HIP_OR_FAIL(amped::launch_permute32(p, d_vals, static_cast<int32_t*>(d_perm), nnz, stream), "permute");
            m.val = static_cast<float*>(p);
            HIP_OR_FAIL(hipStreamSynchronize(stream), "layout build");
            amped::mode_tables_sorted(keys_h.data(), nnz, dims[d], chunk, lay);
            st = upload_tables(t, m, d, lay, d_queues, d_aux);
            if (st != AMPED_OK) goto cleanup;
        }
        t->loss_dev = t->mode[0];
        t->loss_dev.queue = static_cast<unsigned*>(d_queues) + (size_t)order * amped::kQueueSlots;
    } catch (const std::bad_alloc&) {
        st = fail(AMPED_ERR_NOMEM, "host allocation failed");
        goto cleanup;
    }
    for (int w = 0; w < order; ++w) {
        t->device_bytes -= (int64_t)nnz * 4;
        t->release(d_cols[w]);
    }
    t->device_bytes -= (int64_t)nnz * 4;
    t->release(d_vals);
    for (void* q : {d_tmp_perm, d_lex, d_key_a, d_key_b, d_val_b}) {
        if (!q) continue;
        t->device_bytes -= (int64_t)nnz * 4;
        t->release(q);
    }
    if (d_scratch) {
        t->device_bytes -= amped::sort_scratch_words(nnz) * 4;
        t->release(d_scratch);
    }
    (void)hipStreamDestroy(stream);
    *out = t;
    return AMPED_OK;

cleanup:
    if (stream) {
        (void)hipStreamSynchronize(stream);
        (void)hipStreamDestroy(stream);
    }
    t->free_all();
    delete t;
    return st;
}

amped_status amped_tensor_destroy(amped_tensor_t t)
{
    g_err.clear();
    if (!t) return AMPED_OK;
    amped_status st = AMPED_OK;
    {
        DeviceGuard guard(t->device);
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) st = hip_fail(e, "hipDeviceSynchronize");
        t->free_all();
    }
    delete t;
    return st;
}

amped_status amped_tensor_info(amped_tensor_t t, int* order, int64_t* dims, int64_t* nnz, int64_t* chunk_nnz,
                               int64_t* n_chunks, int64_t* touched, int64_t* device_bytes)
{
    g_err.clear();
    if (!t) return fail(AMPED_ERR_INVALID, "tensor is NULL");
    if (order) *order = t->order;
    if (dims)
        for (int w = 0; w < t->order; ++w) dims[w] = t->dims[w];
    if (nnz) *nnz = t->nnz;
    if (chunk_nnz) *chunk_nnz = t->chunk;
    if (n_chunks) *n_chunks = t->n_chunks;
    if (touched)
        for (int w = 0; w < t->order; ++w) touched[w] = t->touched[w];
    if (device_bytes) *device_bytes = t->device_bytes;
    return AMPED_OK;
}

amped_status amped_tensor_layout(amped_tensor_t t, int mode, int32_t* perm, int32_t* out_idx, int32_t* in_idx,
                                 float* values, uint8_t* chunk_flags)
{
    g_err.clear();
    if (!t) return fail(AMPED_ERR_INVALID, "tensor is NULL");
    if (mode < 0 || mode >= t->order) return fail(AMPED_ERR_INVALID, "mode %d outside [0, %d)", mode, t->order);
    if (perm && !t->keep_perm) return fail(AMPED_ERR_INVALID, "permutation not kept (create with keep_perm=1)");
    DeviceGuard guard(t->device);
    if (!guard.ok) return fail(AMPED_ERR_HIP, "cannot select device %d", t->device);
    const ModeDev& m = t->mode[mode];
    const size_t bytes = (size_t)t->nnz * 4;
    amped_status st = AMPED_OK;
    if (t->host_layout) {
        const auto& h = t->hmode[mode];
        if (bytes) {
            if (perm) std::memcpy(perm, t->hperm[mode].data(), bytes);
            if (out_idx) std::memcpy(out_idx, h.out_idx, bytes);
            if (in_idx)
                for (int j = 0; j < t->order - 1; ++j) std::memcpy(in_idx + (int64_t)j * t->nnz, h.in_idx[j], bytes);
            if (values) std::memcpy(values, h.val, bytes);
        }
    } else if (bytes) {
        if (perm) HIP_OR_FAIL(hipMemcpy(perm, t->perm[mode], bytes, hipMemcpyDeviceToHost), "hipMemcpy(perm)");
        if (out_idx) HIP_OR_FAIL(hipMemcpy(out_idx, m.out_idx, bytes, hipMemcpyDeviceToHost), "hipMemcpy(out_idx)");
        if (in_idx)
            for (int j = 0; j < t->order - 1; ++j)
                HIP_OR_FAIL(hipMemcpy(in_idx + (int64_t)j * t->nnz, m.in_idx[j], bytes, hipMemcpyDeviceToHost),
                            "hipMemcpy(in_idx)");
        if (values) HIP_OR_FAIL(hipMemcpy(values, m.val, bytes, hipMemcpyDeviceToHost), "hipMemcpy(values)");
    }
    if (chunk_flags && !t->flags[mode].empty()) std::memcpy(chunk_flags, t->flags[mode].data(), t->flags[mode].size());
    return AMPED_OK;
cleanup:
    return st;
}

namespace {

amped_status check_call(amped_tensor_t t, int mode, int rank, const void* const* factors, const void* out,
                        bool need_own, const char* out_name)
{
    if (!t) return fail(AMPED_ERR_INVALID, "tensor is NULL");
    if (mode < 0 || mode >= t->order) return fail(AMPED_ERR_INVALID, "mode %d outside [0, %d)", mode, t->order);
    if (rank < 1 || rank > 4096) return fail(AMPED_ERR_INVALID, "rank %d outside [1, 4096]", rank);
    if (!factors) return fail(AMPED_ERR_INVALID, "factors is NULL");
    for (int w = 0; w < t->order; ++w) {
        if (w == mode && !need_own) continue;
        if (!factors[w]) return fail(AMPED_ERR_INVALID, "factors[%d] is NULL", w);
        if (!aligned16(factors[w])) return fail(AMPED_ERR_INVALID, "factors[%d] is not 16-byte aligned", w);
    }
    if (!out) return fail(AMPED_ERR_INVALID, "%s is NULL", out_name);
    if (!aligned16(out)) return fail(AMPED_ERR_INVALID, "%s is not 16-byte aligned", out_name);
    return AMPED_OK;
}

amped_status run_mttkrp(amped_tensor_t t, int mode, int rank, const void* const* factors, float* out, void* stream,
                        amped::FactorType ft, amped::Kind kind, float scale, double* loss = nullptr)
{
    const bool grad = (kind != amped::Kind::Mttkrp);
    amped_status st = check_call(t, mode, rank, factors, out, grad, grad ? "grad" : "out");
    if (st != AMPED_OK) return st;
    if (kind == amped::Kind::ResidualGradLoss && !loss) return fail(AMPED_ERR_INVALID, "loss is NULL");
    DeviceGuard guard(t->device);
    if (!guard.ok) return fail(AMPED_ERR_HIP, "cannot select device %d", t->device);
    amped::LaunchArgs a;
    a.m = &t->mode[mode];
    a.nin = t->order - 1;
    a.rank = rank;
    a.ftype = ft;
    a.kind = kind;
    int j = 0;
    for (int w = 0; w < t->order; ++w)
        if (w != mode) {
            a.in_rows[j] = t->dims[w];
            a.in_hot[j] = t->mode[w].hot;
            a.in_factors[j++] = factors[w];
        }
    a.own_factor = grad ? static_cast<const float*>(factors[mode]) : nullptr;
    a.scale = scale;
    a.out = out;
    a.loss = loss;
    a.stream = static_cast<hipStream_t>(stream);
    const char* what = kind == amped::Kind::Mttkrp ? "amped_mttkrp"
                       : kind == amped::Kind::ResidualGrad ? "amped_cp_grad" : "amped_cp_loss_grad";
    auto launch = [&](const ModeDev& m, int i) -> amped_status {
        a.m = &m;
        a.loss_accumulate = i > 0;   // later shards add to the loss of the first
        hipError_t e = amped::launch_mttkrp(a);
        return e == hipSuccess ? AMPED_OK : hip_fail(e, what);
    };
    if (t->host_layout) return stream_shards(t, mode, t->mode[mode], a.stream, ChunkCut{t->nnz, t->stage_len}, launch);
    return launch(t->mode[mode], 0);
}

}  // namespace

amped_status amped_mttkrp(amped_tensor_t t, int mode, int rank, const float* const* factors, float* out,
                          void* stream)
{
    g_err.clear();
    return run_mttkrp(t, mode, rank, reinterpret_cast<const void* const*>(factors), out, stream,
                      amped::FactorType::F32, amped::Kind::Mttkrp, 1.0f);
}

amped_status amped_mttkrp_bf16(amped_tensor_t t, int mode, int rank, const uint16_t* const* factors, float* out,
                               void* stream)
{
    g_err.clear();
    return run_mttkrp(t, mode, rank, reinterpret_cast<const void* const*>(factors), out, stream,
                      amped::FactorType::BF16, amped::Kind::Mttkrp, 1.0f);
}

amped_status amped_cp_grad(amped_tensor_t t, int mode, int rank, const float* const* factors, float scale,
                           float* grad, void* stream)
{
    g_err.clear();
    return run_mttkrp(t, mode, rank, reinterpret_cast<const void* const*>(factors), grad, stream,
                      amped::FactorType::F32, amped::Kind::ResidualGrad, scale);
}

amped_status amped_cp_loss_grad(amped_tensor_t t, int mode, int rank, const float* const* factors, float scale,
                                float* grad, double* loss, void* stream)
{
    g_err.clear();
    return run_mttkrp(t, mode, rank, reinterpret_cast<const void* const*>(factors), grad, stream,
                      amped::FactorType::F32, amped::Kind::ResidualGradLoss, scale, loss);
}

amped_status amped_gram(const float* A, int64_t rows, int rank, double* G, void* stream)
{
    g_err.clear();
    if (!A || !G) return fail(AMPED_ERR_INVALID, "A or G is NULL");
    if (rows < 1) return fail(AMPED_ERR_INVALID, "rows %lld < 1", (long long)rows);
    if (rank < 1 || rank > 128) return fail(AMPED_ERR_INVALID, "rank %d outside [1, 128]", rank);
    int dev = 0;
    amped_status st = check_device(&dev);
    if (st != AMPED_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = (size_t)amped::gram_slabs(rows) * rank * rank * sizeof(float);
    void* partial = nullptr;
    hipError_t e = hipMallocAsync(&partial, bytes, s);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(gram partials)");
    e = amped::launch_gram(A, rows, rank, static_cast<float*>(partial), G, s);
    hipError_t e2 = hipFreeAsync(partial, s);
    if (e != hipSuccess) return hip_fail(e, "amped_gram");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync(gram partials)");
    return AMPED_OK;
}

amped_status amped_gram_noalloc(const float* A, int64_t rows, int rank, double* G, void* stream)
{
    g_err.clear();
    if (!A || !G) return fail(AMPED_ERR_INVALID, "A or G is NULL");
    if (rows < 1) return fail(AMPED_ERR_INVALID, "rows %lld < 1", (long long)rows);
    if (rank < 1 || rank > 128)
        return fail(AMPED_ERR_INVALID, "rank %d outside [1, 128]: the partial sums of larger ranks do not fit the "
                    "fixed 32 MiB device scratch", rank);
    int dev = 0;
    amped_status st = check_device(&dev);
    if (st != AMPED_OK) return st;
    hipError_t e = amped::launch_gram_noalloc(A, rows, rank, G, static_cast<hipStream_t>(stream));
    if (e == hipErrorInvalidValue)
        return fail(AMPED_ERR_INVALID, "amped_gram_noalloc: %lld rows x rank %d exceed the fixed device scratch",
                    (long long)rows, rank);
    return e == hipSuccess ? AMPED_OK : hip_fail(e, "amped_gram_noalloc");
}

amped_status amped_cp_als_sweep(amped_tensor_t t, int rank, float* const* factors, double* lambda, double* fit,
                                unsigned flags, void* stream)
{
    g_err.clear();
    amped_status st = check_call(t, 0, rank, reinterpret_cast<const void* const*>(factors), lambda, true, "lambda");
    if (st != AMPED_OK) return st;
    if (rank > 128) return fail(AMPED_ERR_INVALID, "rank %d above 128 (CP-ALS)", rank);
    if (!fit) return fail(AMPED_ERR_INVALID, "fit is NULL");
    if (flags & ~AMPED_ALS_REUSE_GRAMS) return fail(AMPED_ERR_INVALID, "unknown flags 0x%x", flags);
    const bool reuse = (flags & AMPED_ALS_REUSE_GRAMS) != 0;
    if (reuse && (t->als.rank != rank || !t->als.have_grams))
        return fail(AMPED_ERR_INVALID, "no previous sweep at rank %d to reuse Gram matrices from", rank);
    DeviceGuard guard(t->device);
    if (!guard.ok) return fail(AMPED_ERR_HIP, "cannot select device %d", t->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto& w = t->als;
    const int N = t->order;
    hipError_t e = hipSuccess;
    const size_t RR = (size_t)rank * rank;
    if (w.rank != rank) {
        for (void* q : {(void*)w.M, (void*)w.G, (void*)w.S, (void*)w.partial, (void*)w.scratch, (void*)w.W,
                        (void*)w.wide})
            if (q) t->release(q);
        double* keep_x = w.xnorm2;
        const bool keep_have = w.have_xnorm2;
        w = amped_tensor_s::AlsWork{};
        w.xnorm2 = keep_x;
        w.have_xnorm2 = keep_have;
        int64_t maxrows = 0;
        for (int d = 0; d < N; ++d) maxrows = std::max(maxrows, t->dims[d]);
        void* p = nullptr;
        if ((e = t->alloc(&p, (size_t)maxrows * rank * sizeof(float))) != hipSuccess) return hip_fail(e, "als workspace");
        w.M = static_cast<float*>(p);
        if ((e = t->alloc(&p, N * RR * sizeof(double))) != hipSuccess) return hip_fail(e, "als workspace");
        w.G = static_cast<double*>(p);
        if ((e = t->alloc(&p, RR * sizeof(double))) != hipSuccess) return hip_fail(e, "als workspace");
        w.S = static_cast<double*>(p);
        if ((e = t->alloc(&p, (size_t)amped::gram_slabs(maxrows) * RR * sizeof(float))) != hipSuccess)
            return hip_fail(e, "als workspace");
        w.partial = static_cast<float*>(p);
        if ((e = t->alloc(&p, 4 * RR * sizeof(double))) != hipSuccess) return hip_fail(e, "als workspace");
        w.scratch = static_cast<double*>(p);
        if ((e = t->alloc(&p, RR * sizeof(double))) != hipSuccess) return hip_fail(e, "als workspace");
        w.W = static_cast<double*>(p);
        if ((e = t->alloc(&p, sizeof(int))) != hipSuccess) return hip_fail(e, "als workspace");
        w.wide = static_cast<int*>(p);
        if (!w.xnorm2) {
            if ((e = t->alloc(&p, sizeof(double))) != hipSuccess) return hip_fail(e, "als workspace");
            w.xnorm2 = static_cast<double*>(p);
        }
        w.rank = rank;
    }
    if (!w.have_xnorm2) {
        auto norm = [&](const ModeDev& m, int i) -> amped_status {
            hipError_t en = amped::launch_tensor_norm2(m, N - 1, w.xnorm2, i > 0, s);
            return en == hipSuccess ? AMPED_OK : hip_fail(en, "tensor norm");
        };
        if (t->host_layout) {
            // shards end between runs of equal coordinates (each run is summed
            // before squaring)
            const auto& h = t->hmode[0];
            auto same = [&](int64_t p, int64_t q) {
                if (h.out_idx[p] != h.out_idx[q]) return false;
                for (int j = 0; j < N - 1; ++j)
                    if (h.in_idx[j][p] != h.in_idx[j][q]) return false;
                return true;
            };
            auto cut = [&](int64_t start) {
                int64_t end = std::min(start + t->stage_len, t->nnz);
                if (end < t->nnz)
                    while (end > start && same(end - 1, end)) --end;
                return end;
            };
            st = stream_shards(t, 0, t->mode[0], s, cut, norm);
        } else {
            st = norm(t->mode[0], 0);
        }
        if (st != AMPED_OK) return st;
        w.have_xnorm2 = true;
    }
    w.have_grams = false;   // stays false if the sweep stops part-way
    if (!reuse) {
        for (int m = 0; m < N; ++m)
            if ((e = amped::launch_gram(factors[m], t->dims[m], rank, w.partial, w.G + m * RR, s)) != hipSuccess)
                return hip_fail(e, "gram");
    }
    for (int d = 0; d < N; ++d) {
        st = run_mttkrp(t, d, rank, reinterpret_cast<const void* const*>(factors), w.M, stream,
                        amped::FactorType::F32, amped::Kind::Mttkrp, 1.0f);
        if (st != AMPED_OK) return st;
        if ((e = amped::launch_gram(w.M, t->dims[d], rank, w.partial, w.S, s)) != hipSuccess)
            return hip_fail(e, "gram");
        if ((e = amped::launch_als_small(w.G, w.S, N, d, rank, w.scratch, w.W, w.wide, lambda, d == N - 1,
                                         w.xnorm2, fit, s)) != hipSuccess)
            return hip_fail(e, "als update");
        if ((e = amped::launch_als_solve(w.M, w.W, w.wide, factors[d], t->dims[d], rank, s)) != hipSuccess)
            return hip_fail(e, "als solve");
    }
    w.have_grams = true;   // G now holds the Gram matrices of the factors just written
    return AMPED_OK;
}

#if AMPED_QUEUE_STATS
amped_status amped_queue_stats(uint64_t* records, int64_t max_records, int64_t* n_records, int32_t* waves_per_block,
                               double* clock_hz)
{
    g_err.clear();
    if (!n_records || !waves_per_block || !clock_hz) return fail(AMPED_ERR_INVALID, "NULL output");
    if (records && max_records < 0) return fail(AMPED_ERR_INVALID, "max_records < 0");
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return hip_fail(e, "wall clock rate");
    *clock_hz = 1e3 * khz;
    int wpb = 0;
    e = amped::queue_stats_copy(reinterpret_cast<unsigned long long*>(records), max_records, n_records, &wpb);
    *waves_per_block = wpb;
    return e == hipSuccess ? AMPED_OK : hip_fail(e, "amped_queue_stats");
}
#endif

amped_status amped_cp_loss(amped_tensor_t t, int rank, const float* const* factors, double* loss, void* stream)
{
    g_err.clear();
    amped_status st = check_call(t, 0, rank, reinterpret_cast<const void* const*>(factors), loss, true, "loss");
    if (st != AMPED_OK) return st;
    DeviceGuard guard(t->device);
    if (!guard.ok) return fail(AMPED_ERR_HIP, "cannot select device %d", t->device);
    amped::LossArgs a;
    a.m = &t->loss_dev;
    a.order = t->order;
    a.rank = rank;
    a.own_factor = factors[0];
    for (int w = 1; w < t->order; ++w) {
        a.in_factors[w - 1] = factors[w];
        a.in_rows[w - 1] = t->dims[w];
        a.in_hot[w - 1] = t->mode[w].hot;
    }
    a.loss = loss;
    a.stream = static_cast<hipStream_t>(stream);
    auto launch = [&](const ModeDev& m, int i) -> amped_status {
        a.m = &m;
        a.accumulate = i > 0;
        hipError_t e = amped::launch_cp_loss(a);
        return e == hipSuccess ? AMPED_OK : hip_fail(e, "amped_cp_loss");
    };
    if (t->host_layout) return stream_shards(t, 0, t->loss_dev, a.stream, ChunkCut{t->nnz, t->stage_len}, launch);
    return launch(t->loss_dev, 0);
}

}  // extern "C"
