// Host side of the per-mode layout builder (preprocessing, Sec. 5.7; not part
// of the timed MTTKRP).  For every output mode d the nonzeros are ordered by
// the key (i_d, then the other indices in ascending mode order); exact
// duplicates keep their input order.  The order is computed with stable
// parallel LSD radix sorts:
//   1. if the input is not already lexicographic in (i_0, ..., i_{N-1}), a
//      lexicographic order is built (LSD over the modes, last mode first);
//   2. a stable sort of that order by i_d alone then yields the key above,
//      since among equal i_d the remaining indices stay in lexicographic order.
// The chunk table follows: chunk k holds positions [k*CH, min((k+1)*CH, nnz)),
// the fixed-size stand-in for the paper's equal-size inter-shard partitions
// (Sec. 3.1/3.2).
#include <omp.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace amped {
namespace {

int bits_for(uint64_t n)  // bits needed to hold the values 0..n
{
    int b = 0;
    while (b < 64 && (n >> b)) ++b;
    return b;
}

// Stable LSD radix sort of (key, val) pairs by key, keys < 2^bits.
void radix_sort_pairs(std::vector<uint32_t>& keys, std::vector<int32_t>& vals, int bits)
{
    const int64_t n = (int64_t)keys.size();
    if (n <= 1 || bits == 0) return;
    const int passes = (bits + 11) / 12;
    const int digit = (bits + passes - 1) / passes;
    const int nb = 1 << digit;
    std::vector<uint32_t> k2(n);
    std::vector<int32_t> v2(n);
    int nt = omp_get_max_threads();
    if (nt < 1) nt = 1;
    if (n < (1 << 16)) nt = 1;
    std::vector<int64_t> hist((size_t)nt * nb);
    uint32_t* ks = keys.data();
    int32_t* vs = vals.data();
    uint32_t* kd = k2.data();
    int32_t* vd = v2.data();
    for (int p = 0; p < passes; ++p) {
        const int sh = p * digit;
        const uint32_t mask = (uint32_t)nb - 1;
        std::fill(hist.begin(), hist.end(), 0);
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num();
            const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
            int64_t* h = hist.data() + (size_t)t * nb;
            for (int64_t i = lo; i < hi; ++i) h[(ks[i] >> sh) & mask]++;
#pragma omp barrier
#pragma omp single
            {
                int64_t run = 0;
                for (int b = 0; b < nb; ++b)
                    for (int tt = 0; tt < nt; ++tt) {
                        const int64_t c = hist[(size_t)tt * nb + b];
                        hist[(size_t)tt * nb + b] = run;
                        run += c;
                    }
            }
            for (int64_t i = lo; i < hi; ++i) {
                const int64_t o = h[(ks[i] >> sh) & mask]++;
                kd[o] = ks[i];
                vd[o] = vs[i];
            }
        }
        std::swap(ks, kd);
        std::swap(vs, vd);
    }
    if (ks != keys.data()) {
        keys.swap(k2);
        vals.swap(v2);
    }
}

// Stable sort of `order` (positions) by idx_w[position].
void stable_sort_by(const int32_t* idx_w, int64_t dim, std::vector<int32_t>& order)
{
    const int64_t n = (int64_t)order.size();
    std::vector<uint32_t> keys(n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) keys[i] = (uint32_t)idx_w[order[i]];
    radix_sort_pairs(keys, order, bits_for((uint64_t)(dim - 1)));
}

// Hot-row tables from a sorted key column: the use count of row r is the
// length of its run.  Runs are split among threads by where they start.
template <typename Key>
void hot_tables(int64_t nnz, const Key& key, std::vector<int32_t>& hot)
{
    int nt = omp_get_max_threads();
    if (nt < 1) nt = 1;
    std::vector<int32_t> brow((size_t)nt * kHotMax, kHotEmpty);
    std::vector<int64_t> bcnt((size_t)nt * kHotMax, 0);
#pragma omp parallel num_threads(nt)
    {
        const int t = omp_get_thread_num();
        int32_t* r = &brow[(size_t)t * kHotMax];
        int64_t* c = &bcnt[(size_t)t * kHotMax];
        int64_t p = nnz * t / nt;
        const int64_t hi = nnz * (t + 1) / nt;
        while (p > 0 && p < hi && key(p - 1) == key(p)) ++p;  // the run belongs to an earlier thread
        while (p < hi) {
            const int32_t row = key(p);
            int64_t e = p + 1;
            while (e < nnz && key(e) == row) ++e;
            const int s = row & (kHotMax - 1);
            if (e - p > c[s] || (e - p == c[s] && row < r[s])) {
                c[s] = e - p;
                r[s] = row;
            }
            p = e;
        }
    }
    // merge threads, then halve K: slot s of K takes the better of slots s
    // and s + K of 2K (ties to the smaller row)
    std::vector<int32_t> row(kHotMax, kHotEmpty);
    std::vector<int64_t> cnt(kHotMax, 0);
    for (int t = 0; t < nt; ++t)
        for (int s = 0; s < kHotMax; ++s) {
            const int32_t rr = brow[(size_t)t * kHotMax + s];
            const int64_t cc = bcnt[(size_t)t * kHotMax + s];
            if (cc > cnt[s] || (cc == cnt[s] && cc > 0 && rr < row[s])) {
                cnt[s] = cc;
                row[s] = rr;
            }
        }
    hot.assign(kHotTableLen, kHotEmpty);
    for (int K = kHotMax;; K >>= 1) {
        std::copy(row.begin(), row.begin() + K, hot.begin() + (K - 1));
        if (K == 1) break;
        const int h = K / 2;
        for (int s = 0; s < h; ++s)
            if (cnt[s + h] > cnt[s] || (cnt[s + h] == cnt[s] && cnt[s] > 0 && row[s + h] < row[s])) {
                cnt[s] = cnt[s + h];
                row[s] = row[s + h];
            }
    }
}

}  // namespace

std::vector<int32_t> lex_order(int order, const int64_t* dims, int64_t nnz, const int32_t* idx)
{
    if (is_lexicographic(order, nnz, idx)) return {};
    std::vector<int32_t> perm(nnz);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nnz; ++k) perm[k] = (int32_t)k;
    for (int w = order - 1; w >= 0; --w) stable_sort_by(idx + (int64_t)w * nnz, dims[w], perm);
    return perm;
}

void mode_order(const int64_t* dims, int64_t nnz, const int32_t* idx, const std::vector<int32_t>& base,
                int mode, std::vector<int32_t>& perm)
{
    perm.resize(nnz);
    if (base.empty()) {
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nnz; ++k) perm[k] = (int32_t)k;
    } else {
        std::memcpy(perm.data(), base.data(), (size_t)nnz * sizeof(int32_t));
    }
    if (mode == 0 && base.empty()) return;  // lexicographic input is already in mode-0 order
    stable_sort_by(idx + (int64_t)mode * nnz, dims[mode], perm);
}

namespace {

// A run of len >= kLongGap untouched rows from `start` as (start, length)
// ranges of at most about kGapPiece rows each (every one at least kLongGap).
void push_gap(std::vector<int32_t>& gaps, int64_t start, int64_t len)
{
    const int64_t n = (len + kGapPiece - 1) / kGapPiece;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t a = start + len * i / n, b = start + len * (i + 1) / n;
        gaps.push_back((int32_t)a);
        gaps.push_back((int32_t)(b - a));
    }
}

// Chunk flags, zero-row list, long gaps, hot-row tables and touched count from
// key(p), the output index at position p of the mode's order.
template <typename Key>
void tables_from_keys(int64_t nnz, int64_t rows, int64_t chunk, const Key& key, HostModeLayout& lay)
{
    const int64_t n_chunks = (nnz + chunk - 1) / chunk;
    lay.flags.assign(n_chunks, 0);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n_chunks; ++k) {
        const int64_t s = k * chunk, e = std::min(s + chunk, nnz);
        uint8_t f = 0;
        if (k > 0 && key(s - 1) == key(s)) f |= 1;
        if (e < nnz && key(e - 1) == key(e)) f |= 2;
        lay.flags[k] = f;
    }
    lay.zero_rows.clear();
    for (int64_t k = 1; k < n_chunks; ++k)
        if (lay.flags[k] & 1) {
            const int32_t r = key(k * chunk);
            if (lay.zero_rows.empty() || lay.zero_rows.back() != r) lay.zero_rows.push_back(r);
        }
    // distinct output indices; untouched rows as long runs or single rows
    int nt = omp_get_max_threads();
    if (nt < 1) nt = 1;
    std::vector<std::vector<int32_t>> tgaps(nt), tlone(nt);
    int64_t touched = 0;
#pragma omp parallel num_threads(nt) reduction(+ : touched)
    {
        const int t = omp_get_thread_num();
        const int64_t lo = nnz * t / nt, hi = nnz * (t + 1) / nt;
        for (int64_t p = lo; p < hi; ++p) {
            const int64_t cur = key(p);
            const int64_t prev = (p == 0) ? -1 : key(p - 1);
            if (cur != prev) {
                touched++;
                if (cur - prev - 1 >= kLongGap) {
                    push_gap(tgaps[t], prev + 1, cur - prev - 1);
                } else {
                    for (int64_t r = prev + 1; r < cur; ++r) tlone[t].push_back((int32_t)r);
                }
            }
        }
    }
    lay.touched = touched;
    hot_tables(nnz, key, lay.hot);
    lay.gaps.clear();
    for (int t = 0; t < nt; ++t) {
        lay.gaps.insert(lay.gaps.end(), tgaps[t].begin(), tgaps[t].end());
        lay.zero_rows.insert(lay.zero_rows.end(), tlone[t].begin(), tlone[t].end());
    }
    if (nnz == 0) {
        if (rows >= kLongGap) push_gap(lay.gaps, 0, rows);
        else for (int64_t r = 0; r < rows; ++r) lay.zero_rows.push_back((int32_t)r);
    } else {
        const int64_t last = key(nnz - 1);
        if (rows - last - 1 >= kLongGap) {
            push_gap(lay.gaps, last + 1, rows - last - 1);
        } else {
            for (int64_t r = last + 1; r < rows; ++r) lay.zero_rows.push_back((int32_t)r);
        }
    }
}

}  // namespace

void mode_tables(const int64_t* dims, int64_t nnz, const int32_t* idx, int mode, int64_t chunk,
                 HostModeLayout& lay)
{
    const int32_t* col = idx + (int64_t)mode * nnz;
    const int32_t* perm = lay.perm.data();
    tables_from_keys(nnz, dims[mode], chunk, [&](int64_t p) { return col[perm[p]]; }, lay);
}

void mode_tables_sorted(const int32_t* keys, int64_t nnz, int64_t rows, int64_t chunk, HostModeLayout& lay)
{
    tables_from_keys(nnz, rows, chunk, [&](int64_t p) { return keys[p]; }, lay);
}

bool is_lexicographic(int order, int64_t nnz, const int32_t* idx)
{
    int64_t unsorted = 0;
#pragma omp parallel for reduction(+ : unsorted) schedule(static)
    for (int64_t k = 1; k < nnz; ++k) {
        int cmp = 0;
        for (int w = 0; w < order && cmp == 0; ++w) {
            const int32_t a = idx[(int64_t)w * nnz + k - 1], b = idx[(int64_t)w * nnz + k];
            cmp = (a < b) ? -1 : (a > b) ? 1 : 0;
        }
        if (cmp > 0) unsorted++;
    }
    return unsorted == 0;
}

void gather_i32(const int32_t* src, const int32_t* perm, int64_t p0, int64_t p1, int32_t* dst)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = p0; p < p1; ++p) dst[p - p0] = src[perm[p]];
}

void gather_f32(const float* src, const int32_t* perm, int64_t p0, int64_t p1, float* dst)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = p0; p < p1; ++p) dst[p - p0] = src[perm[p]];
}

}  // namespace amped
