// Host layout builder (paper_2507_15121_amd/csrc/layout.cpp) against brute
// force, meant to be built with AddressSanitizer and UBSan
// (tests/test_host_sanitized.py).  For random COO tensors (orders 2-5, tiny
// and skewed shapes, exact duplicates, lexicographic or shuffled input) it
// checks, per mode:
//   - the order: a stable sort by (i_d, other indices in ascending mode order);
//   - the chunk flags, the distinct-row count, the zero-row list and the long
//     gaps (every untouched or chunk-shared row zeroed exactly once);
//   - the hot-row tables (slot s of K: the most-used row r with r % K == s,
//     ties to the smaller row);
//   - that the tables from the sorted key column equal those from the indices;
//   - the gather helper.
// Exit status 0 when every check passes.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <numeric>
#include <random>
#include <vector>

#include "internal.h"

using namespace amped;

static int fails = 0;
#define CHECK(cond, ...)                                          \
    do {                                                          \
        if (!(cond)) {                                            \
            if (fails++ < 20) {                                   \
                std::printf("FAIL line %d: ", __LINE__);          \
                std::printf(__VA_ARGS__);                         \
                std::printf("\n");                                \
            }                                                     \
        }                                                         \
    } while (0)

struct Case {
    std::vector<int64_t> dims;
    int64_t nnz;
    int64_t chunk;
    int dups;        // exact duplicates appended
    double skew;     // share of nonzeros forced into row 0 of mode 0
    bool shuffle;    // false: input sorted lexicographically
};

static void run_case(const Case& c, uint64_t seed)
{
    const int order = (int)c.dims.size();
    std::mt19937_64 rng(seed);
    const int64_t base = c.nnz;
    const int64_t nnz = base + (base ? c.dups : 0);
    std::vector<int32_t> idx((size_t)order * nnz);
    auto at = [&](int w, int64_t k) -> int32_t& { return idx[(size_t)w * nnz + k]; };
    std::uniform_real_distribution<double> U(0.0, 1.0);
    for (int64_t k = 0; k < base; ++k)
        for (int w = 0; w < order; ++w) {
            int64_t v = (int64_t)(std::pow(U(rng), 3.0) * (double)c.dims[w]);   // power-law-ish
            if (w == 0 && U(rng) < c.skew) v = 0;
            at(w, k) = (int32_t)std::min<int64_t>(v, c.dims[w] - 1);
        }
    for (int64_t k = base; k < nnz; ++k) {
        const int64_t src = (int64_t)(U(rng) * (double)base);
        for (int w = 0; w < order; ++w) at(w, k) = at(w, std::min(src, base - 1));
    }
    std::vector<int64_t> pos(nnz);
    std::iota(pos.begin(), pos.end(), 0);
    auto lex_less = [&](int64_t a, int64_t b) {
        for (int w = 0; w < order; ++w)
            if (at(w, a) != at(w, b)) return at(w, a) < at(w, b);
        return false;
    };
    if (!c.shuffle) {
        std::stable_sort(pos.begin(), pos.end(), lex_less);
        std::vector<int32_t> sorted(idx.size());
        for (int w = 0; w < order; ++w)
            for (int64_t k = 0; k < nnz; ++k) sorted[(size_t)w * nnz + k] = at(w, pos[k]);
        idx.swap(sorted);
    }

    const std::vector<int32_t> lex = lex_order(order, c.dims.data(), nnz, idx.data());
    {
        std::vector<int64_t> ref(nnz);
        std::iota(ref.begin(), ref.end(), 0);
        std::stable_sort(ref.begin(), ref.end(), lex_less);
        if (lex.empty()) {
            for (int64_t k = 0; k < nnz; ++k) CHECK(ref[k] == k, "lex_order empty but input unsorted at %lld", (long long)k);
        } else {
            CHECK((int64_t)lex.size() == nnz, "lex size");
            for (int64_t k = 0; k < nnz && k < (int64_t)lex.size(); ++k)
                CHECK(lex[k] == ref[k], "lex_order at %lld", (long long)k);
        }
    }

    for (int d = 0; d < order; ++d) {
        HostModeLayout lay;
        mode_order(c.dims.data(), nnz, idx.data(), lex, d, lay.perm);
        std::vector<int64_t> ref(nnz);
        std::iota(ref.begin(), ref.end(), 0);
        std::stable_sort(ref.begin(), ref.end(), [&](int64_t a, int64_t b) {
            if (at(d, a) != at(d, b)) return at(d, a) < at(d, b);
            for (int w = 0; w < order; ++w)
                if (w != d && at(w, a) != at(w, b)) return at(w, a) < at(w, b);
            return false;
        });
        CHECK((int64_t)lay.perm.size() == nnz, "perm size mode %d", d);
        for (int64_t k = 0; k < nnz && k < (int64_t)lay.perm.size(); ++k)
            CHECK(lay.perm[k] == ref[k], "mode %d order at %lld", d, (long long)k);

        mode_tables(c.dims.data(), nnz, idx.data(), d, c.chunk, lay);
        std::vector<int32_t> keys(nnz);
        for (int64_t k = 0; k < nnz; ++k) keys[k] = at(d, ref[k]);
        const int64_t rows = c.dims[d], CH = c.chunk;
        const int64_t n_chunks = (nnz + CH - 1) / CH;
        CHECK((int64_t)lay.flags.size() == n_chunks, "flags size");
        std::vector<int64_t> cnt(rows, 0);
        for (int64_t k = 0; k < nnz; ++k) cnt[keys[k]]++;
        std::vector<uint8_t> shared(rows, 0);
        for (int64_t q = 0; q < n_chunks && q < (int64_t)lay.flags.size(); ++q) {
            const int64_t s = q * CH, e = std::min(s + CH, nnz);
            const uint8_t f = (uint8_t)((q > 0 && keys[s - 1] == keys[s] ? 1 : 0) | (e < nnz && keys[e - 1] == keys[e] ? 2 : 0));
            CHECK(lay.flags[q] == f, "mode %d chunk %lld flags %d want %d", d, (long long)q, lay.flags[q], f);
            if (f & 1) shared[keys[s]] = 1;
        }
        int64_t touched = 0;
        for (int64_t r = 0; r < rows; ++r) touched += cnt[r] > 0;
        CHECK(lay.touched == touched, "touched %lld want %lld", (long long)lay.touched, (long long)touched);
        // every row that the kernel does not store is zeroed exactly once
        std::vector<int> cover(rows, 0);
        for (int32_t r : lay.zero_rows) {
            CHECK(r >= 0 && r < rows, "zero row %d out of range", r);
            if (r >= 0 && r < rows) cover[r]++;
        }
        CHECK(lay.gaps.size() % 2 == 0, "gaps not in pairs");
        for (size_t g = 0; g + 1 < lay.gaps.size(); g += 2) {
            const int64_t s = lay.gaps[g], len = lay.gaps[g + 1];
            CHECK(len >= kLongGap && len <= kGapPiece + kLongGap, "gap (%lld, %lld) outside [%d, %d]", (long long)s,
                  (long long)len, kLongGap, kGapPiece + kLongGap);
            for (int64_t r = s; r < s + len; ++r) {
                CHECK(r >= 0 && r < rows, "gap row out of range");
                if (r >= 0 && r < rows) cover[r]++;
            }
        }
        for (int64_t r = 0; r < rows; ++r) {
            const int want = (cnt[r] == 0 || shared[r]) ? 1 : 0;
            CHECK(cover[r] == want, "mode %d row %lld zeroed %d times, want %d", d, (long long)r, cover[r], want);
        }
        // hot tables
        CHECK((int)lay.hot.size() == kHotTableLen, "hot size");
        for (int K = 1; K <= kHotMax; K *= 2)
            for (int s = 0; s < K; ++s) {
                int32_t best = kHotEmpty;
                for (int64_t r = s; r < rows; r += K)
                    if (cnt[r] > 0 && (best == kHotEmpty || cnt[r] > cnt[best])) best = (int32_t)r;
                CHECK(lay.hot[(size_t)(K - 1) + s] == best, "mode %d hot K=%d slot %d: %d want %d", d, K, s,
                      lay.hot[(size_t)(K - 1) + s], best);
            }
        HostModeLayout lay2;
        mode_tables_sorted(keys.data(), nnz, rows, CH, lay2);
        CHECK(lay2.flags == lay.flags && lay2.zero_rows == lay.zero_rows && lay2.gaps == lay.gaps &&
                  lay2.hot == lay.hot && lay2.touched == lay.touched,
              "mode %d: tables from sorted keys differ", d);
        std::vector<int32_t> g(nnz);
        gather_i32(idx.data() + (size_t)d * nnz, lay.perm.data(), 0, nnz, g.data());
        CHECK(g == keys, "gather mode %d", d);
    }
}

int main()
{
    const std::vector<Case> cases = {
        {{5, 4, 3}, 0, 4, 0, 0.0, true},
        {{5, 4, 3}, 1, 4, 0, 0.0, true},
        {{1, 1, 1}, 9, 2, 3, 0.0, true},
        {{7, 9}, 60, 7, 10, 0.0, false},
        {{40, 30, 20}, 3000, 64, 200, 0.3, true},
        {{40, 30, 20}, 3000, 1, 0, 0.0, false},
        {{2000, 1500, 700}, 20000, 256, 1000, 0.1, true},
        {{2000, 1500, 700}, 20000, 4096, 0, 0.5, false},
        {{60, 50, 40, 30}, 5000, 100, 50, 0.0, true},
        {{9, 8, 7, 6, 5}, 4000, 33, 400, 0.2, true},
        {{70000, 3000, 5}, 50000, 512, 0, 0.05, true},
    };
    uint64_t seed = 1;
    for (const Case& c : cases) run_case(c, seed++);
    std::printf("%zu cases, %d failures\n", cases.size(), fails);
    return fails ? 1 : 0;
}
