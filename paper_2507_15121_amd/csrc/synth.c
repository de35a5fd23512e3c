/*
 * Seeded synthetic sparse tensors shaped like the paper's billion-scale
 * workloads (Table 3: 3-5 modes, 10^5-10^8 indices per mode, power-law index
 * popularity).  Input generation only: this file holds none of the MTTKRP
 * arithmetic and is shared, as a generator, by the HIP path's tests/bench and
 * by the oracle's tests.
 *
 * Random numbers come from a counter-based generator: draw k of stream s is
 * the SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014) applied
 * to key(seed, s) + (k + 1) * 0x9E3779B97F4A7C15, so results do not depend on
 * the number of OpenMP threads.
 *
 * Recipe (all counts exact):
 *  - per mode w, a draw picks a popularity rank from a finite Zipf law
 *    P(rank k) = k^-s / H_{I_w,s}, k = 1..I_w (inverse CDF on a float64 table),
 *    or a uniform index; ranks are mapped to indices by a seeded bijection of
 *    [0, I_w) (a 4-round Feistel network with cycle walking) so hot rows are
 *    scattered over the index space;
 *  - raw coordinates are drawn in counter order; the tensor keeps the first
 *    nnz DISTINCT coordinates in draw order (duplicates merged);
 *  - optional hot slice: exactly round(hot_frac * nnz) coordinates have
 *    i_0 = h, h the index of the mode-0 rank floor(I_0/2)+1; their other
 *    indices are drawn as above and deduplicated; no other coordinate has
 *    i_0 = h;
 *  - the output is sorted lexicographically by (i_0, i_1, ...).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream)
{
    return mix64(mix64(seed + GAMMA) ^ (stream * 0xD1B54A32D192ED03ull));
}

static inline uint64_t draw_u64(uint64_t key, uint64_t k) { return mix64(key + (k + 1) * GAMMA); }

static inline double draw_unit(uint64_t key, uint64_t k)
{
    return (double)(draw_u64(key, k) >> 11) * 0x1.0p-53;
}

enum { ST_VALUES = 1, ST_COORD = 100, ST_HOT = 200, ST_FACTOR = 300, ST_PERM = 400 };

/* ------------------------------------------------------------------ uniforms */

void synth_uniform_f32(uint64_t seed, uint64_t stream, int64_t n, float lo, float hi, float *out)
{
    const uint64_t key = stream_key(seed, stream);
    const float span = hi - lo;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const float u = (float)(draw_u64(key, (uint64_t)i) >> 40) * 0x1.0p-24f;
        out[i] = lo + span * u;
    }
}

/* Values U(0,1) for nonzero j in final order, factors U(-1,1) per element. */
void synth_values(uint64_t seed, int64_t nnz, float *out) { synth_uniform_f32(seed, ST_VALUES, nnz, 0.0f, 1.0f, out); }

void synth_factor(uint64_t seed, int mode, int64_t rows, int64_t rank, float *out)
{
    synth_uniform_f32(seed, ST_FACTOR + (uint64_t)mode, rows * rank, -1.0f, 1.0f, out);
}

/* ------------------------------------------------------------ rank -> index */

static int bits_for(uint64_t n) /* bits needed to hold values 0..n */
{
    int b = 0;
    while (b < 64 && (n >> b)) ++b;
    return b;
}

static uint64_t feistel(uint64_t x, int h, const uint64_t *keys)
{
    const uint64_t mask = (h >= 64) ? ~0ull : ((1ull << h) - 1);
    uint64_t L = x >> h, Rr = x & mask;
    for (int r = 0; r < 4; ++r) {
        uint64_t nl = Rr;
        uint64_t nr = L ^ (mix64(Rr ^ keys[r]) & mask);
        L = nl;
        Rr = nr;
    }
    return (L << h) | Rr;
}

/* perm[r] = index of popularity rank r (0-based), a bijection of [0, I). */
static void build_perm(uint64_t seed, int mode, int64_t I, int32_t *perm)
{
    if (I == 1) {
        perm[0] = 0;
        return;
    }
    int b = bits_for((uint64_t)(I - 1));
    if (b < 2) b = 2;
    const int h = (b + 1) / 2;
    uint64_t keys[4];
    const uint64_t sk = stream_key(seed, ST_PERM + (uint64_t)mode);
    for (int r = 0; r < 4; ++r) keys[r] = draw_u64(sk, (uint64_t)r);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < I; ++r) {
        uint64_t y = feistel((uint64_t)r, h, keys);
        while (y >= (uint64_t)I) y = feistel(y, h, keys);
        perm[r] = (int32_t)y;
    }
}

/* --------------------------------------------------------------- Zipf table */

typedef struct {
    int64_t I;
    double total;
    double *cdf;     /* cdf[k] = sum_{j<=k} (j+1)^-s  (unnormalised)        */
    int64_t G;
    int64_t *guide;  /* guide[g] = first k with cdf[k] > g * total / G      */
} zipf_t;

#define ZBLK (1 << 20)

static void zipf_build(zipf_t *z, int64_t I, double s)
{
    z->I = I;
    z->cdf = (double *)malloc((size_t)I * sizeof(double));
    const int64_t nb = (I + ZBLK - 1) / ZBLK;
    double *bsum = (double *)calloc((size_t)nb + 1, sizeof(double));
    /* fixed blocks: the summation order does not depend on the thread count */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t lo = b * ZBLK, hi = (lo + ZBLK < I) ? lo + ZBLK : I;
        double acc = 0.0;
        for (int64_t k = lo; k < hi; ++k) {
            acc += pow((double)(k + 1), -s);
            z->cdf[k] = acc;
        }
        bsum[b + 1] = acc;
    }
    for (int64_t b = 0; b < nb; ++b) bsum[b + 1] += bsum[b];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 1; b < nb; ++b) {
        const int64_t lo = b * ZBLK, hi = (lo + ZBLK < I) ? lo + ZBLK : I;
        for (int64_t k = lo; k < hi; ++k) z->cdf[k] += bsum[b];
    }
    z->total = z->cdf[I - 1];
    free(bsum);
    z->G = I;
    z->guide = (int64_t *)malloc((size_t)(z->G + 1) * sizeof(int64_t));
    int64_t k = 0;
    for (int64_t g = 0; g <= z->G; ++g) {
        const double t = (double)g * (z->total / (double)z->G);
        while (k < I - 1 && z->cdf[k] <= t) ++k;
        z->guide[g] = k;
    }
}

static void zipf_free(zipf_t *z)
{
    free(z->cdf);
    free(z->guide);
}

static inline int64_t zipf_rank(const zipf_t *z, double u)
{
    const double t = u * z->total;
    int64_t g = (int64_t)(u * (double)z->G);
    if (g > z->G) g = z->G;
    int64_t k = z->guide[g];
    while (k > 0 && z->cdf[k - 1] > t) --k;   /* exact even if g*total/G rounds above t */
    while (k < z->I - 1 && z->cdf[k] <= t) ++k;
    return k;
}

/* ------------------------------------------------------------------ records */

typedef struct {
    uint64_t rest;  /* i_1 .. i_{N-1} packed, i_{N-1} least significant */
    uint32_t i0;    /* I_0 marks a discarded draw                       */
    uint32_t k;     /* draw counter                                     */
} rec_t;

typedef struct {
    int order;
    const int64_t *dims;
    int dist;            /* 0 uniform, 1 zipf */
    zipf_t zipf[8];
    int32_t *perm[8];
    uint64_t key[8];
    int64_t hot;         /* -1: none */
    int fixed_i0;        /* hot-slice generation: i0 forced to hot */
} gen_t;

static inline int64_t gen_index(const gen_t *g, int w, uint64_t k)
{
    const double u = draw_unit(g->key[w], k);
    if (g->dist == 0) {
        int64_t i = (int64_t)(u * (double)g->dims[w]);
        return i < g->dims[w] ? i : g->dims[w] - 1;
    }
    return g->perm[w][zipf_rank(&g->zipf[w], u)];
}

static void draw_records(const gen_t *g, uint64_t k0, int64_t m, rec_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) {
        const uint64_t k = k0 + (uint64_t)j;
        uint64_t rest = 0;
        for (int w = 1; w < g->order; ++w)
            rest = rest * (uint64_t)g->dims[w] + (uint64_t)gen_index(g, w, k);
        int64_t i0;
        if (g->fixed_i0) {
            i0 = g->hot;
        } else {
            i0 = gen_index(g, 0, k);
            if (i0 == g->hot) i0 = g->dims[0]; /* the hot slice is generated apart */
        }
        out[j].rest = rest;
        out[j].i0 = (uint32_t)i0;
        out[j].k = (uint32_t)k;
    }
}

/* Stable LSD radix sort of records by (i0, rest), 11-bit digits. */
static void radix_sort(rec_t *a, rec_t *tmp, int64_t n, int rest_bits, int i0_bits)
{
    const int D = 11, NB = 1 << 11;
    const int total = rest_bits + i0_bits;
    const int passes = (total + D - 1) / D;
    int nt = omp_get_max_threads();
    if (nt < 1) nt = 1;
    int64_t *hist = (int64_t *)malloc((size_t)nt * NB * sizeof(int64_t));
    rec_t *src = a, *dst = tmp;
    for (int p = 0; p < passes; ++p) {
        const int sh = p * D;
        memset(hist, 0, (size_t)nt * NB * sizeof(int64_t));
#define DIGIT(r)                                                                              \
    ((sh + D <= rest_bits) ? (uint32_t)(((r).rest >> sh) & (NB - 1))                          \
     : (sh >= rest_bits)   ? (uint32_t)(((uint64_t)(r).i0 >> (sh - rest_bits)) & (NB - 1))    \
                           : (uint32_t)((((r).rest >> sh) | ((uint64_t)(r).i0 << (rest_bits - sh))) & (NB - 1)))
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num();
            const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
            int64_t *h = hist + (size_t)t * NB;
            for (int64_t i = lo; i < hi; ++i) h[DIGIT(src[i])]++;
#pragma omp barrier
#pragma omp single
            {
                int64_t run = 0;
                for (int b = 0; b < NB; ++b)
                    for (int tt = 0; tt < nt; ++tt) {
                        int64_t c = hist[(size_t)tt * NB + b];
                        hist[(size_t)tt * NB + b] = run;
                        run += c;
                    }
            }
            for (int64_t i = lo; i < hi; ++i) dst[h[DIGIT(src[i])]++] = src[i];
        }
#undef DIGIT
        rec_t *sw = src;
        src = dst;
        dst = sw;
    }
    if (src != a) memcpy(a, src, (size_t)n * sizeof(rec_t));
    free(hist);
}

/*
 * Draw until at least `want` distinct coordinates exist, then keep the first
 * `want` distinct ones in draw order.  Returns a malloc'd array of `want`
 * records sorted by (i0, rest), or NULL.  *draws receives the draw count used.
 */
static rec_t *distinct_first(const gen_t *g, int64_t want, double overs, int rest_bits,
                             int i0_bits, int64_t *draws)
{
    if (want == 0) {
        *draws = 0;
        return (rec_t *)malloc(sizeof(rec_t));
    }
    int64_t m = (int64_t)((double)want * overs) + 1024;
    for (int attempt = 0; attempt < 64; ++attempt) {
        if (m > 0xFFFFFFF0ll) m = 0xFFFFFFF0ll;
        rec_t *a = (rec_t *)malloc((size_t)m * sizeof(rec_t));
        rec_t *t = (rec_t *)malloc((size_t)m * sizeof(rec_t));
        if (!a || !t) {
            free(a);
            free(t);
            return NULL;
        }
        draw_records(g, 0, m, a);
        radix_sort(a, t, m, rest_bits, i0_bits);
        free(t);
        const uint32_t bad = (uint32_t)g->dims[0];
        uint8_t *first_at = (uint8_t *)calloc((size_t)m, 1);
        int64_t distinct = 0;
#pragma omp parallel for reduction(+ : distinct) schedule(static)
        for (int64_t j = 0; j < m; ++j) {
            const int first = (j == 0) || a[j].i0 != a[j - 1].i0 || a[j].rest != a[j - 1].rest;
            if (first && a[j].i0 != bad) {
                first_at[a[j].k] = 1;
                distinct++;
            }
        }
        if (distinct >= want) {
            /* threshold T: the first `want` distinct coordinates have k < T */
            int nt = omp_get_max_threads();
            if (nt < 1) nt = 1;
            int64_t *cnt = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
#pragma omp parallel num_threads(nt)
            {
                const int t = omp_get_thread_num();
                const int64_t lo = m * t / nt, hi = m * (t + 1) / nt;
                int64_t c = 0;
                for (int64_t k = lo; k < hi; ++k) c += first_at[k];
                cnt[t + 1] = c;
            }
            int64_t T = m, run = 0;
            for (int t = 0; t < nt; ++t) {
                const int64_t lo = m * t / nt, hi = m * (t + 1) / nt;
                if (run + cnt[t + 1] >= want) {
                    for (int64_t k = lo; k < hi; ++k) {
                        run += first_at[k];
                        if (run == want) {
                            T = k + 1;
                            break;
                        }
                    }
                    break;
                }
                run += cnt[t + 1];
            }
            /* keep the distinct coordinates first drawn before T, in sorted order */
            rec_t *out = (rec_t *)malloc((size_t)want * sizeof(rec_t));
#pragma omp parallel num_threads(nt)
            {
                const int t = omp_get_thread_num();
                const int64_t lo = m * t / nt, hi = m * (t + 1) / nt;
                int64_t c = 0;
                for (int64_t j = lo; j < hi; ++j)
                    c += (a[j].i0 != bad && a[j].k < (uint64_t)T && first_at[a[j].k] &&
                          (j == 0 || a[j].i0 != a[j - 1].i0 || a[j].rest != a[j - 1].rest));
                cnt[t + 1] = c;
#pragma omp barrier
#pragma omp single
                {
                    cnt[0] = 0;
                    for (int tt = 0; tt < nt; ++tt) cnt[tt + 1] += cnt[tt];
                }
                int64_t o = cnt[t];
                for (int64_t j = lo; j < hi; ++j)
                    if (a[j].i0 != bad && a[j].k < (uint64_t)T && first_at[a[j].k] &&
                        (j == 0 || a[j].i0 != a[j - 1].i0 || a[j].rest != a[j - 1].rest) && o < want)
                        out[o++] = a[j];
            }
            const int64_t o = cnt[nt];
            free(cnt);
            free(first_at);
            free(a);
            *draws = T;
            if (o != want) {
                free(out);
                return NULL;
            }
            return out;
        }
        free(first_at);
        free(a);
        if (m >= 0xFFFFFFF0ll) return NULL;
        const double grow = distinct > 0 ? (double)want / (double)distinct : 4.0;
        m = (int64_t)((double)m * grow * 1.15) + 4096;
    }
    return NULL;
}

/*
 * Generate a sorted, duplicate-free COO tensor.
 *   dist: 0 uniform, 1 Zipf with exponent s.   hot_frac: 0 for no hot slice.
 *   idx_out: int32 [order][nnz].   info_out (nullable, 4 entries):
 *   [0] raw draws (main set), [1] raw draws (hot set), [2] hot index or -1,
 *   [3] nonzeros in the hot slice.
 * Returns 0 on success, negative on error.
 */
int synth_coords(int order, const int64_t *dims, int64_t nnz, int dist, double s,
                 double hot_frac, uint64_t seed, int32_t *idx_out, int64_t *info_out)
{
    if (order < 2 || order > 8 || nnz < 0) return -1;
    double space = 1.0;
    for (int w = 0; w < order; ++w) {
        if (dims[w] < 1 || dims[w] > 0x7FFFFFFF) return -1;
        space *= (double)dims[w];
    }
    double rest_space = 1.0;
    for (int w = 1; w < order; ++w) rest_space *= (double)dims[w];
    if (rest_space >= 1.8e19) return -2;
    uint64_t rest_max = 1;
    for (int w = 1; w < order; ++w) rest_max *= (uint64_t)dims[w];
    const int rest_bits = bits_for(rest_max - 1);
    const int i0_bits = bits_for((uint64_t)dims[0]); /* values 0..I_0 (I_0 = discarded) */

    gen_t g;
    memset(&g, 0, sizeof(g));
    g.order = order;
    g.dims = dims;
    g.dist = dist;
    g.hot = -1;
    for (int w = 0; w < order; ++w) {
        g.key[w] = stream_key(seed, ST_COORD + (uint64_t)w);
        if (dist == 1) {
            zipf_build(&g.zipf[w], dims[w], s);
            g.perm[w] = (int32_t *)malloc((size_t)dims[w] * sizeof(int32_t));
            build_perm(seed, w, dims[w], g.perm[w]);
        }
    }
    int64_t n_hot = 0;
    if (hot_frac > 0.0) {
        n_hot = (int64_t)llround(hot_frac * (double)nnz);
        int32_t *p0 = g.perm[0];
        int32_t tmp0 = 0;
        if (!p0) { /* uniform: still a fixed bijection for the hot index */
            p0 = (int32_t *)malloc((size_t)dims[0] * sizeof(int32_t));
            build_perm(seed, 0, dims[0], p0);
        }
        tmp0 = p0[dims[0] / 2];
        if (!g.perm[0]) free(p0);
        g.hot = tmp0;
        if ((double)n_hot > rest_space) return -3;
    }
    const double overs = (dist == 1) ? 1.6 : (1.0 + 2.0 * (double)nnz / space);
    int64_t draws_main = 0, draws_hot = 0;
    rec_t *main_set = distinct_first(&g, nnz - n_hot, overs, rest_bits, i0_bits, &draws_main);
    rec_t *hot_set = NULL;
    int rc = 0;
    if (!main_set) rc = -4;
    if (!rc && n_hot > 0) {
        gen_t gh = g;
        gh.fixed_i0 = 1;
        for (int w = 0; w < order; ++w) gh.key[w] = stream_key(seed, ST_HOT + (uint64_t)w);
        hot_set = distinct_first(&gh, n_hot, overs, rest_bits, 0, &draws_hot);
        if (!hot_set) rc = -5;
    }
    if (!rc) {
        const int64_t n_main = nnz - n_hot;
        /* position of the hot block in lexicographic order */
        int64_t lo = 0, hi = n_main;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if ((int64_t)main_set[mid].i0 < g.hot) lo = mid + 1; else hi = mid;
        }
        const int64_t ins = (n_hot > 0) ? lo : n_main;
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < nnz; ++j) {
            const rec_t *r;
            if (j < ins) r = &main_set[j];
            else if (j < ins + n_hot) r = &hot_set[j - ins];
            else r = &main_set[j - n_hot];
            uint64_t rest = r->rest;
            for (int w = order - 1; w >= 1; --w) {
                idx_out[(int64_t)w * nnz + j] = (int32_t)(rest % (uint64_t)dims[w]);
                rest /= (uint64_t)dims[w];
            }
            idx_out[j] = (int32_t)r->i0;
        }
    }
    if (info_out) {
        info_out[0] = draws_main;
        info_out[1] = draws_hot;
        info_out[2] = g.hot;
        info_out[3] = n_hot;
    }
    free(main_set);
    free(hot_set);
    for (int w = 0; w < order; ++w) {
        if (dist == 1) {
            zipf_free(&g.zipf[w]);
            free(g.perm[w]);
        }
    }
    return rc;
}

/* Exposed for tests: the rank -> index bijection and Zipf rank of u. */
void synth_rank_perm(uint64_t seed, int mode, int64_t I, int32_t *perm) { build_perm(seed, mode, I, perm); }

int64_t synth_zipf_ranks(int64_t I, double s, uint64_t seed, uint64_t stream, int64_t n, int64_t *out)
{
    zipf_t z;
    zipf_build(&z, I, s);
    const uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) out[j] = zipf_rank(&z, draw_unit(key, (uint64_t)j));
    zipf_free(&z);
    return n;
}
