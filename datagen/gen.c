/*
 * Seeded synthetic sparse tf-idf document generator.
 *
 * Input generator shared by the oracle tests, the GPU tests and the benchmark.
 * It holds none of the clustering arithmetic: it only produces the object set
 * (CSR, FP32 values) and seeded index draws (initial-mean objects, random
 * partitions).  Every document is generated from its own counter-derived
 * random stream, so the output does not depend on the thread count.
 *
 * Recipe (one spec, stated here in full):
 *   nnz_i   ~ Poisson(lambda), clipped to [lo, hi] (and to D)
 *   ranks   drawn one by one from the bounded Zipf law P(r) ~ r^-s, r = 1..D,
 *           rejecting repeats, until nnz_i distinct ranks are held
 *   term id = perm[rank - 1], perm a seeded permutation of [0, D)
 *   tf      = 1 + G, G = failures before the first success at p = 1/2
 *   weight  = (1 + ln tf) * ln(N / df_t), exact zeros (df_t == N) dropped
 *   row     L2-normalised in FP64, then rounded to FP32
 *   term ids ascending within each row.
 *
 * Random streams: splitmix64 finaliser to derive a per-(seed, stream, index)
 * state for xoshiro256** (Blackman and Vigna).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { STREAM_LEN = 1, STREAM_TERMS = 2, STREAM_PERM = 3, STREAM_DRAW = 4 };

static inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } rng_t;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t rng_next(rng_t* r) {
    uint64_t* s = r->s;
    const uint64_t out = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return out;
}

static void rng_init(rng_t* r, uint64_t seed, uint64_t stream, uint64_t index) {
    uint64_t h = mix64(seed);
    h = mix64(h ^ mix64(stream + 0x632be59bd9b4e019ULL));
    h = mix64(h ^ mix64(index + 0x8cb92ba72f3d8dd7ULL));
    for (int i = 0; i < 4; ++i) {
        h = mix64(h);
        r->s[i] = h;
    }
}

/* uniform double in [0, 1) with 53 random bits */
static inline double rng_unif(rng_t* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* Poisson(lambda) as a sum of Poisson(lambda/m) parts, each by Knuth's
 * product-of-uniforms method (exact in distribution for any lambda). */
static int64_t rng_poisson(rng_t* r, double lambda) {
    if (lambda <= 0.0) return 0;
    int m = (int)ceil(lambda / 16.0);
    double part = lambda / m, lim = exp(-part);
    int64_t total = 0;
    for (int p = 0; p < m; ++p) {
        int64_t k = 0;
        double prod = rng_unif(r);
        while (prod > lim) {
            ++k;
            prod *= rng_unif(r);
        }
        total += k;
    }
    return total;
}

/* Walker/Vose alias table over ranks 0..D-1 with weights (r+1)^-s. */
typedef struct {
    int64_t d;
    double* prob;
    int32_t* alias;
    double* w; /* normalised weights, used by the exact fallback */
} alias_t;

static int alias_build(alias_t* a, int64_t d, double s) {
    a->d = d;
    a->prob = (double*)malloc(sizeof(double) * d);
    a->alias = (int32_t*)malloc(sizeof(int32_t) * d);
    a->w = (double*)malloc(sizeof(double) * d);
    int32_t* small = (int32_t*)malloc(sizeof(int32_t) * d);
    int32_t* large = (int32_t*)malloc(sizeof(int32_t) * d);
    double* q = (double*)malloc(sizeof(double) * d);
    if (!a->prob || !a->alias || !a->w || !small || !large || !q) return -1;
    double tot = 0.0;
    for (int64_t r = 0; r < d; ++r) {
        a->w[r] = pow((double)(r + 1), -s);
        tot += a->w[r];
    }
    int64_t ns = 0, nl = 0;
    for (int64_t r = 0; r < d; ++r) {
        a->w[r] /= tot;
        q[r] = a->w[r] * (double)d;
        if (q[r] < 1.0) small[ns++] = (int32_t)r; else large[nl++] = (int32_t)r;
    }
    while (ns > 0 && nl > 0) {
        int32_t sm = small[--ns], lg = large[--nl];
        a->prob[sm] = q[sm];
        a->alias[sm] = lg;
        q[lg] = (q[lg] + q[sm]) - 1.0;
        if (q[lg] < 1.0) small[ns++] = lg; else large[nl++] = lg;
    }
    while (nl > 0) { int32_t lg = large[--nl]; a->prob[lg] = 1.0; a->alias[lg] = lg; }
    while (ns > 0) { int32_t sm = small[--ns]; a->prob[sm] = 1.0; a->alias[sm] = sm; }
    free(small); free(large); free(q);
    return 0;
}

static void alias_free(alias_t* a) { free(a->prob); free(a->alias); free(a->w); }

static inline int64_t alias_draw(const alias_t* a, rng_t* r) {
    uint64_t x = rng_next(r);
    int64_t col = (int64_t)((x >> 32) % (uint64_t)a->d);
    double u = (double)(x & 0xffffffffULL) * 0x1.0p-32;
    return u < a->prob[col] ? col : a->alias[col];
}

/* exact draw from the weights restricted to ranks not yet held (O(D)) */
static int64_t draw_remaining(const alias_t* a, const uint8_t* held, rng_t* r) {
    double mass = 0.0;
    for (int64_t i = 0; i < a->d; ++i) if (!held[i]) mass += a->w[i];
    double u = rng_unif(r) * mass, acc = 0.0;
    int64_t last = -1;
    for (int64_t i = 0; i < a->d; ++i) {
        if (held[i]) continue;
        last = i;
        acc += a->w[i];
        if (u < acc) return i;
    }
    return last;
}

static int64_t doc_len(uint64_t seed, int64_t i, double lam, int64_t lo, int64_t hi, int64_t d) {
    rng_t r;
    rng_init(&r, seed, STREAM_LEN, (uint64_t)i);
    int64_t n = rng_poisson(&r, lam);
    if (n < lo) n = lo;
    if (n > hi) n = hi;
    if (n > d) n = d;
    return n;
}

typedef struct { int32_t t; int32_t tf; } term_tf;

static int cmp_term(const void* x, const void* y) {
    int32_t a = ((const term_tf*)x)->t, b = ((const term_tf*)y)->t;
    return (a > b) - (a < b);
}

/*
 * Two-call interface.  gen_count fills len[N] (raw term counts before idf
 * zero-dropping).  gen_fill then writes the final CSR:
 *   indptr[N+1] (int64), indices[cap] (int32), values[cap] (float)
 * with cap = sum(len); *nnz_out receives the nnz after dropping zero weights.
 * Returns 0 on success, negative on allocation failure.
 */
int gen_count(int64_t n, int64_t d, double lam, int64_t lo, int64_t hi, uint64_t seed,
              int64_t* len) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) len[i] = doc_len(seed, i, lam, lo, hi, d);
    return 0;
}

int gen_fill(int64_t n, int64_t d, double lam, int64_t lo, int64_t hi, double s, uint64_t seed,
             const int64_t* len, int64_t* indptr, int32_t* indices, float* values,
             int64_t* nnz_out) {
    (void)lam; (void)lo; (void)hi;
    alias_t al;
    if (alias_build(&al, d, s) != 0) return -1;
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * d);
    int64_t* raw_ptr = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    int64_t* df = (int64_t*)calloc((size_t)d, sizeof(int64_t));
    if (!perm || !raw_ptr || !df) return -1;
    {
        rng_t r;
        rng_init(&r, seed, STREAM_PERM, 0);
        for (int64_t i = 0; i < d; ++i) perm[i] = (int32_t)i;
        for (int64_t i = d - 1; i > 0; --i) {
            int64_t j = (int64_t)(rng_next(&r) % (uint64_t)(i + 1));
            int32_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
        }
    }
    raw_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) raw_ptr[i + 1] = raw_ptr[i] + len[i];
    const int64_t cap = raw_ptr[n];
    uint8_t* tfs = (uint8_t*)malloc((size_t)(cap > 0 ? cap : 1));
    int32_t* raw = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    int64_t* kept = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double* idf = (double*)malloc(sizeof(double) * (size_t)(d > 0 ? d : 1));
    if (!tfs || !raw || !kept || !idf) return -1;
    int err = 0;

    #pragma omp parallel
    {
        uint8_t* held = (uint8_t*)calloc((size_t)d, 1);
        int64_t* rk = (int64_t*)malloc(sizeof(int64_t) * (d > 0 ? d : 1));
        term_tf* buf = (term_tf*)malloc(sizeof(term_tf) * (d > 0 ? d : 1));
        if (!held || !rk || !buf) {
            #pragma omp atomic write
            err = -1;
        } else {
            #pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < n; ++i) {
                rng_t r;
                rng_init(&r, seed, STREAM_TERMS, (uint64_t)i);
                const int64_t m = len[i];
                int64_t got = 0, tries = 0;
                while (got < m) {
                    int64_t x;
                    if (tries > 64 * m + 4096) x = draw_remaining(&al, held, &r);
                    else x = alias_draw(&al, &r);
                    ++tries;
                    if (held[x]) continue;
                    held[x] = 1;
                    rk[got++] = x;
                }
                for (int64_t h = 0; h < m; ++h) {
                    uint64_t b;
                    do { b = rng_next(&r); } while (b == 0);
                    buf[h].t = perm[rk[h]];
                    buf[h].tf = 1 + __builtin_ctzll(b);
                    held[rk[h]] = 0;
                }
                qsort(buf, (size_t)m, sizeof(term_tf), cmp_term);
                int64_t base = raw_ptr[i];
                for (int64_t h = 0; h < m; ++h) {
                    raw[base + h] = buf[h].t;
                    tfs[base + h] = (uint8_t)buf[h].tf;
                }
            }
        }
        free(held); free(rk); free(buf);
    }
    if (err) return err;
    for (int64_t e = 0; e < cap; ++e) df[raw[e]] += 1;
    for (int64_t t = 0; t < d; ++t) idf[t] = df[t] > 0 ? log((double)n / (double)df[t]) : 0.0;

    /* a weight is exactly zero iff idf is (df == N): such entries are dropped */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t e = raw_ptr[i]; e < raw_ptr[i + 1]; ++e) c += idf[raw[e]] != 0.0;
        kept[i] = c;
    }
    indptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) indptr[i + 1] = indptr[i] + kept[i];

    #pragma omp parallel
    {
        double* row = (double*)malloc(sizeof(double) * (d > 0 ? d : 1));
        #pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t o = indptr[i], c = 0;
            for (int64_t e = raw_ptr[i]; e < raw_ptr[i + 1]; ++e) {
                int32_t t = raw[e];
                if (idf[t] == 0.0) continue;
                row[c] = (1.0 + log((double)tfs[e])) * idf[t];
                indices[o + c] = t;
                ++c;
            }
            double ss = 0.0;
            for (int64_t h = 0; h < c; ++h) ss += row[h] * row[h];
            double nrm = sqrt(ss);
            for (int64_t h = 0; h < c; ++h) values[o + h] = (float)(row[h] / nrm);
        }
        free(row);
    }
    *nnz_out = indptr[n];
    free(tfs); free(raw); free(kept); free(idf); free(df); free(raw_ptr); free(perm);
    alias_free(&al);
    return 0;
}

/* First m entries of a seeded uniform permutation of [0, n) (partial
 * Fisher-Yates over a sparse swap map, O(m log m) memory-light). */
typedef struct { int64_t key, val; } kv_t;

static int64_t map_get(kv_t* tab, int64_t capm1, int64_t key) {
    uint64_t h = mix64((uint64_t)key) & (uint64_t)capm1;
    while (tab[h].key != -1) {
        if (tab[h].key == key) return tab[h].val;
        h = (h + 1) & (uint64_t)capm1;
    }
    return key;
}

static void map_put(kv_t* tab, int64_t capm1, int64_t key, int64_t val) {
    uint64_t h = mix64((uint64_t)key) & (uint64_t)capm1;
    while (tab[h].key != -1 && tab[h].key != key) h = (h + 1) & (uint64_t)capm1;
    tab[h].key = key;
    tab[h].val = val;
}

int gen_perm_prefix(int64_t n, int64_t m, uint64_t seed, uint64_t stream, int64_t* out) {
    if (m > n) m = n;
    int64_t cap = 16;
    while (cap < 4 * m + 16) cap <<= 1;
    kv_t* tab = (kv_t*)malloc(sizeof(kv_t) * cap);
    if (!tab) return -1;
    for (int64_t i = 0; i < cap; ++i) tab[i].key = -1;
    rng_t r;
    rng_init(&r, seed, STREAM_DRAW + stream, 0);
    for (int64_t i = 0; i < m; ++i) {
        int64_t j = i + (int64_t)(rng_next(&r) % (uint64_t)(n - i));
        int64_t vi = map_get(tab, cap - 1, i), vj = map_get(tab, cap - 1, j);
        out[i] = vj;
        map_put(tab, cap - 1, j, vi);
        map_put(tab, cap - 1, i, vj);
    }
    free(tab);
    return 0;
}

/* n draws uniform in [0, k) (a seeded random partition) */
int gen_uniform_labels(int64_t n, int32_t k, uint64_t seed, uint64_t stream, int32_t* out) {
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < (n + 4095) / 4096; ++b) {
        rng_t r;
        rng_init(&r, seed, STREAM_DRAW + stream, (uint64_t)b + 1);
        int64_t e = (b + 1) * 4096 < n ? (b + 1) * 4096 : n;
        for (int64_t i = b * 4096; i < e; ++i) out[i] = (int32_t)(rng_next(&r) % (uint64_t)k);
    }
    return 0;
}

/* uniform doubles in [0, 1) for instance-parameter draws */
int gen_uniform01(int64_t n, uint64_t seed, uint64_t stream, double* out) {
    rng_t r;
    rng_init(&r, seed, STREAM_DRAW + stream, 0);
    for (int64_t i = 0; i < n; ++i) out[i] = rng_unif(&r);
    return 0;
}
