/*
 * Seeded synthetic inputs for batch-dynamic rooted spanning forest runs.
 *
 * This library produces graphs, initial forests and update batches.  It holds
 * none of the spanning-forest update arithmetic: it only draws random numbers,
 * builds edge sets, converts them to CSR and runs a plain breadth-first search
 * to produce the initial rooted forest that the update method takes as input.
 * Both the CPU oracle and the GPU path consume its outputs.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) seeds xoshiro256**
 * (Blackman and Vigna, "Scrambled linear pseudorandom number generators",
 * ACM TOMS 2021).  Bounded integers use Lemire's multiply-and-reject method
 * ("Fast random integer generation in an interval", ACM TOMACS 2019).
 * Parallel generation splits work into fixed chunks, each with its own
 * stream, so results do not depend on the thread count.
 *
 * Edge keys: an undirected edge {u, v} with u < v is the 64-bit key
 * (u << 32) | v.  Key arrays returned here are sorted ascending and unique.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------ PRNG */

static inline uint64_t sm64_next(uint64_t *x) {
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } xo_t;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t xo_next(xo_t *r) {
    uint64_t *s = r->s;
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

static void xo_seed(xo_t *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; i++) r->s[i] = sm64_next(&x);
}

/* uniform integer in [0, n) for 0 < n < 2^32 (Lemire) */
static inline uint32_t xo_below32(xo_t *r, uint32_t n) {
    uint64_t m = (uint64_t)(uint32_t)(xo_next(r) >> 32) * n;
    uint32_t lo = (uint32_t)m;
    if (lo < n) {
        uint32_t thresh = (uint32_t)(-n) % n;
        while (lo < thresh) {
            m = (uint64_t)(uint32_t)(xo_next(r) >> 32) * n;
            lo = (uint32_t)m;
        }
    }
    return (uint32_t)(m >> 32);
}

/* uniform integer in [0, n) for 0 < n < 2^63 (rejection on a power-of-two mask) */
static inline uint64_t xo_below64(xo_t *r, uint64_t n) {
    if (n <= 0xffffffffULL) return xo_below32(r, (uint32_t)n);
    uint64_t mask = n - 1;
    mask |= mask >> 1; mask |= mask >> 2; mask |= mask >> 4;
    mask |= mask >> 8; mask |= mask >> 16; mask |= mask >> 32;
    for (;;) {
        uint64_t x = xo_next(r) & mask;
        if (x < n) return x;
    }
}

uint64_t drsfgen_splitmix64(uint64_t x) { return sm64_next(&x); }

/* seed = splitmix64(config_id ^ instance * 2^32 ^ purpose) */
uint64_t drsfgen_seed(uint64_t config_id, uint64_t instance, uint64_t purpose) {
    uint64_t x = config_id ^ (instance << 32) ^ purpose;
    return sm64_next(&x);
}

/* ------------------------------------------------------------- key sets */

static inline uint64_t mkkey(uint32_t u, uint32_t v) {
    return u < v ? (((uint64_t)u << 32) | v) : (((uint64_t)v << 32) | u);
}

/* open-addressing set of 64-bit keys; UINT64_MAX marks an empty slot */
typedef struct { uint64_t *slot; uint64_t mask; } kset_t;

static int kset_init(kset_t *s, uint64_t expected) {
    uint64_t cap = 16;
    while (cap < 2 * expected + 16) cap <<= 1;
    s->slot = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!s->slot) return -1;
    memset(s->slot, 0xff, cap * sizeof(uint64_t));
    s->mask = cap - 1;
    return 0;
}
static void kset_free(kset_t *s) { free(s->slot); s->slot = 0; }
static inline uint64_t kmix(uint64_t k) {
    k ^= k >> 33; k *= 0xff51afd7ed558ccdULL; k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL; k ^= k >> 33; return k;
}
/* returns 1 if inserted, 0 if already present */
static inline int kset_add(kset_t *s, uint64_t k) {
    uint64_t h = kmix(k) & s->mask;
    for (;;) {
        uint64_t cur = s->slot[h];
        if (cur == UINT64_MAX) { s->slot[h] = k; return 1; }
        if (cur == k) return 0;
        h = (h + 1) & s->mask;
    }
}
static inline int kset_has(const kset_t *s, uint64_t k) {
    uint64_t h = kmix(k) & s->mask;
    for (;;) {
        uint64_t cur = s->slot[h];
        if (cur == UINT64_MAX) return 0;
        if (cur == k) return 1;
        h = (h + 1) & s->mask;
    }
}

/* parallel LSD radix sort of 64-bit keys on the low `bits` bits (stable,
 * result independent of thread count).  tmp must hold n keys. */
static void radix_sort_u64(uint64_t *a, uint64_t *tmp, int64_t n, int bits) {
    const int R = 11, B = 1 << R;
    int nthreads = omp_get_max_threads();
    if (nthreads > 64) nthreads = 64;
    int64_t *hist = (int64_t *)malloc((size_t)nthreads * B * sizeof(int64_t));
    uint64_t *src = a, *dst = tmp;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += R, passes++) {
        memset(hist, 0, (size_t)nthreads * B * sizeof(int64_t));
#pragma omp parallel num_threads(nthreads)
        {
            int t = omp_get_thread_num();
            int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
            int64_t *h = hist + (size_t)t * B;
            for (int64_t i = lo; i < hi; i++) h[(src[i] >> shift) & (B - 1)]++;
        }
        int64_t run = 0;
        for (int d = 0; d < B; d++)
            for (int t = 0; t < nthreads; t++) {
                int64_t c = hist[(size_t)t * B + d];
                hist[(size_t)t * B + d] = run;
                run += c;
            }
#pragma omp parallel num_threads(nthreads)
        {
            int t = omp_get_thread_num();
            int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
            int64_t *h = hist + (size_t)t * B;
            for (int64_t i = lo; i < hi; i++) dst[h[(src[i] >> shift) & (B - 1)]++] = src[i];
        }
        uint64_t *sw = src; src = dst; dst = sw;
    }
    if (src != a) memcpy(a, src, (size_t)n * sizeof(uint64_t));
    free(hist);
}

static int key_bits(int32_t n) {
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) < (int64_t)n) b++;
    return 32 + b;
}

/* sort + unique in place; returns the new length */
static int64_t sort_unique(uint64_t *keys, int64_t m, int32_t n) {
    if (m <= 1) return m;
    uint64_t *tmp = (uint64_t *)malloc((size_t)m * sizeof(uint64_t));
    if (!tmp) return -1;
    radix_sort_u64(keys, tmp, m, key_bits(n));
    free(tmp);
    int64_t w = 1;
    for (int64_t i = 1; i < m; i++)
        if (keys[i] != keys[w - 1]) keys[w++] = keys[i];
    return w;
}

/* ------------------------------------------------------------- graphs */

/* G(n, m): m distinct unordered pairs drawn uniformly, no self-loops.
 * keys must hold m entries.  Returns m, or -1 if m is infeasible. */
int64_t drsfgen_gnm(int32_t n, int64_t m, uint64_t seed, uint64_t *keys) {
    if (n < 2 && m > 0) return -1;
    if ((double)m > 0.5 * (double)n * (double)(n - 1)) return -1;
    kset_t s;
    if (kset_init(&s, (uint64_t)m)) return -1;
    xo_t r;
    xo_seed(&r, seed);
    int64_t got = 0;
    while (got < m) {
        uint32_t u = xo_below32(&r, (uint32_t)n), v = xo_below32(&r, (uint32_t)n);
        if (u == v) continue;
        uint64_t k = mkkey(u, v);
        if (kset_add(&s, k)) keys[got++] = k;
    }
    kset_free(&s);
    return sort_unique(keys, m, n);
}

/* R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): `samples` edge draws on
 * 2^scale vertices, one quadrant choice per level with probabilities a, b, c
 * and d = 1 - a - b - c, no noise and no vertex permutation.  Self-loops are
 * dropped, pairs made undirected and duplicates removed.  keys must hold
 * `samples` entries.  Returns the number of unique undirected edges. */
int64_t drsfgen_rmat(int scale, int64_t samples, double a, double b, double c,
                     uint64_t seed, uint64_t *keys) {
    if (scale < 1 || scale > 30) return -1;
    const uint64_t ta = (uint64_t)(a * 4294967296.0);
    const uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
    const uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
    const int64_t CH = 1 << 16;
    const int64_t nch = (samples + CH - 1) / CH;
    int32_t *cnt = (int32_t *)calloc((size_t)nch, sizeof(int32_t));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ch = 0; ch < nch; ch++) {
        xo_t r;
        xo_seed(&r, seed ^ sm64_next(&(uint64_t){(uint64_t)ch * 0x2545f4914f6cdd1dULL + 1}));
        int64_t lo = ch * CH, hi = lo + CH < samples ? lo + CH : samples;
        int32_t w = 0;
        for (int64_t i = lo; i < hi; i++) {
            uint32_t u = 0, v = 0;
            uint64_t bitsleft = 0, rnd = 0;
            for (int l = 0; l < scale; l++) {
                if (bitsleft == 0) { rnd = xo_next(&r); bitsleft = 2; }
                uint64_t x = rnd & 0xffffffffULL;
                rnd >>= 32;
                bitsleft--;
                uint32_t bu, bv;
                if (x < ta) { bu = 0; bv = 0; }
                else if (x < tb) { bu = 0; bv = 1; }
                else if (x < tc) { bu = 1; bv = 0; }
                else { bu = 1; bv = 1; }
                u = (u << 1) | bu;
                v = (v << 1) | bv;
            }
            if (u != v) keys[lo + w++] = mkkey(u, v);
        }
        cnt[ch] = w;
    }
    /* squeeze out the dropped self-loops, chunk by chunk in order */
    int64_t total = 0;
    for (int64_t ch = 0; ch < nch; ch++) {
        int64_t lo = ch * CH;
        if (total != lo) memmove(keys + total, keys + lo, (size_t)cnt[ch] * sizeof(uint64_t));
        total += cnt[ch];
    }
    free(cnt);
    return sort_unique(keys, total, (int32_t)(1u << (scale < 31 ? scale : 30)));
}

/* rows x cols 4-neighbour grid, id = r * cols + c, with exactly n_remove
 * edges removed uniformly without replacement.  keys must hold all
 * rows*(cols-1) + (rows-1)*cols edges.  Returns the surviving count. */
int64_t drsfgen_grid(int32_t rows, int32_t cols, int64_t n_remove, uint64_t seed,
                     uint64_t *keys) {
    int64_t total = (int64_t)rows * (cols - 1) + (int64_t)(rows - 1) * cols;
    if (n_remove < 0 || n_remove > total) return -1;
    int64_t w = 0;
    for (int32_t r = 0; r < rows; r++)
        for (int32_t c = 0; c < cols; c++) {
            uint32_t id = (uint32_t)r * (uint32_t)cols + (uint32_t)c;
            if (c + 1 < cols) keys[w++] = mkkey(id, id + 1);
            if (r + 1 < rows) keys[w++] = mkkey(id, id + (uint32_t)cols);
        }
    /* Floyd's sampling of n_remove distinct indices in [0, total) */
    uint8_t *gone = (uint8_t *)calloc((size_t)total, 1);
    xo_t rr;
    xo_seed(&rr, seed);
    for (int64_t j = total - n_remove; j < total; j++) {
        int64_t t = (int64_t)xo_below64(&rr, (uint64_t)j + 1);
        if (gone[t]) gone[j] = 1; else gone[t] = 1;
    }
    int64_t o = 0;
    for (int64_t i = 0; i < total; i++)
        if (!gone[i]) keys[o++] = keys[i];
    free(gone);
    return sort_unique(keys, o, rows * cols);
}

/* Symmetric CSR with ascending rows from sorted unique keys (u < v). */
void drsfgen_keys_to_csr(int32_t n, const uint64_t *keys, int64_t m, int64_t *row_ptr,
                         int32_t *col) {
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < m; i++) {
        fill[keys[i] >> 32]++;
        fill[(uint32_t)keys[i]]++;
    }
    row_ptr[0] = 0;
    for (int32_t v = 0; v < n; v++) row_ptr[v + 1] = row_ptr[v] + fill[v];
    for (int32_t v = 0; v < n; v++) fill[v] = row_ptr[v];
    /* keys ascending => lower neighbours arrive in ascending order before the
     * upper neighbours of the same row, which also ascend */
    for (int64_t i = 0; i < m; i++) {
        uint32_t u = (uint32_t)(keys[i] >> 32), v = (uint32_t)keys[i];
        col[fill[u]++] = (int32_t)v;
        col[fill[v]++] = (int32_t)u;
    }
    free(fill);
}

/* Canonical initial forest: breadth-first levels from the smallest vertex of
 * each component; every other vertex takes as parent its smallest-id
 * neighbour one level closer to the root; a root points to itself. */
void drsfgen_bfs_forest(int32_t n, const int64_t *row_ptr, const int32_t *col,
                        int32_t *parent) {
    int32_t *dist = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    for (int32_t v = 0; v < n; v++) dist[v] = -1;
    for (int32_t s = 0; s < n; s++) {
        if (dist[s] >= 0) continue;
        int64_t qh = 0, qt = 0;
        dist[s] = 0;
        queue[qt++] = s;
        while (qh < qt) {
            int32_t u = queue[qh++];
            for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
                int32_t w = col[e];
                if (dist[w] < 0) { dist[w] = dist[u] + 1; queue[qt++] = w; }
            }
        }
    }
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; v++) {
        parent[v] = v;
        if (dist[v] == 0) continue;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
            if (dist[col[e]] == dist[v] - 1) { parent[v] = col[e]; break; }
    }
    free(dist);
    free(queue);
}

/* ------------------------------------------------------------- batches */

static int key_in_sorted(const uint64_t *keys, int64_t m, uint64_t k) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo < m && keys[lo] == k;
}

/* nb batches of b uniform random non-edges of the graph given by sorted keys,
 * distinct across all batches; pairs are written as drawn (u, v), u != v.
 * Returns 0, or -1 if not enough non-edges exist. */
int64_t drsfgen_insert_batches(int32_t n, const uint64_t *keys, int64_t m, int64_t nb,
                               int64_t b, uint64_t seed, int32_t *edges) {
    double non_edges = 0.5 * (double)n * (double)(n - 1) - (double)m;
    if ((double)(nb * b) > non_edges) return -1;
    kset_t s;
    if (kset_init(&s, (uint64_t)(nb * b))) return -1;
    xo_t r;
    xo_seed(&r, seed);
    for (int64_t i = 0; i < nb * b;) {
        uint32_t u = xo_below32(&r, (uint32_t)n), v = xo_below32(&r, (uint32_t)n);
        if (u == v) continue;
        uint64_t k = mkkey(u, v);
        if (key_in_sorted(keys, m, k)) continue;
        if (!kset_add(&s, k)) continue;
        edges[2 * i] = (int32_t)u;
        edges[2 * i + 1] = (int32_t)v;
        i++;
    }
    kset_free(&s);
    return 0;
}

/* nb batches of b existing edges each: n_tree drawn uniformly without
 * replacement from the tree edges {v, parent[v]} of the given forest and
 * b - n_tree from the other edges, distinct across all batches, each pair
 * written in a random orientation.  Returns 0, or -1 if too few exist. */
int64_t drsfgen_delete_batches(int32_t n, const uint64_t *keys, int64_t m,
                               const int32_t *parent, int64_t nb, int64_t b, int64_t n_tree,
                               uint64_t seed, int32_t *edges) {
    if (n_tree > b) return -1;
    int64_t trees = 0;
    for (int32_t v = 0; v < n; v++) trees += parent[v] != v;
    if (nb * n_tree > trees || nb * (b - n_tree) > m - trees) return -1;
    kset_t s;
    if (kset_init(&s, (uint64_t)(nb * b))) return -1;
    xo_t r;
    xo_seed(&r, seed);
    for (int64_t bi = 0; bi < nb; bi++) {
        int32_t *out = edges + 2 * bi * b;
        int64_t w = 0;
        while (w < n_tree) {
            uint32_t v = xo_below32(&r, (uint32_t)n);
            if (parent[v] == (int32_t)v) continue;
            uint64_t k = mkkey(v, (uint32_t)parent[v]);
            if (!kset_add(&s, k)) continue;
            uint32_t p = (uint32_t)parent[v];
            int flip = (int)(xo_next(&r) >> 63);
            out[2 * w] = (int32_t)(flip ? p : v);
            out[2 * w + 1] = (int32_t)(flip ? v : p);
            w++;
        }
        while (w < b) {
            uint64_t k = keys[xo_below64(&r, (uint64_t)m)];
            uint32_t u = (uint32_t)(k >> 32), v = (uint32_t)k;
            if (parent[u] == (int32_t)v || parent[v] == (int32_t)u) continue;
            if (!kset_add(&s, k)) continue;
            int flip = (int)(xo_next(&r) >> 63);
            out[2 * w] = (int32_t)(flip ? v : u);
            out[2 * w + 1] = (int32_t)(flip ? u : v);
            w++;
        }
        /* interleave tree and non-tree edges: Fisher-Yates over the batch */
        for (int64_t i = b - 1; i > 0; i--) {
            int64_t j = (int64_t)xo_below64(&r, (uint64_t)i + 1);
            int32_t t0 = out[2 * i], t1 = out[2 * i + 1];
            out[2 * i] = out[2 * j]; out[2 * i + 1] = out[2 * j + 1];
            out[2 * j] = t0; out[2 * j + 1] = t1;
        }
    }
    kset_free(&s);
    return 0;
}

/* Fill out[0..count) with uniform doubles in [0, 1) (53-bit). */
void drsfgen_uniform(uint64_t seed, int64_t count, double *out) {
    xo_t r;
    xo_seed(&r, seed);
    for (int64_t i = 0; i < count; i++) out[i] = (double)(xo_next(&r) >> 11) * 0x1.0p-53;
}

/* Uniform integers in [0, bound) */
void drsfgen_below(uint64_t seed, int64_t count, uint64_t bound, uint64_t *out) {
    xo_t r;
    xo_seed(&r, seed);
    for (int64_t i = 0; i < count; i++) out[i] = xo_below64(&r, bound);
}

int drsfgen_threads(void) { return omp_get_max_threads(); }
