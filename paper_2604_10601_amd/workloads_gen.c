/*
 * workloads_gen.c -- native part of the seeded synthetic input generators.
 *
 * Inputs only: this file builds data graphs and random-walk vertex sets.  It
 * holds none of the matching arithmetic and is shared by the GPU tests, the
 * benchmark and the CPU oracle's tests alike (through workloads.py).
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
 * used as a counter-based generator: value c of stream `key` is the SplitMix64
 * finaliser applied to key + (c + 1) * golden_gamma.  Any value can be drawn
 * independently of the others, so the graphs do not depend on the number of
 * threads that build them.
 *
 * R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): draw i picks one of the
 * four quadrants (a, b, c, d) at each of `scale` levels with one uniform 32-bit
 * number (two per SplitMix64 value, low half first), giving a (source, target)
 * pair.  Self-loops are dropped, pairs are made undirected and deduplicated,
 * vertex ids are renamed by a caller-supplied permutation, and the result is
 * written as a symmetric CSR with every row strictly ascending.
 *
 * Random walk (query extraction): from a uniform vertex of degree >= 1, step to
 * a uniform neighbour; a vertex not seen before is added; after 100 * k steps
 * without a new vertex the walk restarts from a fresh uniform vertex.  The
 * induced edges among the k vertices are reported as pairs of positions.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define WG_OK 0
#define WG_ERR_ARG (-1)
#define WG_ERR_NOMEM (-5)
#define WG_ERR_NOWALK (-6)

static const uint64_t kGamma = 0x9e3779b97f4a7c15ull;

static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* Value c of the stream with key `key`. */
static inline uint64_t sm_at(uint64_t key, uint64_t c) { return sm_mix(key + (c + 1u) * kGamma); }

/* Key of stream `stream` under `seed`. */
static inline uint64_t stream_key(uint64_t seed, uint64_t stream) { return sm_at(sm_mix(seed), stream); }

/* Uniform integer in [0, d) from a 64-bit value (multiply-high; bias below d / 2^64). */
static inline uint64_t below(uint64_t r, uint64_t d) { return (uint64_t)(((unsigned __int128)r * d) >> 64); }

/* ------------------------------------------------------------------------- */
/* A minimal parallel for: `threads` workers take chunks from a shared counter. */

typedef void (*range_fn)(void *ctx, int64_t begin, int64_t end);

typedef struct {
    range_fn fn;
    void *ctx;
    int64_t n, chunk;
    atomic_llong next;
} pfor_t;

static void *pfor_worker(void *p) {
    pfor_t *f = (pfor_t *)p;
    for (;;) {
        int64_t b = atomic_fetch_add(&f->next, f->chunk);
        if (b >= f->n) break;
        int64_t e = b + f->chunk < f->n ? b + f->chunk : f->n;
        f->fn(f->ctx, b, e);
    }
    return NULL;
}

static void parallel_for(int threads, int64_t n, int64_t chunk, range_fn fn, void *ctx) {
    if (n <= 0) return;
    pfor_t f;
    f.fn = fn;
    f.ctx = ctx;
    f.n = n;
    f.chunk = chunk > 0 ? chunk : 1;
    atomic_init(&f.next, 0);
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    pthread_t tid[64];
    int started = 0;
    for (int t = 1; t < threads; ++t)
        if (pthread_create(&tid[started], NULL, pfor_worker, &f) == 0) ++started;
    pfor_worker(&f);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
}

/* ------------------------------------------------------------------------- */
/* Row sorting. */

static int cmp_u32(const void *x, const void *y) {
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return (a > b) - (a < b);
}

static void sort_u32(uint32_t *v, int64_t n) {
    if (n <= 32) {
        for (int64_t i = 1; i < n; ++i) {
            uint32_t x = v[i];
            int64_t j = i;
            while (j > 0 && v[j - 1] > x) {
                v[j] = v[j - 1];
                --j;
            }
            v[j] = x;
        }
    } else {
        qsort(v, (size_t)n, sizeof(uint32_t), cmp_u32);
    }
}

/* ------------------------------------------------------------------------- */
/* R-MAT. */

typedef struct {
    int64_t n;
    int64_t nnz;
    int64_t *row_ptr; /* [n + 1] */
    uint32_t *col;    /* [nnz] */
} wg_graph;

typedef struct {
    int scale;
    uint64_t key;
    uint32_t ta, tab, tabc; /* quadrant thresholds on a 32-bit uniform */
    uint32_t *lo, *hi;      /* canonical pair of each draw; lo == hi marks a dropped loop */
    atomic_uint *deg;       /* per vertex */
    int64_t *ptr;
    atomic_llong *cur;
    uint32_t *dcol;         /* lo -> hi lists */
    int64_t *ulen;          /* distinct entries per lo row */
    const int64_t *perm;
    uint32_t *col;
} rmat_ctx;

static void rmat_draw(void *p, int64_t b, int64_t e) {
    rmat_ctx *c = (rmat_ctx *)p;
    const int halves = (c->scale + 1) / 2;
    for (int64_t i = b; i < e; ++i) {
        uint32_t s = 0, d = 0;
        uint64_t r = 0;
        for (int j = 0; j < c->scale; ++j) {
            if ((j & 1) == 0) r = sm_at(c->key, (uint64_t)i * (uint64_t)halves + (uint64_t)(j >> 1));
            const uint32_t u = (j & 1) ? (uint32_t)(r >> 32) : (uint32_t)r;
            const uint32_t down = u >= c->tab;
            const uint32_t right = (u >= c->ta && u < c->tab) || u >= c->tabc;
            s = (s << 1) | down;
            d = (d << 1) | right;
        }
        c->lo[i] = s < d ? s : d;
        c->hi[i] = s < d ? d : s;
        if (s != d) atomic_fetch_add_explicit(&c->deg[c->lo[i]], 1u, memory_order_relaxed);
    }
}

static void rmat_scatter(void *p, int64_t b, int64_t e) {
    rmat_ctx *c = (rmat_ctx *)p;
    for (int64_t i = b; i < e; ++i) {
        if (c->lo[i] == c->hi[i]) continue;
        const int64_t at = atomic_fetch_add_explicit(&c->cur[c->lo[i]], 1, memory_order_relaxed);
        c->dcol[at] = c->hi[i];
    }
}

static void rmat_dedup(void *p, int64_t b, int64_t e) {
    rmat_ctx *c = (rmat_ctx *)p;
    for (int64_t v = b; v < e; ++v) {
        uint32_t *row = c->dcol + c->ptr[v];
        const int64_t len = c->ptr[v + 1] - c->ptr[v];
        sort_u32(row, len);
        int64_t u = 0;
        for (int64_t t = 0; t < len; ++t)
            if (u == 0 || row[t] != row[u - 1]) row[u++] = row[t];
        c->ulen[v] = u;
        for (int64_t t = 0; t < u; ++t) {
            atomic_fetch_add_explicit(&c->deg[c->perm[v]], 1u, memory_order_relaxed);
            atomic_fetch_add_explicit(&c->deg[c->perm[row[t]]], 1u, memory_order_relaxed);
        }
    }
}

static void rmat_symmetrise(void *p, int64_t b, int64_t e) {
    rmat_ctx *c = (rmat_ctx *)p;
    for (int64_t v = b; v < e; ++v) {
        const uint32_t *row = c->dcol + c->ptr[v];
        const uint32_t pv = (uint32_t)c->perm[v];
        for (int64_t t = 0; t < c->ulen[v]; ++t) {
            const uint32_t pw = (uint32_t)c->perm[row[t]];
            c->col[atomic_fetch_add_explicit(&c->cur[pv], 1, memory_order_relaxed)] = pw;
            c->col[atomic_fetch_add_explicit(&c->cur[pw], 1, memory_order_relaxed)] = pv;
        }
    }
}

typedef struct {
    const int64_t *row_ptr;
    uint32_t *col;
} rows_ctx;

static void sort_rows(void *p, int64_t b, int64_t e) {
    rows_ctx *c = (rows_ctx *)p;
    for (int64_t v = b; v < e; ++v) sort_u32(c->col + c->row_ptr[v], c->row_ptr[v + 1] - c->row_ptr[v]);
}

/* Exclusive prefix sum of deg into ptr[0 .. n] (sequential: n is at most 2^31). */
static void prefix(const atomic_uint *deg, int64_t n, int64_t *ptr) {
    ptr[0] = 0;
    for (int64_t v = 0; v < n; ++v) ptr[v + 1] = ptr[v] + (int64_t)atomic_load_explicit(&deg[v], memory_order_relaxed);
}

/*
 * Builds the R-MAT graph with 2^scale vertices from edge_factor * 2^scale draws
 * (quadrant probabilities a, b, c, 1 - a - b - c), renamed by perm (a
 * permutation of 0 .. 2^scale - 1).  On success *out holds the graph; read it
 * with wg_graph_size / wg_graph_fetch and release it with wg_graph_free.
 */
int wg_rmat(int scale, int edge_factor, double a, double b, double c, uint64_t seed, const int64_t *perm,
            int threads, wg_graph **out) {
    if (!out || !perm || scale < 1 || scale > 30 || edge_factor < 1 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0)
        return WG_ERR_ARG;
    *out = NULL;
    const int64_t n = (int64_t)1 << scale;
    const int64_t draws = (int64_t)edge_factor << scale;
    rmat_ctx x;
    memset(&x, 0, sizeof(x));
    x.scale = scale;
    x.key = stream_key(seed, 0);
    x.ta = (uint32_t)(a * 4294967296.0);
    x.tab = (uint32_t)((a + b) * 4294967296.0);
    x.tabc = (a + b + c) >= 1.0 ? 0xffffffffu : (uint32_t)((a + b + c) * 4294967296.0);
    x.perm = perm;
    wg_graph *g = (wg_graph *)calloc(1, sizeof(wg_graph));
    x.lo = (uint32_t *)malloc((size_t)draws * 4);
    x.hi = (uint32_t *)malloc((size_t)draws * 4);
    x.deg = (atomic_uint *)calloc((size_t)n, sizeof(atomic_uint));
    x.ptr = (int64_t *)malloc((size_t)(n + 1) * 8);
    x.cur = (atomic_llong *)malloc((size_t)n * sizeof(atomic_llong));
    x.ulen = (int64_t *)malloc((size_t)n * 8);
    int rc = WG_ERR_NOMEM;
    if (!g || !x.lo || !x.hi || !x.deg || !x.ptr || !x.cur || !x.ulen) goto fail;

    /* 1. draws, canonical pairs, lo-row lengths */
    parallel_for(threads, draws, 1 << 16, rmat_draw, &x);
    /* 2. lists lo -> hi */
    prefix(x.deg, n, x.ptr);
    x.dcol = (uint32_t *)malloc((size_t)(x.ptr[n] > 0 ? x.ptr[n] : 1) * 4);
    if (!x.dcol) goto fail;
    for (int64_t v = 0; v < n; ++v) atomic_init(&x.cur[v], x.ptr[v]);
    parallel_for(threads, draws, 1 << 16, rmat_scatter, &x);
    free(x.lo);
    free(x.hi);
    x.lo = x.hi = NULL;
    /* 3. sort and deduplicate every lo row; count renamed degrees of both ends */
    for (int64_t v = 0; v < n; ++v) atomic_init(&x.deg[v], 0u);
    parallel_for(threads, n, 1 << 12, rmat_dedup, &x);
    /* 4. symmetric CSR under the renaming, rows sorted */
    g->n = n;
    g->row_ptr = (int64_t *)malloc((size_t)(n + 1) * 8);
    if (!g->row_ptr) goto fail;
    prefix(x.deg, n, g->row_ptr);
    g->nnz = g->row_ptr[n];
    g->col = (uint32_t *)malloc((size_t)(g->nnz > 0 ? g->nnz : 1) * 4);
    if (!g->col) goto fail;
    x.col = g->col;
    for (int64_t v = 0; v < n; ++v) atomic_init(&x.cur[v], g->row_ptr[v]);
    parallel_for(threads, n, 1 << 12, rmat_symmetrise, &x);
    rows_ctx rc2 = {g->row_ptr, g->col};
    parallel_for(threads, n, 1 << 12, sort_rows, &rc2);
    rc = WG_OK;
    *out = g;
    g = NULL;
fail:
    free(x.lo);
    free(x.hi);
    free(x.deg);
    free(x.ptr);
    free(x.cur);
    free(x.ulen);
    free(x.dcol);
    if (g) {
        free(g->row_ptr);
        free(g->col);
        free(g);
    }
    return rc;
}

int64_t wg_graph_nnz(const wg_graph *g) { return g ? g->nnz : -1; }

/* Copies the CSR into row_ptr[n + 1] and col[nnz]. */
int wg_graph_fetch(const wg_graph *g, int64_t *row_ptr, int32_t *col) {
    if (!g || !row_ptr || (g->nnz > 0 && !col)) return WG_ERR_ARG;
    memcpy(row_ptr, g->row_ptr, (size_t)(g->n + 1) * 8);
    if (g->nnz > 0) memcpy(col, g->col, (size_t)g->nnz * 4);
    return WG_OK;
}

void wg_graph_free(wg_graph *g) {
    if (!g) return;
    free(g->row_ptr);
    free(g->col);
    free(g);
}

/* ------------------------------------------------------------------------- */
/* Random walks. */

static int adjacent(const int64_t *row_ptr, const int32_t *col, int32_t u, int32_t v) {
    int64_t lo = row_ptr[u], hi = row_ptr[u + 1];
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo < row_ptr[u + 1] && col[lo] == v;
}

/*
 * k distinct vertices visited by the random walk of stream `stream` under
 * `seed` (vertices in discovery order), and the induced edges among them as
 * position pairs (a, b), a < b, in lexicographic order: edges[2 * t], edges[2 *
 * t + 1] for t < *m.  live[0 .. nlive) lists the vertices of degree >= 1.
 * Returns the number of walks started (>= 1), WG_ERR_NOWALK when max_walks
 * walks all ended in components of fewer than k vertices, or WG_ERR_ARG.
 */
int64_t wg_walk(const int64_t *row_ptr, const int32_t *col, const int32_t *live, int64_t nlive, int k,
                uint64_t seed, uint64_t stream, int64_t max_walks, int32_t *verts, int32_t *edges, int32_t *m) {
    if (!row_ptr || !col || !live || nlive < 1 || k < 1 || k > 64 || !verts || !edges || !m) return WG_ERR_ARG;
    const uint64_t key = stream_key(seed, stream);
    uint64_t ctr = 0;
    int64_t walks = 0;
    int have = 0;
    while (have < k) {
        if (walks == max_walks) return WG_ERR_NOWALK;
        ++walks;
        int32_t cur = live[below(sm_at(key, ctr++), (uint64_t)nlive)];
        verts[0] = cur;
        have = 1;
        int idle = 0;
        while (have < k && idle < 100 * k) {
            const int64_t d = row_ptr[cur + 1] - row_ptr[cur];
            const int32_t nxt = col[row_ptr[cur] + (int64_t)below(sm_at(key, ctr++), (uint64_t)d)];
            int seen = 0;
            for (int t = 0; t < have; ++t) seen |= verts[t] == nxt;
            if (seen) {
                ++idle;
            } else {
                verts[have++] = nxt;
                idle = 0;
            }
            cur = nxt;
        }
    }
    int32_t cnt = 0;
    for (int x = 0; x < k; ++x)
        for (int y = x + 1; y < k; ++y)
            if (adjacent(row_ptr, col, verts[x], verts[y])) {
                edges[2 * cnt] = x;
                edges[2 * cnt + 1] = y;
                ++cnt;
            }
    *m = cnt;
    return walks;
}
