/*
 * oracle.c -- CPU reference matcher.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the package smoke check and the benchmark's CPU-baseline
 * leg load this library.  The GPU product path never links, loads or calls it,
 * and it shares no code, header or table with that path.
 *
 * What it computes (gMatch paper, arXiv 2604.10601):
 *   - A match is an injective map M: V(Q) -> V(G) that preserves vertex labels
 *     and sends every query edge onto a data edge (Def. 1).  Extra data edges
 *     among the images are allowed (non-induced), and every such map is counted
 *     (no symmetry breaking).
 *   - Query vertices are mapped one at a time along a connected matching order
 *     phi (Sec. 2.2: every vertex after the first has a backward neighbour), by
 *     depth-first search over partial matches (Alg. 1, DFS-Search / Search /
 *     Process).
 *   - The local candidates of the next query vertex u are the neighbours of
 *     M[u'], u' being the backward neighbour of u whose image has the fewest
 *     neighbours (Sec. 4.1, definition of C^L_M(u)).  Among equal degrees the
 *     backward neighbour earliest in phi is taken.
 *   - A candidate v is kept iff L(v) = L(u), d(v) >= d_Q(u) (degree filter,
 *     Sec. 6.1 "Metrics"), v is not already an image, and v is a neighbour of
 *     the image of every other backward neighbour of u, tested by binary search
 *     in the sorted neighbour list (Sec. 5.2, "Time Cost").
 *
 * Work counters, used to check that the GPU explores the same search tree:
 *   groups = number of valid partial matches of length 1..k-1 that were extended
 *            (one task group each, Sec. 4.1),
 *   tasks  = sum of |C^L| over those groups (one task per candidate).
 *
 * Cap and time limit: the reported count is min(#matches, cap).  Outcome is
 * CAPPED when the number of matches found reaches the cap, else TIMEOUT when the
 * time limit expired first (count is then a lower bound), else DONE.
 *
 * Parallelism: plain pthreads; each thread takes the next root vertex (the
 * image of phi[0]) from a shared atomic index and searches its whole subtree.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#include <unistd.h>

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_GRAPH (-2)
#define ORC_ERR_QUERY (-3)
#define ORC_ERR_ORDER (-4)
#define ORC_ERR_NOMEM (-5)

#define ORC_DONE 0
#define ORC_CAPPED 1
#define ORC_TIMEOUT 2

#define ORC_MAX_K 32

typedef struct {
    uint64_t count;
    int32_t outcome;
    int32_t threads;
    uint64_t tasks;
    uint64_t groups;
    uint64_t rows;
    double seconds;
} orc_result;

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static int popcount32(uint32_t x) {
    int c = 0;
    while (x) {
        x &= x - 1;
        c++;
    }
    return c;
}

/* ------------------------------------------------------------------------ */
/* Input checks                                                             */
/* ------------------------------------------------------------------------ */

static int has_edge(const int64_t *row_ptr, const int32_t *col, int32_t a, int32_t b) {
    /* binary search for b in the ascending list N(a) */
    int64_t lo = row_ptr[a], hi = row_ptr[a + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < b)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < row_ptr[a + 1] && col[lo] == b;
}

/* G must be simple and undirected: ascending rows of ids in [0, n), no loops,
 * and (when asked) every edge present in both directions. */
int orc_check_graph(int32_t n, const int64_t *row_ptr, const int32_t *col, int32_t check_symmetry) {
    if (n < 0 || (n > 0 && row_ptr == NULL)) return ORC_ERR_ARG;
    if (n == 0) return ORC_OK;
    if (row_ptr[0] != 0) return ORC_ERR_GRAPH;
    for (int32_t v = 0; v < n; v++)
        if (row_ptr[v + 1] < row_ptr[v]) return ORC_ERR_GRAPH;
    if (row_ptr[n] > 0 && col == NULL) return ORC_ERR_ARG;
    for (int32_t v = 0; v < n; v++) {
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int32_t w = col[e];
            if (w < 0 || w >= n || w == v) return ORC_ERR_GRAPH;
            if (e > row_ptr[v] && col[e - 1] >= w) return ORC_ERR_GRAPH;
        }
    }
    if (check_symmetry) {
        for (int32_t v = 0; v < n; v++)
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
                if (!has_edge(row_ptr, col, col[e], v)) return ORC_ERR_GRAPH;
    }
    return ORC_OK;
}

/* Q must have 1..32 vertices, simple undirected edges and be connected. */
static int build_query_adj(int32_t k, int32_t m, const int32_t *edges, uint32_t adj[ORC_MAX_K]) {
    if (k < 1 || k > ORC_MAX_K || m < 0 || (m > 0 && edges == NULL)) return ORC_ERR_QUERY;
    memset(adj, 0, sizeof(uint32_t) * ORC_MAX_K);
    for (int32_t e = 0; e < m; e++) {
        int32_t a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || a >= k || b < 0 || b >= k || a == b) return ORC_ERR_QUERY;
        if (adj[a] & (1u << b)) return ORC_ERR_QUERY; /* duplicate edge */
        adj[a] |= 1u << b;
        adj[b] |= 1u << a;
    }
    /* connectivity by repeated frontier growth from vertex 0 */
    uint32_t all = (k == 32) ? 0xffffffffu : ((1u << k) - 1u);
    uint32_t reach = 1u, prev = 0;
    while (reach != prev) {
        prev = reach;
        for (int32_t u = 0; u < k; u++)
            if (reach & (1u << u)) reach |= adj[u];
    }
    if (reach != all) return ORC_ERR_QUERY;
    return ORC_OK;
}

int orc_check_query(int32_t k, int32_t m, const int32_t *edges) {
    uint32_t adj[ORC_MAX_K];
    return build_query_adj(k, m, edges, adj);
}

/* An order must be a permutation of 0..k-1 in which every vertex after the first
 * has an earlier neighbour (connected order, Sec. 2.2). */
static int order_ok(int32_t k, const uint32_t adj[ORC_MAX_K], const int32_t *order) {
    uint32_t seen = 0;
    for (int32_t i = 0; i < k; i++) {
        int32_t u = order[i];
        if (u < 0 || u >= k || (seen & (1u << u))) return ORC_ERR_ORDER;
        if (i > 0 && (adj[u] & seen) == 0) return ORC_ERR_ORDER;
        seen |= 1u << u;
    }
    return ORC_OK;
}

int orc_check_order(int32_t k, int32_t m, const int32_t *edges, const int32_t *order) {
    uint32_t adj[ORC_MAX_K];
    int rc = build_query_adj(k, m, edges, adj);
    if (rc) return rc;
    if (order == NULL) return ORC_ERR_ARG;
    return order_ok(k, adj, order);
}

/* ------------------------------------------------------------------------ */
/* Matching order: RI "greatest constraint first" (Bonnici et al., 2013), the */
/* method the paper uses on the CPU (Sec. 3).                                */
/*   first vertex: largest query degree;                                     */
/*   then repeatedly the unordered vertex u maximising, lexicographically,   */
/*     (a) # ordered neighbours of u,                                        */
/*     (b) # ordered vertices adjacent to some unordered neighbour of u,     */
/*     (c) # unordered neighbours of u with no ordered neighbour;            */
/*   ties go to the smallest vertex id.                                      */
/* ------------------------------------------------------------------------ */
int orc_ri_order(int32_t k, int32_t m, const int32_t *edges, int32_t *order_out) {
    uint32_t adj[ORC_MAX_K];
    int rc = build_query_adj(k, m, edges, adj);
    if (rc) return rc;
    if (order_out == NULL) return ORC_ERR_ARG;
    int32_t first = 0;
    for (int32_t u = 1; u < k; u++)
        if (popcount32(adj[u]) > popcount32(adj[first])) first = u;
    uint32_t ordered = 1u << first;
    order_out[0] = first;
    for (int32_t pos = 1; pos < k; pos++) {
        int32_t best = -1;
        int ba = -1, bb = -1, bc = -1;
        for (int32_t u = 0; u < k; u++) {
            if (ordered & (1u << u)) continue;
            uint32_t open_nb = adj[u] & ~ordered;
            int a = popcount32(adj[u] & ordered);
            uint32_t touched = 0;
            int c = 0;
            for (int32_t w = 0; w < k; w++) {
                if (!(open_nb & (1u << w))) continue;
                touched |= adj[w] & ordered;
                if ((adj[w] & ordered) == 0) c++;
            }
            int b = popcount32(touched);
            if (a > ba || (a == ba && (b > bb || (b == bb && c > bc)))) {
                best = u;
                ba = a;
                bb = b;
                bc = c;
            }
        }
        order_out[pos] = best;
        ordered |= 1u << best;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Search                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    /* data graph */
    int32_t n;
    const int64_t *row_ptr;
    const int32_t *col;
    const int32_t *glabels;
    /* query along phi: position i holds phi[i] */
    int32_t k;
    int32_t phi[ORC_MAX_K];
    int32_t lab[ORC_MAX_K];  /* L(phi[i]) */
    int64_t qdeg[ORC_MAX_K]; /* d_Q(phi[i]) */
    uint32_t bwd[ORC_MAX_K]; /* positions j < i adjacent to phi[i] */
    /* limits and shared state */
    uint64_t cap;
    double deadline; /* 0 = none */
    int32_t *rows;
    uint64_t rows_cap;
    _Atomic uint64_t next_root;
    _Atomic uint64_t total;
    _Atomic uint64_t row_cursor;
    _Atomic int stop;
    _Atomic int timed_out;
    _Atomic uint64_t tasks;
    _Atomic uint64_t groups;
} search_ctx;

typedef struct {
    search_ctx *s;
    int32_t M[ORC_MAX_K]; /* M[i] = image of phi[i] */
    uint64_t found;       /* matches not yet added to s->total */
    uint64_t tasks, groups, since_clock;
} worker;

#define FLUSH_EVERY 4096

static void flush_found(worker *w) {
    search_ctx *s = w->s;
    if (w->found == 0) return;
    uint64_t before = atomic_fetch_add(&s->total, w->found);
    if (s->cap && before + w->found >= s->cap) atomic_store(&s->stop, 1);
    w->found = 0;
}

static void emit(worker *w) {
    search_ctx *s = w->s;
    if (s->rows) {
        uint64_t slot = atomic_fetch_add(&s->row_cursor, 1);
        if (slot < s->rows_cap)
            for (int32_t i = 0; i < s->k; i++) s->rows[slot * (uint64_t)s->k + (uint64_t)s->phi[i]] = w->M[i];
    }
    w->found++;
    if (w->found >= FLUSH_EVERY || (s->cap && w->found >= s->cap)) flush_found(w);
}

static int64_t degree(const search_ctx *s, int32_t v) { return s->row_ptr[v + 1] - s->row_ptr[v]; }

static void extend(worker *w, int32_t i) {
    search_ctx *s = w->s;
    if (atomic_load_explicit(&s->stop, memory_order_relaxed)) return;
    if (i == s->k) {
        emit(w);
        return;
    }
    /* i >= 1: one task group; its local candidates are N(M[jstar]) */
    int32_t jstar = -1;
    int64_t best = 0;
    for (int32_t j = 0; j < i; j++) {
        if (!(s->bwd[i] & (1u << j))) continue;
        int64_t d = degree(s, w->M[j]);
        if (jstar < 0 || d < best) {
            jstar = j;
            best = d;
        }
    }
    w->groups++;
    w->tasks += (uint64_t)best;
    w->since_clock += (uint64_t)best + 1;
    if (s->deadline > 0 && w->since_clock >= 65536) {
        w->since_clock = 0;
        if (now_s() > s->deadline) {
            atomic_store(&s->timed_out, 1);
            atomic_store(&s->stop, 1);
            return;
        }
    }
    const int32_t *cand = s->col + s->row_ptr[w->M[jstar]];
    for (int64_t t = 0; t < best; t++) {
        int32_t v = cand[t];
        if (s->glabels[v] != s->lab[i]) continue;
        if (degree(s, v) < s->qdeg[i]) continue;
        int ok = 1;
        for (int32_t j = 0; j < i && ok; j++) {
            if (w->M[j] == v)
                ok = 0;
            else if (j != jstar && (s->bwd[i] & (1u << j)) && !has_edge(s->row_ptr, s->col, w->M[j], v))
                ok = 0;
        }
        if (!ok) continue;
        w->M[i] = v;
        extend(w, i + 1);
        if (atomic_load_explicit(&s->stop, memory_order_relaxed)) return;
    }
}

static void *worker_main(void *arg) {
    worker *w = (worker *)arg;
    search_ctx *s = w->s;
    for (;;) {
        if (atomic_load_explicit(&s->stop, memory_order_relaxed)) break;
        uint64_t r = atomic_fetch_add(&s->next_root, 1);
        if (r >= (uint64_t)s->n) break;
        int32_t v = (int32_t)r;
        if (s->deadline > 0 && (r & 255) == 0 && now_s() > s->deadline) {
            atomic_store(&s->timed_out, 1);
            atomic_store(&s->stop, 1);
            break;
        }
        /* position 0 has no backward neighbour: every vertex is a candidate */
        if (s->glabels[v] != s->lab[0] || degree(s, v) < s->qdeg[0]) continue;
        w->M[0] = v;
        extend(w, 1);
    }
    flush_found(w);
    atomic_fetch_add(&s->tasks, w->tasks);
    atomic_fetch_add(&s->groups, w->groups);
    return NULL;
}

/*
 * Count (and optionally list) all matches of Q in G.
 *   G: n vertices, CSR row_ptr[n+1] / col[row_ptr[n]] (ascending rows), glabels[n].
 *   Q: k vertices, m edges (edges[2e], edges[2e+1]), qlabels[k].
 *   order: phi as k query-vertex ids, or NULL for the RI order above.
 *   cap: 0 = none.  time_limit_s <= 0: none.  nthreads <= 0: all online CPUs.
 *   rows: NULL, or room for rows_cap rows of k int32; row r holds the image of
 *         query vertex 0..k-1 of the r-th match found (in no particular order).
 * The graph is assumed checked (orc_check_graph); Q and the order are checked here.
 */
int orc_match(int32_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *glabels, int32_t k,
              int32_t m, const int32_t *edges, const int32_t *qlabels, const int32_t *order, uint64_t cap,
              double time_limit_s, int32_t nthreads, int32_t *rows, uint64_t rows_cap, orc_result *out) {
    if (out == NULL || n < 0 || qlabels == NULL) return ORC_ERR_ARG;
    if (n > 0 && (row_ptr == NULL || glabels == NULL)) return ORC_ERR_ARG;
    memset(out, 0, sizeof(*out));
    uint32_t adj[ORC_MAX_K];
    int rc = build_query_adj(k, m, edges, adj);
    if (rc) return rc;
    int32_t phi[ORC_MAX_K];
    if (order) {
        rc = order_ok(k, adj, order);
        if (rc) return rc;
        memcpy(phi, order, sizeof(int32_t) * (size_t)k);
    } else {
        orc_ri_order(k, m, edges, phi);
    }
    search_ctx *s = (search_ctx *)calloc(1, sizeof(search_ctx));
    if (!s) return ORC_ERR_NOMEM;
    s->n = n;
    s->row_ptr = row_ptr;
    s->col = col;
    s->glabels = glabels;
    s->k = k;
    for (int32_t i = 0; i < k; i++) {
        s->phi[i] = phi[i];
        s->lab[i] = qlabels[phi[i]];
        s->qdeg[i] = popcount32(adj[phi[i]]);
        uint32_t b = 0;
        for (int32_t j = 0; j < i; j++)
            if (adj[phi[i]] & (1u << phi[j])) b |= 1u << j;
        s->bwd[i] = b;
    }
    s->cap = cap;
    s->rows = rows;
    s->rows_cap = rows ? rows_cap : 0;
    double t0 = now_s();
    s->deadline = time_limit_s > 0 ? t0 + time_limit_s : 0;
    if (nthreads <= 0) nthreads = (int32_t)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    worker *ws = (worker *)calloc((size_t)nthreads, sizeof(worker));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!ws || !th) {
        free(ws);
        free(th);
        free(s);
        return ORC_ERR_NOMEM;
    }
    int started = 0;
    for (int32_t t = 0; t < nthreads; t++) {
        ws[t].s = s;
        if (t == 0) continue; /* thread 0 is the caller */
        if (pthread_create(&th[t], NULL, worker_main, &ws[t]) == 0) started++;
        else break;
    }
    worker_main(&ws[0]);
    for (int32_t t = 1; t <= started; t++) pthread_join(th[t], NULL);
    uint64_t total = atomic_load(&s->total);
    out->seconds = now_s() - t0;
    out->threads = started + 1;
    out->tasks = atomic_load(&s->tasks);
    out->groups = atomic_load(&s->groups);
    if (cap && total >= cap) {
        out->count = cap;
        out->outcome = ORC_CAPPED;
    } else {
        out->count = total;
        out->outcome = atomic_load(&s->timed_out) ? ORC_TIMEOUT : ORC_DONE;
    }
    uint64_t rc_rows = atomic_load(&s->row_cursor);
    out->rows = rc_rows < s->rows_cap ? rc_rows : s->rows_cap;
    free(ws);
    free(th);
    free(s);
    return ORC_OK;
}
