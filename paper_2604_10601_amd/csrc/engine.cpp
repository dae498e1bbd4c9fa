// Host side of the C ABI declared in include/gmatch.h: input checks, the
// matching-order plan, device buffers and the launch sequence of one search
// (root candidates -> breadth-first pool up to tau -> persistent depth-first
// search), following Alg. 2 of the gMatch paper.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gm_internal.h"
#include "gmatch.h"

using gm::Control;
using gm::kMaxK;
using gm::Plan;
using gm::SearchArgs;
using gm::VInfo;

namespace {

thread_local std::string g_create_error;

// Hub bitmaps: vertices with at least this many neighbours, at most this many, in this many bytes.
constexpr int64_t kHubMinDegree = 256;
constexpr int32_t kMaxHubs = 4096;
constexpr int32_t kHubDefaultMiB = 1024;

struct QueryRec {
    bool live = false;
    int32_t k = 0;
    int32_t split = 0;  // task split of the two-phase pool (position-1 tasks kept with a root); 0 = engine's
    std::vector<int32_t> labels;
    uint32_t adj[kMaxK] = {};
    std::vector<int32_t> order;
    // symmetry breaking (opt-in): bit u of less[v] requires M(v) < M(u)
    bool sb = false;
    uint32_t less[kMaxK] = {};
    uint64_t aut = 1;  // |Aut(Q)| (saturating)
};

// Is there an automorphism of q (a permutation of its vertices preserving
// labels and edges) that fixes every vertex in `fixed` and maps v to u?
// Depth-first over the vertices in breadth-first order from v; `budget` bounds
// the nodes searched (false with budget exhausted when it runs out).
bool automorphism_exists(const QueryRec &q, uint32_t fixed, int32_t v, int32_t u, long long &budget) {
    const int32_t k = q.k;
    int32_t seq[kMaxK], n = 0;
    uint32_t seen = 1u << v;
    seq[n++] = v;
    for (int32_t h = 0; h < n; ++h)
        for (uint32_t m = q.adj[seq[h]] & ~seen; m; m &= m - 1) {
            seen |= 1u << __builtin_ctz(m);
            seq[n++] = __builtin_ctz(m);
        }
    for (int32_t x = 0; x < k; ++x)
        if (!((seen >> x) & 1u)) seq[n++] = x;  // (q is connected: not reached)
    int32_t img[kMaxK];
    for (int32_t x = 0; x < k; ++x) img[x] = -1;
    uint32_t used = 0;
    auto fits = [&](int32_t x, int32_t y) {
        if ((used >> y) & 1u) return false;
        if (q.labels[x] != q.labels[y] || __builtin_popcount(q.adj[x]) != __builtin_popcount(q.adj[y])) return false;
        if (((fixed >> x) & 1u) && x != y) return false;
        if (((fixed >> y) & 1u) && x != y) return false;
        for (int32_t z = 0; z < k; ++z)
            if (img[z] >= 0 && (((q.adj[x] >> z) & 1u) != ((q.adj[y] >> img[z]) & 1u))) return false;
        return true;
    };
    std::function<bool(int32_t)> go = [&](int32_t i) -> bool {
        if (i == k) return true;
        if (--budget < 0) return false;
        const int32_t x = seq[i];
        for (int32_t y = (i == 0 ? u : 0); y < (i == 0 ? u + 1 : k); ++y) {
            if (!fits(x, y)) continue;
            img[x] = y;
            used |= 1u << y;
            if (go(i + 1)) return true;
            img[x] = -1;
            used &= ~(1u << y);
            if (budget < 0) return false;
        }
        return false;
    };
    return go(0);
}

// Symmetry-breaking conditions along a stabilizer chain (Grochow and Kellis
// 2007): while the group fixing the chosen vertices is not trivial, take the
// vertex with the largest orbit under it (the smallest id on ties), require it
// to map below every other vertex of that orbit, and fix it.  Exactly one map
// of every class {M o a : a in Aut(Q)} meets all conditions, and |Aut(Q)| is
// the product of the orbit sizes.  Returns false if the search budget ran out.
bool symmetry_conditions(QueryRec &q) {
    long long budget = 20000000;
    std::fill(q.less, q.less + kMaxK, 0u);
    q.aut = 1;
    uint32_t fixed = 0;
    for (;;) {
        int32_t best = -1;
        uint32_t best_orbit = 0;
        for (int32_t v = 0; v < q.k; ++v) {
            if ((fixed >> v) & 1u) continue;
            uint32_t orbit = 1u << v;
            for (int32_t u = 0; u < q.k; ++u) {
                if (u == v || ((fixed >> u) & 1u)) continue;
                if (automorphism_exists(q, fixed, v, u, budget)) orbit |= 1u << u;
                if (budget < 0) return false;
            }
            if (best < 0 || __builtin_popcount(orbit) > __builtin_popcount(best_orbit)) {
                best = v;
                best_orbit = orbit;
            }
        }
        if (best < 0 || __builtin_popcount(best_orbit) == 1) return true;
        q.less[best] |= best_orbit & ~(1u << best);
        const uint64_t o = static_cast<uint64_t>(__builtin_popcount(best_orbit));
        q.aut = q.aut > UINT64_MAX / o ? UINT64_MAX : q.aut * o;
        fixed |= 1u << best;
    }
}

int popcount(uint32_t x) { return __builtin_popcount(x); }

// RI "greatest constraint first" order (Bonnici et al. 2013; the paper builds
// its order with RI on the CPU, Sec. 3).  Start at the largest degree; then
// repeatedly the unordered vertex with the lexicographically largest
// (#ordered neighbours, #ordered vertices next to one of its unordered
// neighbours, #unordered neighbours with no ordered neighbour); ties -> smaller id.
std::vector<int32_t> ri_order(int32_t k, const uint32_t *adj) {
    std::vector<int32_t> order;
    order.reserve(k);
    int32_t start = 0;
    for (int32_t u = 0; u < k; ++u)
        if (popcount(adj[u]) > popcount(adj[start])) start = u;
    uint32_t placed = 1u << start;
    order.push_back(start);
    while (static_cast<int32_t>(order.size()) < k) {
        long best_key = -1;
        int32_t best_u = -1;
        for (int32_t u = 0; u < k; ++u) {
            if (placed & (1u << u)) continue;
            const uint32_t outside = adj[u] & ~placed;
            uint32_t reached = 0;
            int free_nb = 0;
            for (uint32_t m = outside; m; m &= m - 1) {
                const int w = __builtin_ctz(m);
                reached |= adj[w] & placed;
                free_nb += (adj[w] & placed) == 0;
            }
            // three fields of at most 32 each, packed so larger means better
            const long key = (static_cast<long>(popcount(adj[u] & placed)) << 16) |
                             (static_cast<long>(popcount(reached)) << 8) | free_nb;
            if (key > best_key) {
                best_key = key;
                best_u = u;
            }
        }
        placed |= 1u << best_u;
        order.push_back(best_u);
    }
    return order;
}

bool connected_order(int32_t k, const uint32_t *adj, const int32_t *order) {
    uint32_t seen = 0;
    for (int32_t i = 0; i < k; ++i) {
        const int32_t u = order[i];
        if (u < 0 || u >= k || (seen >> u) & 1u) return false;
        if (i > 0 && (adj[u] & seen) == 0) return false;
        seen |= 1u << u;
    }
    return true;
}

// Runs f(begin, end) over [0, n) on the host's cores.
template <class F>
void parallel_ranges(int64_t n, F f) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t parts = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 4, n / 65536 + 1));
    std::vector<std::thread> th;
    const int64_t chunk = (n + parts - 1) / parts;
    for (int64_t p = 1; p < parts; ++p) {
        const int64_t b = p * chunk, e = std::min(n, b + chunk);
        if (b < e) th.emplace_back(f, b, e);
    }
    f(0, std::min(n, chunk));
    for (auto &t : th) t.join();
}

}  // namespace

// Device state of one persistent launch in flight: its HIP stream and events,
// the control block, per-query plans and result blocks, work-item streams and
// the stealing mailboxes.  The engine has one for its own calls; a server has
// one per slot, so several launches can run at once.
struct LaunchCtx {
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    Control *d_ctl = nullptr;
    Plan *d_plans = nullptr;       // per-query plans of a launch
    gm::QCtl *d_qctl = nullptr;    // per-query results of a launch
    size_t plans_cap = 0;
    gm::StreamCtl *d_streams = nullptr;  // work-item streams of a launch
    size_t streams_cap = 0;
    gm::Mailbox *d_mail = nullptr;
    unsigned long long *d_idle_bits = nullptr;
    int32_t steal_slots = 0;
    uint2 *d_parked = nullptr;     // parked task groups of the wavefronts (levels x 64 per wavefront)
    size_t parked_cap = 0;         // in entries
    std::vector<Plan> h_plans;     // host copies (kept until the uploads complete)
    std::vector<gm::QCtl> h_qctl;
    std::vector<gm::StreamCtl> h_streams;
};

struct gm_engine {
    int32_t device = -1;
    gm_options opt{};
    mutable std::mutex mu;
    mutable std::string err;

    bool has_graph = false;
    int32_t n = 0;
    uint64_t nnz = 0;
    VInfo *d_vinfo = nullptr;
    int32_t *d_col = nullptr;
    bool col_owned = true;         // false: the caller's device buffer (gm_load_graph_device)
    int32_t *d_lcol = nullptr;     // lists ordered by (label, id); aliases d_col when not partitioned
    uint32_t *d_loff = nullptr;    // label slice bounds
    int32_t loff_stride = 1;
    std::unordered_map<int32_t, int32_t> label_id;  // G's label value -> compact id
    // vertices grouped by label, by degree descending within a label: the
    // candidates of a first query vertex are a prefix of its label's bucket
    int32_t *d_bylabel = nullptr;
    int32_t *d_hub_id = nullptr;          // adjacency bitmaps of the highest-degree vertices
    uint32_t *d_hub_bits = nullptr;
    uint64_t hub_words = 0;
    int32_t hubs = 0;
    std::vector<int64_t> lab_start;       // [labels + 1] bucket bounds
    std::vector<uint32_t> bylabel_deg;    // degree of each bucket entry (host copy)

    std::vector<QueryRec> queries;

    int32_t *d_pool[2] = {nullptr, nullptr};
    size_t pool_cap[2] = {0, 0};  // in int32
    int32_t *d_rows = nullptr;
    size_t rows_cap = 0;           // in int32
    uint32_t *d_vlen = nullptr;    // virtual level-1 pool: slice length, start and first task per root
    uint32_t *d_vstart = nullptr;
    uint32_t *d_voff = nullptr;
    uint32_t *d_vtmp = nullptr;    // chunk totals of the prefix sum
    size_t v_cap = 0;
    // candidate graph of the query searched last (built per call, buffers kept)
    int32_t *d_cbits = nullptr;    // C(l) bitmaps by position
    int32_t *d_crank = nullptr;    // scratch: word ranks, then list lengths and offsets
    int32_t *d_ctmp = nullptr;     // prefix-sum scratch
    int32_t *d_clist = nullptr;    // candidates of every position, ids ascending
    int32_t *d_cedges = nullptr;   // per query edge: gm::CandEdge
    int32_t *d_gbounds = nullptr;  // list bounds per query edge and candidate
    int32_t *d_gcol = nullptr;     // the lists
    int32_t *d_cmisc = nullptr;    // [0..3] sweep flags, [4..5] list total, [8 ..] position bounds
    size_t cbits_cap = 0, crank_cap = 0, ctmp_cap = 0, clist_cap = 0, cedges_cap = 0, gbounds_cap = 0, gcol_cap = 0,
           cmisc_cap = 0;
    std::vector<gm::CandEdge> h_cedges;
    LaunchCtx lc;                  // device state of the engine's own launches
    void *scratch = nullptr;       // this device's arena for gm_count_noalloc (shared by its engines)
    std::atomic<int> servers{0};   // open servers (the graph must stay as it is)
    int num_cu = 0;
    long long wall_khz = 0;

    // the message of the last failure; a server's worker thread may set it too
    mutable std::mutex err_mu;
    gm_status fail(gm_status s, const std::string &msg) const {
        std::lock_guard<std::mutex> lk(err_mu);
        err = msg;
        return s;
    }
    std::string last_error() const {
        std::lock_guard<std::mutex> lk(err_mu);
        return err;
    }
};

namespace {

// Stream, events and control block of a launch context (the rest is allocated on first use).
hipError_t ctx_create(LaunchCtx &c) {
    hipError_t h = hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking);
    if (h == hipSuccess) h = hipEventCreate(&c.ev0);
    if (h == hipSuccess) h = hipEventCreate(&c.ev1);
    if (h == hipSuccess) h = hipMalloc(reinterpret_cast<void **>(&c.d_ctl), sizeof(Control));
    return h;
}

// Waits for the context's work and frees everything it holds.
void ctx_destroy(LaunchCtx &c) {
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    for (void *b : {static_cast<void *>(c.d_ctl), static_cast<void *>(c.d_plans), static_cast<void *>(c.d_qctl),
                    static_cast<void *>(c.d_streams), static_cast<void *>(c.d_mail), static_cast<void *>(c.d_idle_bits),
                    static_cast<void *>(c.d_parked)})
        if (b) (void)hipFree(b);
    if (c.ev0) (void)hipEventDestroy(c.ev0);
    if (c.ev1) (void)hipEventDestroy(c.ev1);
    if (c.stream) (void)hipStreamDestroy(c.stream);
    c = LaunchCtx{};
}

gm_status hip_fail(const gm_engine *e, hipError_t h, const char *what) {
    return e->fail(GM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(h));
}

#define HIP_TRY(e, call)                                  \
    do {                                                  \
        hipError_t h_ = (call);                           \
        if (h_ != hipSuccess) return hip_fail(e, h_, #call); \
    } while (0)

gm_status ensure_buffer(gm_engine *e, int32_t **buf, size_t *cap, size_t need_ints) {
    if (need_ints <= *cap && *buf) return GM_OK;
    if (*buf) {
        (void)hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    size_t want = std::max<size_t>(need_ints, 1024);
    want += want / 4;
    hipError_t h = hipMalloc(reinterpret_cast<void **>(buf), want * sizeof(int32_t));
    if (h != hipSuccess) {
        *buf = nullptr;
        // retry without slack
        want = std::max<size_t>(need_ints, 1);
        h = hipMalloc(reinterpret_cast<void **>(buf), want * sizeof(int32_t));
        if (h != hipSuccess) {
            *buf = nullptr;
            return e->fail(GM_ERR_NOMEM, "device allocation of " + std::to_string(want * 4) + " bytes failed");
        }
    }
    *cap = want;
    return GM_OK;
}

// Room for the virtual level-1 pool of up to R roots.
gm_status ensure_level1(gm_engine *e, size_t R) {
    if (R <= e->v_cap && e->d_voff) return GM_OK;
    uint32_t **bufs[] = {&e->d_vlen, &e->d_vstart, &e->d_voff, &e->d_vtmp};
    for (uint32_t **b : bufs) {
        if (*b) (void)hipFree(*b);
        *b = nullptr;
    }
    e->v_cap = 0;
    const size_t want = std::max<size_t>(R, 4096);
    hipError_t h = hipSuccess;
    for (int i = 0; i < 3 && h == hipSuccess; ++i) h = hipMalloc(reinterpret_cast<void **>(bufs[i]), want * 4);
    if (h == hipSuccess) h = hipMalloc(reinterpret_cast<void **>(&e->d_vtmp), (want / 4096 + 2) * 4);
    if (h != hipSuccess) {
        for (uint32_t **b : bufs) {
            if (*b) (void)hipFree(*b);
            *b = nullptr;
        }
        return e->fail(GM_ERR_NOMEM, "device allocation of the level-1 pool failed");
    }
    e->v_cap = want;
    return GM_OK;
}

// Room for ns work-item streams on the device.
gm_status ensure_streams(gm_engine *e, LaunchCtx &c, size_t ns) {
    if (ns <= c.streams_cap && c.d_streams) return GM_OK;
    if (c.d_streams) (void)hipFree(c.d_streams);
    c.d_streams = nullptr;
    c.streams_cap = 0;
    const size_t want = std::max<size_t>(ns, 64);
    if (hipMalloc(reinterpret_cast<void **>(&c.d_streams), want * sizeof(gm::StreamCtl)) != hipSuccess) {
        c.d_streams = nullptr;
        return e->fail(GM_ERR_NOMEM, "device allocation of work streams failed");
    }
    c.streams_cap = want;
    return GM_OK;
}

// Room for nq plans and per-query result blocks on the device.
gm_status ensure_query_slots(gm_engine *e, LaunchCtx &c, size_t nq) {
    if (nq <= c.plans_cap && c.d_plans && c.d_qctl) return GM_OK;
    if (c.d_plans) (void)hipFree(c.d_plans);
    if (c.d_qctl) (void)hipFree(c.d_qctl);
    c.d_plans = nullptr;
    c.d_qctl = nullptr;
    c.plans_cap = 0;
    const size_t want = std::max<size_t>(nq, 64);
    hipError_t h = hipMalloc(reinterpret_cast<void **>(&c.d_plans), want * sizeof(Plan));
    if (h == hipSuccess) h = hipMalloc(reinterpret_cast<void **>(&c.d_qctl), want * sizeof(gm::QCtl));
    if (h != hipSuccess) {
        if (c.d_plans) (void)hipFree(c.d_plans);
        c.d_plans = nullptr;
        c.d_qctl = nullptr;
        return e->fail(GM_ERR_NOMEM, "device allocation of query plans failed");
    }
    c.plans_cap = want;
    return GM_OK;
}

void free_graph(gm_engine *e) {
    if (e->d_vinfo) (void)hipFree(e->d_vinfo);
    if (e->d_lcol && e->d_lcol != e->d_col) (void)hipFree(e->d_lcol);
    if (e->d_col && e->col_owned) (void)hipFree(e->d_col);
    e->col_owned = true;
    if (e->d_loff) (void)hipFree(e->d_loff);
    if (e->d_bylabel) (void)hipFree(e->d_bylabel);
    if (e->d_hub_id) (void)hipFree(e->d_hub_id);
    if (e->d_hub_bits) (void)hipFree(e->d_hub_bits);
    e->d_bylabel = nullptr;
    e->d_hub_id = nullptr;
    e->d_hub_bits = nullptr;
    e->hub_words = 0;
    e->hubs = 0;
    e->lab_start.clear();
    e->bylabel_deg.clear();
    e->d_vinfo = nullptr;
    e->d_col = nullptr;
    e->d_lcol = nullptr;
    e->d_loff = nullptr;
    e->loff_stride = 1;
    e->has_graph = false;
    e->n = 0;
    e->nnz = 0;
    e->label_id.clear();
}

// Stack layout: the option, else slim (measured faster at 8 and at 12-32 vertices).
// A slim stack entry holds a vertex id in 24 bits, so larger graphs use the full one.
constexpr int32_t kSlimMaxVertices = 1 << 24;
bool use_slim(const gm_engine *e, int32_t k) {
    (void)k;
    return e->opt.stack_layout != 1 && e->n <= kSlimMaxVertices;
}



gm_status check_graph(gm_engine *e, int32_t n, const int64_t *row_ptr, const int32_t *col, bool symmetric) {
    if (row_ptr[0] != 0) return e->fail(GM_ERR_GRAPH, "row_ptr[0] must be 0");
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return e->fail(GM_ERR_GRAPH, "row_ptr must be non-decreasing");
    const int64_t nnz = row_ptr[n];
    if (nnz >= (int64_t(1) << 32)) return e->fail(GM_ERR_GRAPH, "more than 2^32 - 1 adjacency entries");
    if (nnz > 0 && col == nullptr) return e->fail(GM_ERR_ARG, "col is null");
    std::atomic<int> bad{0};  // 1 order/range/loop, 2 degree limit, 3 symmetry
    parallel_ranges(n, [&](int64_t b, int64_t end) {
        for (int64_t v = b; v < end && !bad.load(std::memory_order_relaxed); ++v) {
            const int64_t lo = row_ptr[v], hi = row_ptr[v + 1];
            if (hi - lo >= (int64_t(1) << 24)) {
                bad = 2;
                return;
            }
            for (int64_t p = lo; p < hi; ++p) {
                const int32_t w = col[p];
                if (w < 0 || w >= n || w == v || (p > lo && col[p - 1] >= w)) {
                    bad = 1;
                    return;
                }
            }
        }
    });
    if (bad == 1) return e->fail(GM_ERR_GRAPH, "adjacency rows must be strictly ascending ids in [0, n) without self-loops");
    if (bad == 2) return e->fail(GM_ERR_GRAPH, "a vertex degree exceeds 2^24 - 1");
    if (symmetric) {
        parallel_ranges(n, [&](int64_t b, int64_t end) {
            for (int64_t v = b; v < end && !bad.load(std::memory_order_relaxed); ++v) {
                for (int64_t p = row_ptr[v]; p < row_ptr[v + 1]; ++p) {
                    const int32_t w = col[p];
                    if (!std::binary_search(col + row_ptr[w], col + row_ptr[w + 1], static_cast<int32_t>(v))) {
                        bad = 3;
                        return;
                    }
                }
            }
        });
        if (bad == 3) return e->fail(GM_ERR_GRAPH, "graph is not symmetric (an edge is stored in one direction only)");
    }
    return GM_OK;
}

// Host-side description of a graph being loaded: sizes, degrees, compact label
// ids and the map from G's label values to them.
struct HostGraph {
    int32_t n = 0;
    uint64_t nnz = 0;
    std::vector<uint32_t> deg;   // [n]
    std::vector<uint8_t> clab;   // [n]
    int32_t labels_used = 0;
    std::unordered_map<int32_t, int32_t> ids;
};

// G's label values -> compact ids 0 .. labels_used - 1 in ascending value order.
gm_status compact_labels(gm_engine *e, const int32_t *labels, int32_t n, HostGraph &hg) {
    hg.clab.resize(static_cast<size_t>(n));
    if (n == 0) return GM_OK;
    int32_t lo = labels[0], hi = labels[0];
    for (int32_t v = 1; v < n; ++v) {
        lo = std::min(lo, labels[v]);
        hi = std::max(hi, labels[v]);
    }
    std::vector<int32_t> values;
    if (static_cast<int64_t>(hi) - lo < (int64_t(1) << 20)) {
        std::vector<int32_t> id(static_cast<size_t>(static_cast<int64_t>(hi) - lo + 1), -1);
        for (int32_t v = 0; v < n; ++v) id[labels[v] - lo] = 0;
        int32_t used = 0;
        for (size_t i = 0; i < id.size(); ++i)
            if (id[i] == 0) {
                if (used >= 255) return e->fail(GM_ERR_GRAPH, "more than 255 distinct vertex labels");
                id[i] = used++;
                hg.ids.emplace(static_cast<int32_t>(lo + static_cast<int64_t>(i)), id[i]);
            }
        parallel_ranges(n, [&](int64_t b, int64_t en) {
            for (int64_t v = b; v < en; ++v) hg.clab[v] = static_cast<uint8_t>(id[labels[v] - lo]);
        });
        hg.labels_used = used;
        return GM_OK;
    }
    std::unordered_map<int32_t, int32_t> seen;
    for (int32_t v = 0; v < n; ++v) {
        if (seen.emplace(labels[v], 0).second && seen.size() > 255)
            return e->fail(GM_ERR_GRAPH, "more than 255 distinct vertex labels");
    }
    for (auto &kv : seen) values.push_back(kv.first);
    std::sort(values.begin(), values.end());
    for (size_t i = 0; i < values.size(); ++i) hg.ids[values[i]] = static_cast<int32_t>(i);
    for (int32_t v = 0; v < n; ++v) hg.clab[v] = static_cast<uint8_t>(hg.ids[labels[v]]);
    hg.labels_used = static_cast<int32_t>(values.size());
    return GM_OK;
}

// Label-partitioned lists need (labels + 1) bounds per vertex; they are skipped
// when asked, when there is one label, or when the table would exceed 8 GiB.
int32_t slice_stride(const gm_engine *e, int32_t n, int32_t labels_used) {
    const int32_t stride = labels_used + 1;
    if (e->opt.disable_label_index || labels_used <= 1 ||
        static_cast<uint64_t>(n) * static_cast<uint64_t>(stride) * 4ull > (8ull << 30))
        return 1;
    return stride;
}

// Vertices grouped by label, highest degree first within a label, ties by id
// (two stable counting sorts), and all vertices by degree (highest first).
void order_vertices(const HostGraph &hg, std::vector<int64_t> &lab_start, std::vector<int32_t> &bylabel,
                    std::vector<uint32_t> &bylabel_deg, std::vector<int32_t> &by_degree) {
    const int32_t n = hg.n;
    uint32_t maxd = 0;
    for (int32_t v = 0; v < n; ++v) maxd = std::max(maxd, hg.deg[v]);
    std::vector<int64_t> at(static_cast<size_t>(maxd) + 2, 0);
    for (int32_t v = 0; v < n; ++v) ++at[maxd - hg.deg[v] + 1];  // bucket 0 = the largest degree
    for (size_t i = 1; i < at.size(); ++i) at[i] += at[i - 1];
    by_degree.assign(static_cast<size_t>(n), 0);
    for (int32_t v = 0; v < n; ++v) by_degree[at[maxd - hg.deg[v]]++] = v;
    lab_start.assign(static_cast<size_t>(hg.labels_used) + 1, 0);
    for (int32_t v = 0; v < n; ++v) ++lab_start[hg.clab[v] + 1];
    for (int32_t c = 0; c < hg.labels_used; ++c) lab_start[c + 1] += lab_start[c];
    std::vector<int64_t> fill(lab_start.begin(), lab_start.end() - 1);
    bylabel.assign(static_cast<size_t>(n), 0);
    bylabel_deg.assign(static_cast<size_t>(n), 0);
    for (int32_t v : by_degree) {
        const int64_t pos = fill[hg.clab[v]]++;
        bylabel[pos] = v;
        bylabel_deg[pos] = hg.deg[v];
    }
}

gm_status install_host_only(gm_engine *e, HostGraph &hg) {
    std::vector<int64_t> lab_start;
    std::vector<int32_t> bylabel, by_degree;
    std::vector<uint32_t> bylabel_deg;
    order_vertices(hg, lab_start, bylabel, bylabel_deg, by_degree);
    free_graph(e);
    e->loff_stride = slice_stride(e, hg.n, hg.labels_used);
    e->label_id = std::move(hg.ids);
    e->lab_start = std::move(lab_start);
    e->bylabel_deg = std::move(bylabel_deg);
    e->n = hg.n;
    e->nnz = hg.nnz;
    e->has_graph = true;
    return GM_OK;
}

// Is p device memory of the engine's device?
bool device_buffer(const gm_engine *e, const void *p) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice && at.device == e->device;
}

// Checks the graph on the device and builds every derived structure there:
// vertex records, label slices, the vertex order by label and degree, hub
// bitmaps.  d_row_ptr, d_col and d_clab are device arrays; d_col becomes the
// engine's adjacency array (freed with the graph when col_owned, and freed here
// on failure).  On success the previous graph is released and replaced.
gm_status install_device(gm_engine *e, HostGraph &hg, const void *d_row_ptr, int rp_bytes, int32_t *d_col,
                         bool col_owned, const uint8_t *d_clab, hipStream_t s) {
    const int32_t n = hg.n;
    VInfo *vinfo = nullptr;
    uint32_t *loff = nullptr;
    int32_t *lcol = nullptr, *bylabel_d = nullptr, *hub_id = nullptr, *hub_list = nullptr;
    uint32_t *hub_bits = nullptr;
    unsigned int *d_err = nullptr;
    auto release = [&](bool all) {
        if (d_err) (void)hipFree(d_err);
        if (hub_list) (void)hipFree(hub_list);
        d_err = nullptr;
        hub_list = nullptr;
        if (!all) return;
        for (void *p : {static_cast<void *>(vinfo), static_cast<void *>(loff), static_cast<void *>(lcol),
                        static_cast<void *>(bylabel_d), static_cast<void *>(hub_id), static_cast<void *>(hub_bits)})
            if (p) (void)hipFree(p);
        if (col_owned && d_col) (void)hipFree(d_col);
    };
    auto device_error = [&](hipError_t h, const char *what) {
        (void)hipStreamSynchronize(s);
        release(true);
        return e->fail(h == hipErrorOutOfMemory ? GM_ERR_NOMEM : GM_ERR_DEVICE,
                       std::string("graph load, ") + what + ": " + hipGetErrorString(h));
    };
    // 1. checks: offsets first (they bound every row the second pass reads)
    hipError_t h = hipMalloc(reinterpret_cast<void **>(&d_err), sizeof(unsigned int));
    unsigned int err = 0;
    for (int pass = 0; pass < 2 && h == hipSuccess && err == 0; ++pass) {
        h = hipMemsetAsync(d_err, 0, sizeof(unsigned int), s);
        if (h == hipSuccess)
            h = gm::launch_graph_check(d_row_ptr, rp_bytes, d_col, n, e->opt.skip_symmetry_check == 0, d_err, pass == 1,
                                       e->num_cu, s);
        if (h == hipSuccess) h = hipMemcpyAsync(&err, d_err, sizeof(err), hipMemcpyDeviceToHost, s);
        if (h == hipSuccess) h = hipStreamSynchronize(s);
    }
    if (h != hipSuccess) return device_error(h, "check");
    if (err) {
        release(true);
        if (err & gm::kGraphBadRowPtr) return e->fail(GM_ERR_GRAPH, "row_ptr must start at 0 and be non-decreasing");
        if (err & gm::kGraphBadDegree) return e->fail(GM_ERR_GRAPH, "a vertex degree exceeds 2^24 - 1");
        if (err & gm::kGraphBadEntry)
            return e->fail(GM_ERR_GRAPH, "adjacency rows must be strictly ascending ids in [0, n) without self-loops");
        return e->fail(GM_ERR_GRAPH, "graph is not symmetric (an edge is stored in one direction only)");
    }
    // 2. vertex records and label slices
    const int32_t stride = slice_stride(e, n, hg.labels_used);
    const size_t loff_len = stride > 1 ? static_cast<size_t>(n) * stride : static_cast<size_t>(n) + 1;
    h = hipMalloc(reinterpret_cast<void **>(&vinfo), std::max<size_t>(n, 1) * sizeof(VInfo));
    if (h == hipSuccess) h = hipMalloc(reinterpret_cast<void **>(&loff), std::max<size_t>(loff_len, 1) * sizeof(uint32_t));
    if (h == hipSuccess && stride > 1)
        h = hipMalloc(reinterpret_cast<void **>(&lcol), std::max<uint64_t>(hg.nnz, gm::kListWindow) * sizeof(int32_t));
    if (h == hipSuccess) h = hipMalloc(reinterpret_cast<void **>(&bylabel_d), std::max<size_t>(n, 1) * sizeof(int32_t));
    if (h == hipSuccess)
        h = gm::launch_graph_build(d_row_ptr, rp_bytes, d_col, d_clab, n, stride, vinfo, loff, stride > 1 ? lcol : nullptr,
                                   e->num_cu, s);
    if (h != hipSuccess) return device_error(h, "vertex records and label slices");
    // 3. vertices by label and degree (host), hubs: the highest degrees
    std::vector<int64_t> lab_start;
    std::vector<int32_t> bylabel, by_degree;
    std::vector<uint32_t> bylabel_deg;
    order_vertices(hg, lab_start, bylabel, bylabel_deg, by_degree);
    if (n) h = hipMemcpyAsync(bylabel_d, bylabel.data(), static_cast<size_t>(n) * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (h != hipSuccess) return device_error(h, "vertex order");
    const uint64_t words = (static_cast<uint64_t>(n) + 31) / 32;
    int32_t hubs = 0;
    if (!e->opt.disable_hub_bitmaps && n > 0) {
        int64_t big = 0;
        while (big < n && hg.deg[by_degree[big]] >= kHubMinDegree) ++big;
        const uint64_t mib = e->opt.hub_bitmap_mib > 0 ? e->opt.hub_bitmap_mib : kHubDefaultMiB;
        const uint64_t fit = (mib << 20) / (words * 4);
        hubs = static_cast<int32_t>(std::min<uint64_t>({static_cast<uint64_t>(big), static_cast<uint64_t>(kMaxHubs), fit}));
    }
    if (hubs > 0) {
        h = hipMalloc(reinterpret_cast<void **>(&hub_id), static_cast<size_t>(n) * sizeof(int32_t));
        if (h == hipSuccess) h = hipMalloc(reinterpret_cast<void **>(&hub_bits), static_cast<size_t>(hubs) * words * sizeof(uint32_t));
        if (h == hipSuccess) h = hipMalloc(reinterpret_cast<void **>(&hub_list), static_cast<size_t>(hubs) * sizeof(int32_t));
        if (h == hipSuccess) h = hipMemsetAsync(hub_id, 0xff, static_cast<size_t>(n) * sizeof(int32_t), s);
        if (h == hipSuccess) h = hipMemsetAsync(hub_bits, 0, static_cast<size_t>(hubs) * words * sizeof(uint32_t), s);
        if (h == hipSuccess)
            h = hipMemcpyAsync(hub_list, by_degree.data(), static_cast<size_t>(hubs) * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (h == hipSuccess) h = gm::launch_hub_bitmaps(vinfo, d_col, hub_list, hubs, hub_bits, words, hub_id, e->num_cu, s);
        if (h != hipSuccess) return device_error(h, "hub bitmaps");
    }
    h = hipStreamSynchronize(s);
    if (h == hipSuccess) h = hipGetLastError();
    if (h != hipSuccess) return device_error(h, "build");
    release(false);
    free_graph(e);
    e->d_vinfo = vinfo;
    e->d_col = d_col;
    e->col_owned = col_owned;
    e->d_loff = loff;
    e->d_lcol = stride > 1 ? lcol : d_col;
    e->loff_stride = stride;
    e->d_bylabel = bylabel_d;
    e->d_hub_id = hub_id;
    e->d_hub_bits = hub_bits;
    e->hub_words = hubs > 0 ? words : 0;
    e->hubs = hubs;
    e->label_id = std::move(hg.ids);
    e->lab_start = std::move(lab_start);
    e->bylabel_deg = std::move(bylabel_deg);
    e->n = n;
    e->nnz = hg.nnz;
    e->has_graph = true;
    return GM_OK;
}

gm_status get_query(const gm_engine *e, int32_t qid, const QueryRec **q) {
    if (qid < 0 || qid >= static_cast<int32_t>(e->queries.size()) || !e->queries[qid].live)
        return e->fail(GM_ERR_STATE, "unknown or freed query id " + std::to_string(qid));
    *q = &e->queries[qid];
    return GM_OK;
}

gm_status read_ctl(gm_engine *e, LaunchCtx &c, Control *host) {
    HIP_TRY(e, hipMemcpyAsync(host, c.d_ctl, sizeof(Control), hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(e, hipStreamSynchronize(c.stream));
    return GM_OK;
}

// Empty idle bitmap and mailboxes, zero busy and idle counts before a launch that steals.
gm_status reset_stealing(gm_engine *e, LaunchCtx &c, const SearchArgs &a) {
    if (!a.mail) return GM_OK;
    HIP_TRY(e, hipMemsetAsync(&c.d_ctl->busy, 0, sizeof(int), c.stream));
    HIP_TRY(e, hipMemsetAsync(&c.d_ctl->idle_count, 0, sizeof(int), c.stream));
    HIP_TRY(e, gm::launch_steal_init(a.mail, a.idle_bits, a.steal_slots, c.stream));
    return GM_OK;
}

// Plan of a query along its order (a0): labels as G's compact ids (255 when
// absent from G, which leaves no candidates), query degrees and backward masks.
Plan make_plan(const gm_engine *e, const QueryRec &q, bool *label_missing) {
    Plan plan{};
    plan.k = q.k;
    plan.depth = 1;
    plan.flush = ~0ull;
    *label_missing = false;
    for (int32_t i = 0; i < q.k; ++i) {
        const int32_t u = q.order[i];
        plan.phi[i] = u;
        auto it = e->label_id.find(q.labels[u]);
        plan.lab[i] = it == e->label_id.end() ? 255 : it->second;
        *label_missing |= it == e->label_id.end();
        plan.qdeg[i] = popcount(q.adj[u]);
        uint32_t b = 0;
        for (int32_t j = 0; j < i; ++j)
            if ((q.adj[u] >> q.order[j]) & 1u) b |= 1u << j;
        plan.bwd[i] = b;
        if (q.sb) {
            for (int32_t j = 0; j < i; ++j) {
                const int32_t w = q.order[j];
                if ((q.less[w] >> u) & 1u) plan.sb_lt[i] |= 1u << j;  // M(w) < M(u)
                if ((q.less[u] >> w) & 1u) plan.sb_gt[i] |= 1u << j;  // M(u) < M(w)
            }
        }
    }
    return plan;
}

// Local matches a wavefront keeps before adding them to the query's count: small
// enough that the cap is seen soon after it is reached.
unsigned long long flush_for_cap(const gm_engine *e, uint64_t cap) {
    if (!cap) return ~0ull;
    const unsigned long long per = cap / (static_cast<unsigned long long>(e->num_cu) * 64ull);
    return std::max<unsigned long long>(1, std::min<unsigned long long>(4096, per));
}

// Mailboxes and idle bitmap for work stealing (allocated on first use).
// Device memory where each wavefront parks the task groups of the levels below
// the one it scatters: a.levels x 64 entries per wavefront that can be resident
// (at most 32 per CU).  Grows with the deepest launch; kept in the context.
gm_status attach_parked(gm_engine *e, LaunchCtx &c, SearchArgs &a) {
    const int32_t waves = e->num_cu * 32;
    const size_t need = static_cast<size_t>(waves) * static_cast<size_t>(std::max(a.levels, 1)) * gm::kWave;
    if (need > c.parked_cap) {
        if (c.d_parked) (void)hipFree(c.d_parked);
        c.d_parked = nullptr;
        c.parked_cap = 0;
        if (hipMalloc(reinterpret_cast<void **>(&c.d_parked), need * sizeof(uint2)) != hipSuccess)
            return e->fail(GM_ERR_NOMEM, "allocation of the parked task groups failed");
        c.parked_cap = need;
    }
    a.parked = c.d_parked;
    a.park_waves = waves;
    return GM_OK;
}

gm_status attach_stealing(gm_engine *e, LaunchCtx &c, SearchArgs &a) {
    gm_status st = attach_parked(e, c, a);
    if (st) return st;
    a.mail = nullptr;
    a.idle_bits = nullptr;
    a.steal_slots = 0;
    a.steal_threshold = e->opt.steal_threshold > 0 ? e->opt.steal_threshold : 128;
    if (e->opt.disable_stealing) return GM_OK;
    if (!c.d_mail) {
        // one mailbox per wavefront that can be resident (at most 32 per CU)
        const int32_t slots = e->num_cu * 32;
        hipError_t h = hipMalloc(reinterpret_cast<void **>(&c.d_mail), sizeof(gm::Mailbox) * slots);
        if (h == hipSuccess)
            h = hipMalloc(reinterpret_cast<void **>(&c.d_idle_bits), sizeof(unsigned long long) * ((slots + 63) / 64));
        if (h != hipSuccess) {
            if (c.d_mail) (void)hipFree(c.d_mail);
            c.d_mail = nullptr;
            c.d_idle_bits = nullptr;
            return e->fail(GM_ERR_NOMEM, "work-stealing mailbox allocation failed");
        }
        c.steal_slots = slots;
    }
    a.mail = c.d_mail;
    a.idle_bits = c.d_idle_bits;
    a.steal_slots = c.steal_slots;
    return GM_OK;
}

// Staging entries per lane of the LDS-staged intersection (0 = never stage).
int32_t merge_slots(const gm_engine *e) {
    return e->opt.merge_ratio < 0 ? 0 : (e->opt.merge_ratio == 0 ? gm::kDefaultMergeSlots : e->opt.merge_ratio);
}

SearchArgs graph_args(const gm_engine *e, const LaunchCtx &c) {
    SearchArgs a{};
    a.vinfo = e->d_vinfo;
    a.col = e->d_col;
    a.lcol = e->d_lcol;
    a.loff = e->d_loff;
    a.loff_stride = e->loff_stride;
    a.hub_id = e->d_hub_id;
    a.hub_bits = e->d_hub_bits;
    a.hub_words = e->hub_words;
    a.ctl = c.d_ctl;
    a.plans = c.d_plans;
    a.qctl = c.d_qctl;
    a.streams = c.d_streams;
    a.merge_slots = merge_slots(e);
    a.merge_auto = e->opt.merge_ratio == 0 ? 1 : 0;
    return a;
}

unsigned long long items_of(unsigned long long rows) { return (rows + gm::kWave - 1) / gm::kWave; }

// Does a plan carry symmetry-breaking conditions (then its launch takes the kernel that checks them)?
bool has_sb(const Plan &p) {
    for (int32_t i = 0; i < p.k; ++i)
        if (p.sb_lt[i] | p.sb_gt[i]) return true;
    return false;
}

// Two-phase pool: tasks of position 1 a root keeps in its first-phase item
// (default).  Measured one query per launch on the 12-32-vertex queries on
// R-MAT scale 24: 16, 8, 4, 2 and 1 gave 54.6, 56.2, 57.1, 58.0 and 58.8 G
// embeddings/s, with the slowest query and p99 falling too; the 8-vertex
// queries on scale 20 ran level (within 1 %) from 8 down to 1, and 32 and more
// were slower there.  Every root still gets one task in the first phase, so it
// is sampled early; the rest of its list spreads over second-phase items.
constexpr uint32_t kHubCut = 1;
// ... unless a first-phase item holds one root (fewer roots than resident
// wavefronts, as on a candidate graph): a cut of 1 would then give the item a
// single task, one busy lane in 64.  There the default is 8: on the candidate
// graph of the G(n, M) workload, cut 1 took the search from 46 to 94 ms.
constexpr uint32_t kHubCutFewRoots = 8;

// Task split of a query's two-phase pool: its own setting, else the engine's, else the default.
int32_t query_split(const gm_engine *e, const QueryRec &q) {
    if (q.split > 0) return q.split;
    return e->opt.pool_hub_cut > 0 ? e->opt.pool_hub_cut : static_cast<int32_t>(kHubCut);
}

// A query is finished when every work item of it was claimed (its stream's
// counter passed them) and every unit of its work (item or donation) ran to its end.
bool query_finished(const Plan &p, const gm::QCtl &qc, const gm::StreamCtl &sc) {
    return qc.live == 0 && sc.next >= p.item_end;
}

// Multiplier of the order in which a share of n roots is visited: near n times
// the golden ratio's fraction and coprime to n, so consecutive work items mix
// high- and low-degree roots (the bucket stores them by degree).  A capped
// search that starts on the hubs alone can spend its time in their subtrees
// (one 32-vertex query on the scale-24 graph: 5 s without reaching the cap,
// 0.1 s with the roots in id order).
unsigned long long root_order(unsigned long long n) {
    if (n < 3) return 0;
    unsigned long long m = static_cast<unsigned long long>(static_cast<double>(n) * 0.6180339887498949) | 1ull;
    auto gcd = [](unsigned long long x, unsigned long long y) {
        while (y) {
            const unsigned long long t = x % y;
            x = y;
            y = t;
        }
        return x;
    };
    while (gcd(m, n) != 1) m += 2;
    return m % n;
}

// Candidates of the first query vertex as a share of the label buckets: the
// vertices with its label and at least its degree, a prefix of that bucket.
void root_share(const gm_engine *e, const Plan &p, unsigned long long *row0, unsigned long long *rows) {
    *row0 = 0;
    *rows = 0;
    if (p.lab[0] == 255 || e->n == 0) return;
    const int64_t b = e->lab_start[p.lab[0]], en = e->lab_start[p.lab[0] + 1];
    const uint32_t need = static_cast<uint32_t>(p.qdeg[0]);
    auto first = e->bylabel_deg.begin() + b;
    auto it = std::partition_point(first, e->bylabel_deg.begin() + en, [need](uint32_t d) { return d >= need; });
    *row0 = static_cast<unsigned long long>(b);
    *rows = static_cast<unsigned long long>(it - first);
}

// Candidate graph G' of one query (the filtering pass that EGSM-style matchers
// run first; the paper searches EGSM's G' when comparing with it, Sec. 6.1, and
// App. C describes it).  C(l) starts as the vertices with position l's label
// and at least its query degree, and sweeps drop a vertex while some query
// neighbour's set holds none of its neighbours, until a sweep drops nothing
// (the largest such family).  Then, for each query edge (i, l) with i before
// l, the list of every v in C(i) is N(v) restricted to C(l).  The candidates
// of position 0, ids ascending, are the roots.
struct CandInfo {
    const int32_t *roots = nullptr;
    unsigned long long nroots = 0;
    unsigned long long edges = 0;
    int32_t rounds = 0;
};

// Vertices with label id c and degree >= d: a prefix of c's bucket.
unsigned long long bucket_prefix(const gm_engine *e, int32_t c, int32_t d) {
    if (c < 0 || c >= static_cast<int32_t>(e->lab_start.size()) - 1) return 0;
    auto first = e->bylabel_deg.begin() + e->lab_start[c];
    auto it = std::partition_point(first, e->bylabel_deg.begin() + e->lab_start[c + 1],
                                   [d](uint32_t x) { return x >= static_cast<uint32_t>(d); });
    return static_cast<unsigned long long>(it - first);
}

gm_status build_candidate_graph(gm_engine *e, const Plan &p, CandInfo *ci, uint32_t *gslot) {
    hipStream_t s = e->lc.stream;
    const int32_t n = e->n;
    const int32_t k = p.k;
    gm::CandQuery cq{};
    cq.k = k;
    std::vector<gm::CandEdge> edges;
    unsigned long long c0[kMaxK] = {}, c0_all = 0;
    for (int l = 0; l < k; ++l) {
        cq.lab[l] = p.lab[l];
        cq.qdeg[l] = p.qdeg[l];
        cq.adj[l] |= p.bwd[l];
        c0[l] = bucket_prefix(e, p.lab[l], p.qdeg[l]);  // C(l) is a subset of this prefix
        c0_all += c0[l];
        gslot[l] = static_cast<uint32_t>(edges.size());
        for (int j = 0; j < l; ++j) {
            if (!((p.bwd[l] >> j) & 1u)) continue;
            cq.adj[j] |= 1u << l;
            gm::CandEdge ed{};
            ed.src = j;
            ed.dst = l;
            edges.push_back(ed);
        }
    }
    const int32_t m = static_cast<int32_t>(edges.size());
    unsigned long long t_most = 0;
    for (const gm::CandEdge &ed : edges) t_most += c0[ed.src];
    const unsigned long long wp = gm::cand_bitmap_words(n), words = wp * static_cast<unsigned long long>(k);
    const unsigned long long bounds_bytes = 2ull * m * static_cast<unsigned long long>(n) * sizeof(uint32_t);
    if (c0_all >= (1ull << 32) || t_most >= (1ull << 32) || bounds_bytes > (64ull << 30))
        return e->fail(GM_ERR_NOMEM, "candidate graph too large for this graph and query");
    *ci = CandInfo{};
    gm_status st = ensure_buffer(e, &e->d_cbits, &e->cbits_cap, static_cast<size_t>(words));
    if (!st) st = ensure_buffer(e, &e->d_cmisc, &e->cmisc_cap, 64);
    if (!st) st = ensure_buffer(e, &e->d_crank, &e->crank_cap, static_cast<size_t>(std::max(words, t_most)));
    if (!st) st = ensure_buffer(e, &e->d_ctmp, &e->ctmp_cap,
                                static_cast<size_t>(gm::cand_scan_temp_words(std::max(words, t_most))));
    if (!st) st = ensure_buffer(e, &e->d_clist, &e->clist_cap, static_cast<size_t>(std::max<unsigned long long>(c0_all, 1)));
    if (!st && m > 0) st = ensure_buffer(e, &e->d_cedges, &e->cedges_cap, m * sizeof(gm::CandEdge) / sizeof(int32_t));
    if (!st && m > 0)
        st = ensure_buffer(e, &e->d_gbounds, &e->gbounds_cap, static_cast<size_t>(bounds_bytes / sizeof(int32_t)));
    if (st) return st;
    uint32_t *bits = reinterpret_cast<uint32_t *>(e->d_cbits);
    uint32_t *flag = reinterpret_cast<uint32_t *>(e->d_cmisc);
    auto *list_total = reinterpret_cast<unsigned long long *>(e->d_cmisc + 4);
    uint32_t *bounds = reinterpret_cast<uint32_t *>(e->d_cmisc + 8);  // k + 1 words
    uint32_t *scratch = reinterpret_cast<uint32_t *>(e->d_crank);
    uint32_t *tmp = reinterpret_cast<uint32_t *>(e->d_ctmp);

    HIP_TRY(e, gm::launch_cand_init(e->d_vinfo, n, cq, bits, e->num_cu, s));
    // Sweeps go kSweeps at a time, each with its own flag, and one read-back
    // per group: a sweep after the fixed point clears nothing and costs one
    // pass, where a host round trip per sweep would cost more.
    constexpr int kSweeps = 4;
    for (bool done = false; !done;) {
        uint32_t changed[kSweeps] = {};
        HIP_TRY(e, hipMemsetAsync(flag, 0, sizeof(changed), s));
        for (int r = 0; r < kSweeps; ++r)
            HIP_TRY(e, gm::launch_cand_refine(e->d_lcol, e->d_loff, e->loff_stride, n, cq, bits, flag + r, e->num_cu, s));
        HIP_TRY(e, hipMemcpyAsync(changed, flag, sizeof(changed), hipMemcpyDeviceToHost, s));
        HIP_TRY(e, hipStreamSynchronize(s));
        for (int r = 0; r < kSweeps && !done; ++r) {
            ++ci->rounds;
            done = changed[r] == 0;
        }
    }
    uint32_t hb[kMaxK + 1] = {};
    HIP_TRY(e, gm::launch_cand_lists(bits, n, k, scratch, tmp, e->d_clist, bounds, e->num_cu, s));
    HIP_TRY(e, hipMemcpyAsync(hb, bounds, (k + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(e, hipStreamSynchronize(s));
    ci->roots = e->d_clist + hb[0];
    ci->nroots = hb[1] - hb[0];
    if (m == 0) return GM_OK;
    unsigned long long first = 0, most = 1;
    for (gm::CandEdge &ed : edges) {
        ed.start = hb[ed.src];
        ed.len = hb[ed.src + 1] - hb[ed.src];
        ed.first = static_cast<uint32_t>(first);
        first += ed.len;
        most = std::max<unsigned long long>(most, ed.len);
    }
    e->h_cedges = edges;  // kept until the upload below has completed
    const gm::CandEdge *d_edges = reinterpret_cast<const gm::CandEdge *>(e->d_cedges);
    unsigned long long total = 0;
    HIP_TRY(e, hipMemcpyAsync(e->d_cedges, e->h_cedges.data(), m * sizeof(gm::CandEdge), hipMemcpyHostToDevice, s));
    HIP_TRY(e, hipMemsetAsync(list_total, 0, sizeof(unsigned long long), s));
    HIP_TRY(e, gm::launch_cand_count(e->d_lcol, e->d_loff, e->loff_stride, n, cq, bits, d_edges, m, most, e->d_clist,
                                     scratch, list_total, e->num_cu, s));
    HIP_TRY(e, hipMemcpyAsync(&total, list_total, sizeof(total), hipMemcpyDeviceToHost, s));
    HIP_TRY(e, hipStreamSynchronize(s));
    if (total >= (1ull << 32)) return e->fail(GM_ERR_NOMEM, "candidate graph holds 2^32 list entries or more");
    ci->edges = total;
    HIP_TRY(e, gm::launch_exclusive_scan(scratch, first, tmp, s));
    st = ensure_buffer(e, &e->d_gcol, &e->gcol_cap, static_cast<size_t>(std::max<unsigned long long>(total, gm::kListWindow)));
    if (st) return st;
    HIP_TRY(e, gm::launch_cand_fill(e->d_lcol, e->d_loff, e->loff_stride, n, cq, bits, d_edges, m, most, e->d_clist,
                                    scratch, e->d_gcol, reinterpret_cast<uint32_t *>(e->d_gbounds), e->num_cu, s));
    HIP_TRY(e, hipStreamSynchronize(s));  // the build's time ends with its last kernel
    return GM_OK;
}

// One search with the two-phase pool (the default).  The roots are a bucket
// prefix, visited in a mixed order.  First-phase items hold 64 roots each, every
// root with at most its first kHubCut tasks of position 1, so every root is
// sampled early and a hub holds up one wavefront, not all of them.  The rest of
// the hubs' tasks form the second phase: one pass gives each root's remaining
// slice, a prefix sum lays them out as one task list, and an item is 64
// consecutive tasks of it, so a hub's work spreads over many wavefronts.
// Wavefronts that find no first-phase item start on second-phase items at once.
// Everything is queued without a host round trip.
gm_status run_virtual(gm_engine *e, const QueryRec *q, const Plan &base_plan, uint64_t cap, double time_limit_s,
                      int32_t *rows, gm_result *out) {
    const bool enumerate = rows != nullptr;
    const auto t_start = std::chrono::steady_clock::now();
    Plan p = base_plan;
    unsigned long long row0 = 0, R = 0;
    root_share(e, p, &row0, &R);
    out->pool_depth = 1;
    out->pool_rows = R;
    out->outcome = GM_DONE;
    if (R == 0 || q->k == 1) {
        // no candidates, or a single query vertex: its candidates are the matches
        out->count = cap && R >= cap ? cap : R;
        out->outcome = cap && R >= cap ? GM_CAPPED : GM_DONE;
        if (enumerate && out->count) {
            HIP_TRY(e, hipMemcpyAsync(rows, e->d_bylabel + row0, out->count * sizeof(int32_t), hipMemcpyDeviceToHost,
                                      e->lc.stream));
            HIP_TRY(e, hipStreamSynchronize(e->lc.stream));
            out->rows = out->count;
        }
        std::chrono::duration<double, std::milli> ms = std::chrono::steady_clock::now() - t_start;
        out->search_ms = ms.count();
        return GM_OK;
    }
    if (R >= (1ull << 31)) return e->fail(GM_ERR_GRAPH, "more than 2^31 candidates for the first query vertex");
    // candidate graph: the roots become C(phi[0]) and every list is read from G'
    const bool cg = e->opt.candidate_graph != 0;
    const int32_t *pool = e->d_bylabel;
    if (cg) {
        CandInfo ci;
        const auto t_cg = std::chrono::steady_clock::now();
        gm_status cst = build_candidate_graph(e, p, &ci, p.gslot);
        if (cst) return cst;
        std::chrono::duration<double, std::milli> cg_ms = std::chrono::steady_clock::now() - t_cg;
        out->candidate_ms = cg_ms.count();
        out->candidate_rounds = ci.rounds;
        out->candidate_edges = ci.edges;
        pool = ci.roots;
        row0 = 0;
        R = ci.nroots;
        out->pool_rows = R;
        if (R == 0) {
            std::chrono::duration<double, std::milli> ms = std::chrono::steady_clock::now() - t_start;
            out->search_ms = ms.count();
            return GM_OK;
        }
    }
    gm_status st = ensure_query_slots(e, e->lc, 2);
    if (!st) st = ensure_streams(e, e->lc, 1);
    if (!st) st = ensure_level1(e, R);
    if (!st && enumerate) st = ensure_buffer(e, &e->d_rows, &e->rows_cap, static_cast<size_t>(cap) * q->k);
    if (st) return st;

    p.depth = 1;
    p.cap = cap;
    p.flush = flush_for_cap(e, cap);
    p.row0 = row0;
    p.rows = R;
    p.item0 = 0;
    p.item_end = 0;  // set on the device from the level-1 total
    p.vmode = 1;
    p.hub_cut = static_cast<uint32_t>(query_split(e, *q));
    p.vrow0 = 0;
    p.perm_mul = root_order(R);
    if (e->opt.pool_roots_per_item > 0) {
        p.rpi = static_cast<uint32_t>(e->opt.pool_roots_per_item);
    } else {
        // Fewer roots than resident wavefronts: one root per item, so every root
        // starts on a wavefront of its own (a candidate graph often leaves that
        // few).  Otherwise 64: measured on the scale-20 workload, items of R /
        // wavefronts roots (about 3) ran 3 % slower than 64.
        const unsigned long long waves = static_cast<unsigned long long>(
            std::max(1, gm::search_waves(q->k, e->num_cu, e->opt.waves_per_cu, cg || use_slim(e, q->k), merge_slots(e),
                                             e->opt.merge_ratio == 0)));
        p.rpi = R < waves ? 1u : static_cast<uint32_t>(gm::kWave);
    }
    if (q->split <= 0 && e->opt.pool_hub_cut <= 0 && p.rpi < static_cast<uint32_t>(gm::kWave))
        p.hub_cut = std::max(p.hub_cut, kHubCutFewRoots);
    p.item_split = (R + p.rpi - 1) / p.rpi;
    e->lc.h_plans.assign(1, p);
    e->lc.h_streams.assign(1, gm::StreamCtl{});
    e->lc.h_streams[0].plan0 = 0;
    e->lc.h_streams[0].plan1 = 1;
    HIP_TRY(e, hipMemsetAsync(e->lc.d_ctl, 0, sizeof(Control), e->lc.stream));
    HIP_TRY(e, hipMemsetAsync(e->lc.d_qctl, 0, 2 * sizeof(gm::QCtl), e->lc.stream));
    HIP_TRY(e, hipMemcpyAsync(e->lc.d_plans, e->lc.h_plans.data(), sizeof(Plan), hipMemcpyHostToDevice, e->lc.stream));
    HIP_TRY(e, hipMemcpyAsync(e->lc.d_streams, e->lc.h_streams.data(), sizeof(gm::StreamCtl), hipMemcpyHostToDevice,
                              e->lc.stream));
    HIP_TRY(e, gm::launch_start_clock(e->lc.d_ctl, e->lc.stream));
    // the second phase's scanned candidates go to the second slot
    // (on G' position 1's lists are those of the query edge (0, 1))
    const int32_t lab1 = cg ? 0 : (e->loff_stride > 1 ? p.lab[1] : 0);
    const uint32_t *loff1 = cg ? reinterpret_cast<const uint32_t *>(e->d_gbounds) +
                                     2ull * static_cast<unsigned long long>(p.gslot[1]) * static_cast<unsigned long long>(e->n)
                               : e->d_loff;
    const bool slim = cg || use_slim(e, q->k);
    HIP_TRY(e, gm::launch_level1(pool + row0, static_cast<int32_t>(R), p.perm_mul, p.hub_cut, loff1,
                                 cg ? 2 : e->loff_stride, lab1, e->d_vlen, e->d_vstart, e->d_voff, e->d_vtmp,
                                 e->lc.d_qctl + 1, e->lc.d_plans, e->lc.d_streams, e->num_cu, e->lc.stream));
    SearchArgs a = graph_args(e, e->lc);
    a.nq = 1;
    a.nstreams = 1;
    a.levels = q->k;
    a.pool = pool;
    if (cg) {
        a.cg = 1;
        a.lcol = e->d_gcol;
        a.gbounds = reinterpret_cast<const uint32_t *>(e->d_gbounds);
        a.gn = static_cast<unsigned long long>(e->n);
    }
    a.voff = e->d_voff;
    a.vstart = e->d_vstart;
    a.slim = slim ? 1 : 0;
    a.sb = has_sb(p) ? 1 : 0;
    a.budget = time_limit_s > 0
                   ? std::max<unsigned long long>(
                         1, static_cast<unsigned long long>(time_limit_s * 1000.0 * static_cast<double>(e->wall_khz)))
                   : 0ull;
    a.out = enumerate ? e->d_rows : nullptr;
    a.out_cap = enumerate ? cap : 0;
    st = attach_stealing(e, e->lc, a);
    if (!st) st = reset_stealing(e, e->lc, a);
    if (st) return st;
    int grid_waves = 0;
    float kernel_ms = 0.f;
    HIP_TRY(e, hipEventRecord(e->lc.ev0, e->lc.stream));
    HIP_TRY(e, gm::launch_search(a, enumerate, e->num_cu, e->opt.waves_per_cu, e->lc.stream, &grid_waves));
    HIP_TRY(e, hipEventRecord(e->lc.ev1, e->lc.stream));
    gm::QCtl qc[2];
    gm::StreamCtl sc{};
    Control c{};
    HIP_TRY(e, hipMemcpyAsync(qc, e->lc.d_qctl, 2 * sizeof(gm::QCtl), hipMemcpyDeviceToHost, e->lc.stream));
    HIP_TRY(e, hipMemcpyAsync(&sc, e->lc.d_streams, sizeof(gm::StreamCtl), hipMemcpyDeviceToHost, e->lc.stream));
    st = read_ctl(e, e->lc, &c);
    if (st) return st;
    HIP_TRY(e, hipEventElapsedTime(&kernel_ms, e->lc.ev0, e->lc.ev1));

    const gm::QCtl &k0 = qc[0], &l1 = qc[1];
    if (cap && k0.count >= cap) {
        out->count = cap;
        out->outcome = GM_CAPPED;
    } else {
        out->count = k0.count;
        const bool done = k0.live == 0 && sc.next >= sc.items && c.abort != gm::kAbortTime;
        out->outcome = done ? GM_DONE : GM_TIMEOUT;
    }
    out->groups = k0.groups + l1.groups;
    out->tasks = k0.tasks + l1.tasks;
    out->lanes_active = k0.lanes_active;
    out->lanes_issued = k0.lanes_issued;
    out->probes = k0.probes;
    out->steals = k0.steals;
    out->kernel_ms = kernel_ms;
    out->grid_waves = grid_waves;
    out->kernel_tasks = k0.tasks;
    out->kernel_probes = k0.probes;
    out->kernel_groups = k0.groups;
    out->scanned = k0.scanned + l1.scanned;
    out->kernel_scanned = k0.scanned + l1.scanned;  // the search launch reads the level-1 candidates itself
    out->kernel_lookups = k0.lookups;
    out->kernel_bytes = k0.bytes;
    out->kernel_bytes_late = k0.bytes_late;
    if (enumerate) {
        const uint64_t nrows = std::min<uint64_t>(out->count, std::min<uint64_t>(c.out_rows, cap));
        if (nrows) {
            HIP_TRY(e, hipMemcpyAsync(rows, e->d_rows, nrows * q->k * sizeof(int32_t), hipMemcpyDeviceToHost,
                                      e->lc.stream));
            HIP_TRY(e, hipStreamSynchronize(e->lc.stream));
        }
        out->rows = nrows;
    }
    std::chrono::duration<double, std::milli> ms = std::chrono::steady_clock::now() - t_start;
    out->search_ms = ms.count();
    return GM_OK;
}

// One search (Alg. 2): root candidates, breadth-first pool to tau, then the
// persistent depth-first kernel.  rows != null selects enumeration.
gm_status run_search(gm_engine *e, int32_t qid, uint64_t cap, double time_limit_s, int32_t *rows,
                     gm_result *out) {
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    if (!e->has_graph) return e->fail(GM_ERR_STATE, "no data graph loaded");
    if (e->device < 0) return e->fail(GM_ERR_DEVICE, "host-only engine (created with device -1) cannot search");
    std::memset(out, 0, sizeof(*out));
    HIP_TRY(e, hipSetDevice(e->device));

    bool label_missing = false;
    const Plan base_plan = make_plan(e, *q, &label_missing);
    const bool enumerate = rows != nullptr;
    if (label_missing || e->n == 0) {
        out->outcome = GM_DONE;
        return GM_OK;
    }
    if (e->opt.tau == 0) return run_virtual(e, q, base_plan, cap, time_limit_s, rows, out);
    st = ensure_query_slots(e, e->lc, 1);
    if (!st) st = ensure_streams(e, e->lc, 1);
    if (st) return st;

    const auto t_start = std::chrono::steady_clock::now();
    const long long budget_ticks =
        time_limit_s > 0 ? static_cast<long long>(time_limit_s * 1000.0 * static_cast<double>(e->wall_khz)) : 0;
    auto timed_out_host = [&]() {
        if (time_limit_s <= 0) return false;
        std::chrono::duration<double> el = std::chrono::steady_clock::now() - t_start;
        return el.count() > time_limit_s;
    };

    HIP_TRY(e, hipMemsetAsync(e->lc.d_ctl, 0, sizeof(Control), e->lc.stream));
    HIP_TRY(e, hipMemsetAsync(e->lc.d_qctl, 0, sizeof(gm::QCtl), e->lc.stream));
    st = ensure_buffer(e, &e->d_pool[0], &e->pool_cap[0], static_cast<size_t>(e->n));
    if (st) return st;
    // the root scan also bounds the next level: each root's label slice for position 1
    const int32_t lab1 = q->k >= 2 ? (e->loff_stride > 1 ? base_plan.lab[1] : 0) : -1;
    HIP_TRY(e, gm::launch_root_scan(e->d_vinfo, e->n, base_plan.lab[0], base_plan.qdeg[0], e->d_pool[0], e->d_loff,
                                    e->loff_stride, lab1, e->lc.d_ctl, e->num_cu, e->lc.stream));
    Control c{};
    st = read_ctl(e, e->lc, &c);
    if (st) return st;
    uint64_t pool_rows = c.out_rows;
    uint64_t bound = c.measure;  // upper bound on the rows of the next level
    int cur = 0;
    int32_t depth = 1;

    SearchArgs a = graph_args(e, e->lc);
    a.nq = 1;
    a.nstreams = 1;
    a.levels = q->k;
    a.budget = static_cast<unsigned long long>(budget_ticks);
    a.slim = use_slim(e, q->k) ? 1 : 0;
    a.sb = has_sb(base_plan) ? 1 : 0;
    st = attach_stealing(e, e->lc, a);
    if (st) return st;

    if (q->k == 1) {
        // a single query vertex: its candidates are the matches
        const uint64_t cnt = pool_rows;
        out->count = cap && cnt >= cap ? cap : cnt;
        out->outcome = cap && cnt >= cap ? GM_CAPPED : GM_DONE;
        out->pool_rows = pool_rows;
        out->pool_depth = 1;
        if (enumerate && out->count) {
            HIP_TRY(e, hipMemcpyAsync(rows, e->d_pool[0], out->count * sizeof(int32_t), hipMemcpyDeviceToHost,
                                      e->lc.stream));
            HIP_TRY(e, hipStreamSynchronize(e->lc.stream));
            out->rows = out->count;
        }
        std::chrono::duration<double, std::milli> ms = std::chrono::steady_clock::now() - t_start;
        out->search_ms = ms.count();
        return GM_OK;
    }

    // Plan 0 with the current pool level as its share (one query, items from 0).
    auto upload_plan = [&](int32_t d, uint64_t nrows, unsigned long long flush) -> gm_status {
        e->lc.h_plans.assign(1, base_plan);
        Plan &p = e->lc.h_plans[0];
        p.depth = d;
        p.cap = cap;
        p.flush = flush;
        p.row0 = 0;
        p.rows = nrows;
        p.item0 = 0;
        p.item_end = items_of(nrows);
        e->lc.h_streams.assign(1, gm::StreamCtl{});
        e->lc.h_streams[0].items = p.item_end;
        e->lc.h_streams[0].plan0 = 0;
        e->lc.h_streams[0].plan1 = 1;
        HIP_TRY(e, hipMemcpyAsync(e->lc.d_plans, &p, sizeof(Plan), hipMemcpyHostToDevice, e->lc.stream));
        HIP_TRY(e, hipMemcpyAsync(e->lc.d_streams, e->lc.h_streams.data(), sizeof(gm::StreamCtl), hipMemcpyHostToDevice,
                                  e->lc.stream));
        HIP_TRY(e, hipMemsetAsync(&e->lc.d_ctl->out_rows, 0, sizeof(unsigned long long), e->lc.stream));
        return GM_OK;
    };
    gm::QCtl qc{};
    gm::StreamCtl sc{};
    auto read_results = [&]() -> gm_status {
        HIP_TRY(e, hipMemcpyAsync(&qc, e->lc.d_qctl, sizeof(gm::QCtl), hipMemcpyDeviceToHost, e->lc.stream));
        HIP_TRY(e, hipMemcpyAsync(&sc, e->lc.d_streams, sizeof(gm::StreamCtl), hipMemcpyDeviceToHost, e->lc.stream));
        return read_ctl(e, e->lc, &c);
    };

    // Initialisation phase (Sec. 4.3): breadth-first levels until >= tau rows.
    const int64_t tau = e->opt.tau;  // > 0 here: breadth-first to tau; < 0: no expansion
    const int64_t row_limit = e->opt.pool_row_limit > 0 ? e->opt.pool_row_limit : 64 * std::max<int64_t>(tau, 1);
    bool aborted = false;
    while (tau > 0 && pool_rows > 0 && pool_rows < static_cast<uint64_t>(tau) && depth < q->k - 1) {
        if (bound > static_cast<uint64_t>(row_limit)) break;
        st = ensure_buffer(e, &e->d_pool[cur ^ 1], &e->pool_cap[cur ^ 1], bound * static_cast<size_t>(depth + 1));
        if (st) return st;
        st = upload_plan(depth, pool_rows, ~0ull);
        if (st) return st;
        HIP_TRY(e, hipMemsetAsync(&e->lc.d_ctl->measure, 0, sizeof(unsigned long long), e->lc.stream));
        a.pool = e->d_pool[cur];
        a.out = e->d_pool[cur ^ 1];
        a.out_cap = bound;
        a.measure_next = depth + 1 < q->k - 1 ? 1 : 0;  // bound of the level after this one
        st = reset_stealing(e, e->lc, a);
        if (st) return st;
        HIP_TRY(e, gm::launch_expand(a, e->num_cu, e->lc.stream));
        st = read_results();
        if (st) return st;
        if (c.abort != gm::kAbortNone || timed_out_host()) {
            aborted = true;
            break;
        }
        pool_rows = c.out_rows;
        bound = c.measure;
        cur ^= 1;
        ++depth;
    }

    int grid_waves = 0;
    float kernel_ms = 0.f;
    gm::QCtl before = qc;
    bool finished = !aborted;
    if (!aborted && pool_rows > 0) {
        if (enumerate) {
            st = ensure_buffer(e, &e->d_rows, &e->rows_cap, static_cast<size_t>(cap) * q->k);
            if (st) return st;
        }
        st = upload_plan(depth, pool_rows, flush_for_cap(e, cap));
        if (st) return st;
        a.pool = e->d_pool[cur];
        a.out = enumerate ? e->d_rows : nullptr;
        a.out_cap = enumerate ? cap : 0;
        a.measure_next = 0;
        st = reset_stealing(e, e->lc, a);
        if (st) return st;
        HIP_TRY(e, hipEventRecord(e->lc.ev0, e->lc.stream));
        HIP_TRY(e, gm::launch_search(a, enumerate, e->num_cu, e->opt.waves_per_cu, e->lc.stream, &grid_waves));
        HIP_TRY(e, hipEventRecord(e->lc.ev1, e->lc.stream));
        st = read_results();
        if (st) return st;
        HIP_TRY(e, hipEventElapsedTime(&kernel_ms, e->lc.ev0, e->lc.ev1));
        finished = query_finished(e->lc.h_plans[0], qc, sc);
    }

    const uint64_t total = qc.count;
    if (cap && total >= cap) {
        out->count = cap;
        out->outcome = GM_CAPPED;
    } else {
        out->count = total;
        out->outcome = finished ? GM_DONE : GM_TIMEOUT;
    }
    out->pool_rows = pool_rows;
    out->pool_depth = depth;
    out->groups = qc.groups;
    out->tasks = qc.tasks;
    out->lanes_active = qc.lanes_active;
    out->lanes_issued = qc.lanes_issued;
    out->probes = qc.probes;
    out->steals = qc.steals;
    out->kernel_ms = kernel_ms;
    out->grid_waves = grid_waves;
    out->kernel_tasks = qc.tasks - before.tasks;
    out->kernel_probes = qc.probes - before.probes;
    out->kernel_groups = qc.groups - before.groups;
    out->scanned = qc.scanned;
    out->kernel_scanned = qc.scanned - before.scanned;
    out->kernel_lookups = qc.lookups - before.lookups;
    out->kernel_bytes = qc.bytes - before.bytes;
    out->kernel_bytes_late = qc.bytes_late - before.bytes_late;
    if (enumerate) {
        const uint64_t nrows = std::min<uint64_t>(out->count, std::min<uint64_t>(c.out_rows, cap));
        if (nrows) {
            HIP_TRY(e, hipMemcpyAsync(rows, e->d_rows, nrows * q->k * sizeof(int32_t), hipMemcpyDeviceToHost,
                                      e->lc.stream));
            HIP_TRY(e, hipStreamSynchronize(e->lc.stream));
        }
        out->rows = nrows;
    }
    std::chrono::duration<double, std::milli> ms = std::chrono::steady_clock::now() - t_start;
    out->search_ms = ms.count();
    return GM_OK;
}

// Wavefronts per CU a search launch for a query of k vertices keeps resident.
int residency(const gm_engine *e, int32_t k) {
    return gm::search_waves(k, e->num_cu, e->opt.waves_per_cu, use_slim(e, k), merge_slots(e),
                            e->opt.merge_ratio == 0);
}

// Work-item streams of a batched launch: the option, else 64 (queries in flight).
int32_t batch_streams(const gm_engine *e) { return e->opt.batch_streams > 0 ? e->opt.batch_streams : 64; }

// One persistent launch of a group of queries on a launch context.  Plans are
// laid out stream by stream (member j of the group goes to stream j mod ns);
// pos[] maps each plan slot back to the caller's index.
struct GroupLaunch {
    std::vector<int32_t> pos;
    int32_t nq = 0;
    int32_t ns = 0;
    int grid_waves = 0;
    bool launched = false;  // false: no query of the group has any work item
};

// Lays out the group plans[members[0 .. g)] and queues its launch on c.stream
// (nothing waits for it).  Levels = the largest query of the group.
gm_status launch_group(gm_engine *e, LaunchCtx &c, const std::vector<Plan> &plans, const int32_t *members, int32_t g,
                       int32_t nstreams, int waves_per_cu, GroupLaunch &gl) {
    int32_t levels = 0;
    for (int32_t j = 0; j < g; ++j) levels = std::max(levels, plans[members[j]].k);
    const int32_t ns = std::max(1, std::min(g, nstreams));
    gl = GroupLaunch{};
    gl.nq = g;
    gl.ns = ns;
    c.h_plans.clear();
    c.h_streams.assign(static_cast<size_t>(ns), gm::StreamCtl{});
    unsigned long long items = 0;
    for (int32_t sidx = 0; sidx < ns; ++sidx) {
        gm::StreamCtl &sc = c.h_streams[sidx];
        sc.plan0 = static_cast<int32_t>(c.h_plans.size());
        unsigned long long local = 0;
        for (int32_t j = sidx; j < g; j += ns) {
            Plan p = plans[members[j]];
            p.item0 = local;
            local += items_of(p.rows);
            p.item_end = local;
            c.h_plans.push_back(p);
            gl.pos.push_back(members[j]);
        }
        sc.plan1 = static_cast<int32_t>(c.h_plans.size());
        sc.items = local;
        items += local;
    }
    if (items == 0) return GM_OK;
    gm_status st = ensure_query_slots(e, c, static_cast<size_t>(g));
    if (!st) st = ensure_streams(e, c, static_cast<size_t>(ns));
    if (st) return st;
    HIP_TRY(e, hipMemsetAsync(c.d_ctl, 0, sizeof(Control), c.stream));
    HIP_TRY(e, hipMemsetAsync(c.d_qctl, 0, sizeof(gm::QCtl) * static_cast<size_t>(g), c.stream));
    HIP_TRY(e, hipMemcpyAsync(c.d_plans, c.h_plans.data(), sizeof(Plan) * static_cast<size_t>(g),
                              hipMemcpyHostToDevice, c.stream));
    HIP_TRY(e, hipMemcpyAsync(c.d_streams, c.h_streams.data(), sizeof(gm::StreamCtl) * static_cast<size_t>(ns),
                              hipMemcpyHostToDevice, c.stream));
    SearchArgs a = graph_args(e, c);
    a.nq = g;
    a.nstreams = ns;
    a.levels = levels;
    a.pool = e->d_bylabel;
    a.slim = use_slim(e, levels) ? 1 : 0;
    a.sb = 0;
    for (const Plan &p : c.h_plans) a.sb |= has_sb(p) ? 1 : 0;
    a.budget = 0;  // limits are per query (plan budgets)
    st = attach_stealing(e, c, a);
    if (!st) st = reset_stealing(e, c, a);
    if (st) return st;
    HIP_TRY(e, gm::launch_start_clock(c.d_ctl, c.stream));
    HIP_TRY(e, hipEventRecord(c.ev0, c.stream));
    HIP_TRY(e, gm::launch_search(a, false, e->num_cu, waves_per_cu, c.stream, &gl.grid_waves));
    HIP_TRY(e, hipEventRecord(c.ev1, c.stream));
    gl.launched = true;
    return GM_OK;
}

// Waits for a launched group and writes each query's result to out[pos[j]]
// (gm_count's rules with the plan's own cap); adds to *sum if not null.
gm_status harvest_group(gm_engine *e, LaunchCtx &c, const GroupLaunch &gl, gm_result *out, gm_batch_info *sum) {
    c.h_qctl.resize(static_cast<size_t>(gl.nq));
    HIP_TRY(e, hipMemcpyAsync(c.h_qctl.data(), c.d_qctl, sizeof(gm::QCtl) * static_cast<size_t>(gl.nq),
                              hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(e, hipMemcpyAsync(c.h_streams.data(), c.d_streams, sizeof(gm::StreamCtl) * static_cast<size_t>(gl.ns),
                              hipMemcpyDeviceToHost, c.stream));
    Control ctl{};
    gm_status st = read_ctl(e, c, &ctl);
    if (st) return st;
    float kernel_ms = 0.f;
    HIP_TRY(e, hipEventElapsedTime(&kernel_ms, c.ev0, c.ev1));
    if (sum) {
        sum->kernel_ms += kernel_ms;
        sum->launches += 1;
        sum->grid_waves = std::max(sum->grid_waves, gl.grid_waves);
    }
    for (int32_t sidx = 0; sidx < gl.ns; ++sidx) {
        const gm::StreamCtl &sc = c.h_streams[sidx];
        for (int32_t j = sc.plan0; j < sc.plan1; ++j) {
            const Plan &p = c.h_plans[j];
            const gm::QCtl &qc = c.h_qctl[j];
            gm_result &r = out[gl.pos[j]];
            if (p.cap && qc.count >= p.cap) {
                r.count = p.cap;
                r.outcome = GM_CAPPED;
            } else {
                r.count = qc.count;
                const bool done = p.rows == 0 || (qc.abort != gm::kAbortTime && query_finished(p, qc, sc));
                r.outcome = done ? GM_DONE : GM_TIMEOUT;
            }
            r.groups = r.kernel_groups = qc.groups;
            r.tasks = r.kernel_tasks = qc.tasks;
            r.lanes_active = qc.lanes_active;
            r.lanes_issued = qc.lanes_issued;
            r.probes = r.kernel_probes = qc.probes;
            r.steals = qc.steals;
            r.scanned = r.kernel_scanned = qc.scanned;
            r.kernel_lookups = qc.lookups;
            r.kernel_bytes = qc.bytes;
            r.kernel_bytes_late = qc.bytes_late;
            r.query_ms = qc.t_start && qc.t_last > qc.t_start
                             ? static_cast<double>(qc.t_last - qc.t_start) / static_cast<double>(e->wall_khz)
                             : 0.0;
            r.kernel_ms = kernel_ms;
            r.grid_waves = gl.grid_waves;
            if (sum) {
                sum->lookups += qc.lookups;
                sum->bytes += qc.bytes;
                sum->bytes_late += qc.bytes_late;
            }
        }
    }
    return GM_OK;
}

// Several queries in shared persistent launches: every query's first-vertex
// candidates (a prefix of its label's bucket, highest degree first) are its
// pool share, and wavefronts move between queries as they claim work items or
// take donations.  Queries are grouped by the residency their stack depth
// allows (or all in one launch), each group one launch.
gm_status run_batch(gm_engine *e, int32_t nq, const int32_t *qids, uint64_t cap, double time_limit_s,
                    gm_result *out, gm_batch_info *info) {
    if (nq < 0) return e->fail(GM_ERR_ARG, "nq must be >= 0");
    if (nq > 0 && (!qids || !out)) return e->fail(GM_ERR_ARG, "qids and out must not be null");
    std::vector<const QueryRec *> recs(static_cast<size_t>(nq));
    for (int32_t i = 0; i < nq; ++i) {
        gm_status st = get_query(e, qids[i], &recs[i]);
        if (st) return st;
    }
    gm_batch_info sum{};
    if (nq == 0) {
        if (info) *info = sum;
        return GM_OK;
    }
    if (!e->has_graph) return e->fail(GM_ERR_STATE, "no data graph loaded");
    if (e->device < 0) return e->fail(GM_ERR_DEVICE, "host-only engine (created with device -1) cannot search");
    const auto t_start = std::chrono::steady_clock::now();
    auto elapsed_s = [&]() {
        std::chrono::duration<double> el = std::chrono::steady_clock::now() - t_start;
        return el.count();
    };
    HIP_TRY(e, hipSetDevice(e->device));
    std::memset(out, 0, sizeof(gm_result) * static_cast<size_t>(nq));

    // each query's limit runs from its first work item on the device
    unsigned long long budget_ticks = 0;
    if (time_limit_s > 0)
        budget_ticks = std::max<unsigned long long>(
            1, static_cast<unsigned long long>(time_limit_s * 1000.0 * static_cast<double>(e->wall_khz)));
    std::vector<Plan> plans(static_cast<size_t>(nq));
    for (int32_t i = 0; i < nq; ++i) {
        bool missing = false;
        Plan p = make_plan(e, *recs[i], &missing);
        p.cap = cap;
        p.flush = flush_for_cap(e, cap);
        p.depth = 1;
        p.budget = budget_ticks;
        if (!missing) root_share(e, p, &p.row0, &p.rows);
        p.perm_mul = root_order(p.rows);
        plans[i] = p;
        out[i].pool_depth = 1;
        out[i].pool_rows = p.rows;
        out[i].outcome = GM_DONE;
    }

    // launch groups: larger residency (shallower stacks) first
    std::vector<int32_t> idx(static_cast<size_t>(nq));
    std::vector<int> key(static_cast<size_t>(nq));
    for (int32_t i = 0; i < nq; ++i) {
        idx[i] = i;
        key[i] = e->opt.batch_single_launch ? 0 : residency(e, plans[i].k);
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return key[x] > key[y]; });

    for (size_t g0 = 0; g0 < idx.size();) {
        size_t g1 = g0;
        while (g1 < idx.size() && key[idx[g1]] == key[idx[g0]]) ++g1;
        GroupLaunch gl;
        gm_status st = launch_group(e, e->lc, plans, idx.data() + g0, static_cast<int32_t>(g1 - g0), batch_streams(e),
                                    e->opt.waves_per_cu, gl);
        if (!st && gl.launched) st = harvest_group(e, e->lc, gl, out, &sum);
        if (st) return st;
        g0 = g1;
    }
    const double total_ms = elapsed_s() * 1000.0;
    for (int32_t i = 0; i < nq; ++i) {
        out[i].search_ms = total_ms;
        sum.count += out[i].count;
        sum.tasks += out[i].tasks;
        sum.scanned += out[i].scanned;
        sum.probes += out[i].probes;
        sum.groups += out[i].groups;
        sum.steals += out[i].steals;
    }
    sum.total_ms = total_ms;
    if (info) *info = sum;
    return GM_OK;
}

// Autotuner of the batched launch: coordinate descent over the settings, each
// knob over a fixed list with the others at their best so far; the measure is
// the batch's device time, and counts must not depend on the setting.
gm_status run_tune(gm_engine *e, int32_t nq, const int32_t *qids, uint64_t cap, double time_limit_s,
                   gm_tuning *out) {
    const gm_options saved = e->opt;
    std::vector<gm_result> ref(static_cast<size_t>(std::max(nq, 1))), res(ref.size());
    gm_batch_info info{};
    gm_status st = run_batch(e, nq, qids, cap, time_limit_s, ref.data(), &info);
    if (st) return st;
    gm_options best = saved;
    best.steal_threshold = saved.steal_threshold > 0 ? saved.steal_threshold : 128;
    best.stack_layout = saved.stack_layout == 1 ? 1 : 2;
    best.batch_streams = batch_streams(e);
    best.merge_ratio = saved.merge_ratio;  // 0 (stage where it costs no residency) is a setting of its own
    double best_ms = info.kernel_ms;
    const double default_ms = info.kernel_ms;
    int32_t trials = 1;
    struct Knob {
        int32_t gm_options::*field;
        std::vector<int32_t> values;
    };
    const Knob knobs[] = {
        {&gm_options::batch_streams, {1, 16, 64, 256}},
        {&gm_options::waves_per_cu, {0, 12, 8}},
        {&gm_options::stack_layout, {2, 1}},
        {&gm_options::steal_threshold, {32, 128, 512}},
        {&gm_options::merge_ratio, {0, -1, 1, 2, 4}},
        {&gm_options::batch_single_launch, {0, 1}},
    };
    for (const Knob &kb : knobs) {
        const gm_options base = best;
        for (int32_t v : kb.values) {
            if (v == base.*kb.field) continue;  // measured already
            e->opt = base;
            e->opt.*kb.field = v;
            st = run_batch(e, nq, qids, cap, time_limit_s, res.data(), &info);
            if (st) {
                e->opt = saved;
                return st;
            }
            ++trials;
            for (int32_t i = 0; i < nq; ++i) {
                const bool both = ref[i].outcome != GM_TIMEOUT && res[i].outcome != GM_TIMEOUT;
                if (both && (ref[i].count != res[i].count || ref[i].outcome != res[i].outcome)) {
                    e->opt = saved;
                    return e->fail(GM_ERR_STATE, "tuning: query " + std::to_string(qids[i]) +
                                                     " counted differently under two settings");
                }
            }
            if (info.kernel_ms < best_ms) {
                best_ms = info.kernel_ms;
                best = e->opt;
            }
        }
    }
    e->opt = best;
    gm_tuning t{};
    t.waves_per_cu = best.waves_per_cu;
    t.steal_threshold = best.steal_threshold;
    t.stack_layout = best.stack_layout;
    t.batch_single_launch = best.batch_single_launch;
    t.batch_streams = best.batch_streams;
    t.merge_ratio = best.merge_ratio;
    t.trials = trials;
    t.best_ms = best_ms;
    t.default_ms = default_ms;
    if (out) *out = t;
    return GM_OK;
}

// Candidates of a query vertex in G: vertices with its label and at least its
// degree (0 when the label is absent from G); and G's vertices with its label.
uint64_t vertex_candidates(const gm_engine *e, const QueryRec &q, int32_t u, uint64_t *with_label) {
    *with_label = 0;
    auto it = e->label_id.find(q.labels[u]);
    if (it == e->label_id.end() || e->n == 0) return 0;
    const int64_t b = e->lab_start[it->second], en = e->lab_start[it->second + 1];
    *with_label = static_cast<uint64_t>(en - b);
    const uint32_t need = static_cast<uint32_t>(popcount(q.adj[u]));
    auto first = e->bylabel_deg.begin() + b;
    auto pos = std::partition_point(first, e->bylabel_deg.begin() + en, [need](uint32_t d) { return d >= need; });
    return static_cast<uint64_t>(pos - first);
}

void order_features(const gm_engine *e, const QueryRec &q, const int32_t *order, float *out) {
    std::fill(out, out + GM_ORDER_FEATURES, 0.f);
    uint64_t cand[kMaxK], lab[kMaxK];
    for (int32_t u = 0; u < q.k; ++u) cand[u] = vertex_candidates(e, q, u, &lab[u]);
    auto lg = [](uint64_t x) { return static_cast<float>(std::log2(1.0 + static_cast<double>(x))) / 24.f; };
    uint32_t placed = 0;
    int32_t edges = 0;
    for (int32_t i = 0; i < q.k; ++i) {
        const int32_t u = order[i];
        const uint32_t back = q.adj[u] & placed;
        uint64_t best = 0;
        bool any = false;
        for (uint32_t m = back; m; m &= m - 1) {
            const uint64_t c = cand[__builtin_ctz(m)];
            best = any ? std::min(best, c) : c;
            any = true;
        }
        float *f = out + 5 * i;
        f[0] = lg(cand[u]);
        f[1] = static_cast<float>(popcount(q.adj[u])) / 8.f;
        f[2] = static_cast<float>(popcount(back)) / 8.f;
        f[3] = any ? lg(best) : 0.f;
        f[4] = lg(lab[u]);
        placed |= 1u << u;
        edges += popcount(back);
    }
    out[160] = static_cast<float>(q.k) / 32.f;
    out[161] = static_cast<float>(edges) / 64.f;
    out[162] = static_cast<float>(std::log2(static_cast<double>(query_split(e, q)))) / 8.f;
}

// Candidate orders: the heuristic order, the fewest-candidates greedy order,
// then random connected orders, without duplicates.
std::vector<std::vector<int32_t>> candidate_orders(const gm_engine *e, const QueryRec &q, int32_t max_orders,
                                                   uint64_t seed) {
    std::vector<std::vector<int32_t>> out;
    if (max_orders < 1) return out;
    auto add = [&](const std::vector<int32_t> &o) {
        for (const auto &x : out)
            if (x == o) return;
        out.push_back(o);
    };
    add(ri_order(q.k, q.adj));
    uint64_t cand[kMaxK], lab;
    for (int32_t u = 0; u < q.k; ++u) cand[u] = vertex_candidates(e, q, u, &lab);
    {
        std::vector<int32_t> o;
        uint32_t placed = 0;
        for (int32_t i = 0; i < q.k; ++i) {
            int32_t best = -1;
            for (int32_t u = 0; u < q.k; ++u) {
                if ((placed >> u) & 1u) continue;
                if (i > 0 && (q.adj[u] & placed) == 0) continue;
                if (best < 0 || cand[u] < cand[best]) best = u;
            }
            o.push_back(best);
            placed |= 1u << best;
        }
        if (static_cast<int32_t>(out.size()) < max_orders) add(o);
    }
    std::mt19937_64 rng(seed ^ (0x9e3779b97f4a7c15ull * static_cast<uint64_t>(q.k + 1)));
    for (int32_t tries = 0; static_cast<int32_t>(out.size()) < max_orders && tries < 8 * max_orders; ++tries) {
        std::vector<int32_t> o;
        uint32_t placed = 0;
        for (int32_t i = 0; i < q.k; ++i) {
            int32_t pick[kMaxK], np = 0;
            for (int32_t u = 0; u < q.k; ++u)
                if (!((placed >> u) & 1u) && (i == 0 || (q.adj[u] & placed))) pick[np++] = u;
            const int32_t u = pick[rng() % static_cast<uint64_t>(np)];
            o.push_back(u);
            placed |= 1u << u;
        }
        add(o);
    }
    if (static_cast<int32_t>(out.size()) > max_orders) out.resize(static_cast<size_t>(max_orders));
    return out;
}

}  // namespace

// ---------------------------------------------------------------------------
// Serving: a worker thread runs continuous batching over `slots` launch contexts.
// ---------------------------------------------------------------------------
struct gm_server {
    struct Request {
        uint64_t ticket = 0;
        int32_t qid = 0;
        Plan plan{};
        double submit_ms = 0;
    };
    struct Slot {
        LaunchCtx c;
        GroupLaunch gl;
        bool busy = false;
        size_t bytes = 0;       // device memory of its launch's working state
        std::vector<Request> reqs;
        std::vector<Plan> plans;
        std::vector<int32_t> members;
        std::vector<gm_result> res;
        double start_ms = 0;
    };

    gm_engine *e = nullptr;
    gm_serve_options opt{};
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable wake;  // new requests, or stop
    std::condition_variable ready_cv;
    std::deque<Request> pending;
    std::deque<gm_serve_result> ready;
    int64_t running = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    gm_status error = GM_OK;
    std::string err;
    std::thread worker;
    size_t budget = 0;  // device memory of the launches in flight, in bytes
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now_ms() const {
        std::chrono::duration<double, std::milli> d = std::chrono::steady_clock::now() - t0;
        return d.count();
    }
};

namespace {

// Wavefronts of a slot's launch whose largest query has `levels` positions.
int64_t slot_waves(const gm_server *s, int32_t levels) {
    const gm_engine *e = s->e;
    int32_t wpc = s->opt.waves_per_cu;
    if (wpc <= 0)
        wpc = std::max(1, residency(e, levels) / std::max(1, e->num_cu) / static_cast<int32_t>(s->slots.size()));
    return static_cast<int64_t>(e->num_cu) * wpc;
}

// Device memory of a launch's working state: g requests (plan, result block,
// work stream) and, per wavefront, a stealing mailbox and the parked task
// groups of `levels` levels.
size_t launch_state_bytes(const gm_server *s, size_t g, int32_t levels) {
    const bool steal = s->e->opt.disable_stealing == 0;
    const size_t per_wave = (steal ? sizeof(gm::Mailbox) : 0) + static_cast<size_t>(levels) * gm::kWave * sizeof(uint2);
    return g * (sizeof(Plan) + sizeof(gm::QCtl) + sizeof(gm::StreamCtl)) +
           static_cast<size_t>(slot_waves(s, levels)) * per_wave;
}

// Results of a slot's finished (or empty, or failed) launch into the ready queue.
void publish(gm_server *s, gm_server::Slot &sl, double done_ms, int32_t slot_id, gm_status status = GM_OK) {
    for (size_t j = 0; j < sl.reqs.size(); ++j) {
        gm_serve_result r{};
        r.ticket = sl.reqs[j].ticket;
        r.qid = sl.reqs[j].qid;
        r.slot = slot_id;
        r.submit_ms = sl.reqs[j].submit_ms;
        r.start_ms = sl.start_ms;
        r.done_ms = done_ms;
        r.result = sl.res[j];
        r.result.search_ms = done_ms - sl.start_ms;
        r.status = status;
        s->ready.push_back(r);
    }
    s->running -= static_cast<int64_t>(sl.reqs.size());
    sl.reqs.clear();
    sl.busy = false;
    sl.bytes = 0;
}

// A request that never ran (the server failed before admitting it).
void publish_unrun(gm_server *s, const gm_server::Request &q, gm_status status) {
    gm_serve_result r{};
    r.ticket = q.ticket;
    r.qid = q.qid;
    r.slot = -1;
    r.submit_ms = q.submit_ms;
    r.start_ms = r.done_ms = s->now_ms();
    r.status = status;
    s->ready.push_back(r);
}

void serve_loop(gm_server *s) {
    gm_engine *e = s->e;
    (void)hipSetDevice(e->device);
    const int32_t nslots = static_cast<int32_t>(s->slots.size());
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = false;
        // harvest finished launches; a launch whose end event reports an error
        // is finished too, and its requests come back with that error
        for (int32_t i = 0; i < nslots; ++i) {
            gm_server::Slot &sl = s->slots[i];
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.c.ev1);
            if (q == hipErrorNotReady) continue;
            gm_status st = GM_OK;
            if (q != hipSuccess) {
                st = hip_fail(e, q, "server launch");
            } else {
                lk.unlock();
                st = harvest_group(e, sl.c, sl.gl, sl.res.data(), nullptr);
                lk.lock();
            }
            if (st && !s->error) {
                s->error = st;
                s->err = e->last_error();
            }
            publish(s, sl, s->now_ms(), i, st);
            progress = true;
        }
        if (progress) s->ready_cv.notify_all();
        // admit queued requests into free slots, oldest first, while the working
        // state of the launches in flight and of the new one fits the budget
        for (int32_t i = 0; i < nslots && !s->pending.empty() && !s->error; ++i) {
            gm_server::Slot &sl = s->slots[i];
            if (sl.busy) continue;
            size_t inflight = 0;
            for (const gm_server::Slot &x : s->slots) inflight += x.busy ? x.bytes : 0;
            size_t g = 0, bytes = 0;
            int32_t lv = 0;
            while (g < s->pending.size() && g < static_cast<size_t>(s->opt.max_batch)) {
                const int32_t next = std::max(lv, s->pending[g].plan.k);
                const size_t b = launch_state_bytes(s, g + 1, next);
                if (inflight + b > s->budget) break;
                lv = next;
                bytes = b;
                ++g;
            }
            if (g == 0) break;  // the oldest request waits until launches in flight free memory
            sl.reqs.assign(s->pending.begin(), s->pending.begin() + static_cast<long>(g));
            s->pending.erase(s->pending.begin(), s->pending.begin() + static_cast<long>(g));
            s->running += static_cast<int64_t>(g);
            sl.busy = true;
            sl.bytes = bytes;
            sl.start_ms = s->now_ms();
            lk.unlock();
            sl.plans.resize(g);
            sl.members.resize(g);
            sl.res.assign(g, gm_result{});
            int32_t levels = 0;
            for (size_t j = 0; j < g; ++j) {
                sl.plans[j] = sl.reqs[j].plan;
                sl.members[j] = static_cast<int32_t>(j);
                levels = std::max(levels, sl.plans[j].k);
                gm_result &r = sl.res[j];
                r.pool_depth = 1;
                r.pool_rows = sl.plans[j].rows;
                r.outcome = GM_DONE;
            }
            const int32_t wpc = static_cast<int32_t>(slot_waves(s, levels) / std::max(1, e->num_cu));
            const int32_t streams = s->opt.batch_streams > 0 ? s->opt.batch_streams : batch_streams(e);
            const gm_status st = launch_group(e, sl.c, sl.plans, sl.members.data(), static_cast<int32_t>(g), streams,
                                              wpc, sl.gl);
            lk.lock();
            if (st && !s->error) {
                s->error = st;
                s->err = e->last_error();
            }
            if (st || !sl.gl.launched) {  // nothing to run (or a failure): results as they stand
                publish(s, sl, s->now_ms(), i, st);
                s->ready_cv.notify_all();
            }
            progress = true;
        }
        bool busy = false;
        for (const gm_server::Slot &sl : s->slots) busy |= sl.busy;
        if (s->stop && s->pending.empty() && !busy) break;
        if (s->error && !busy) {  // what is still queued comes back with the error
            while (!s->pending.empty()) {
                publish_unrun(s, s->pending.front(), s->error);
                s->pending.pop_front();
            }
            s->ready_cv.notify_all();
            if (s->stop) break;
        }
        if (!progress) {
            if (busy) s->wake.wait_for(lk, std::chrono::microseconds(20));
            else s->wake.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

}  // namespace

extern "C" {

gm_status gm_create(int32_t device, const gm_options *opt, gm_engine **out) {
    if (!out) {
        g_create_error = "out is null";
        return GM_ERR_ARG;
    }
    *out = nullptr;
    if (device < -1) {
        g_create_error = "device must be >= 0, or -1 for a host-only engine";
        return GM_ERR_ARG;
    }
    gm_options o{};
    if (opt) o = *opt;
    if (o.stack_layout < 0 || o.stack_layout > 2 || o.steal_threshold < 0 || o.waves_per_cu < 0 ||
        o.pool_row_limit < 0 || o.batch_single_launch < 0 || o.batch_single_launch > 1 || o.batch_streams < 0 ||
        o.pool_hub_cut < 0 || o.hub_bitmap_mib < 0 || o.candidate_graph < 0 || o.candidate_graph > 1 ||
        o.pool_roots_per_item < 0 || o.pool_roots_per_item > 64 || o.merge_ratio < -1 || o.merge_ratio > 8) {
        g_create_error = "option out of range";
        return GM_ERR_ARG;
    }
    if (o.candidate_graph && (o.tau != 0 || o.stack_layout == 1)) {
        g_create_error = "the candidate graph needs tau = 0 and the slim stack layout";
        return GM_ERR_ARG;
    }
    gm_engine *e = new (std::nothrow) gm_engine();
    if (!e) {
        g_create_error = "out of host memory";
        return GM_ERR_NOMEM;
    }
    e->device = device;
    e->opt = o;
    if (device >= 0) {
        int count = 0;
        hipError_t h = hipGetDeviceCount(&count);
        if (h != hipSuccess || device >= count) {
            g_create_error = std::string("no HIP device ") + std::to_string(device) +
                             (h != hipSuccess ? std::string(": ") + hipGetErrorString(h) : std::string());
            delete e;
            return GM_ERR_DEVICE;
        }
        hipDeviceProp_t prop{};
        int khz = 0;
        if ((h = hipSetDevice(device)) != hipSuccess || (h = hipGetDeviceProperties(&prop, device)) != hipSuccess ||
            (h = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device)) != hipSuccess ||
            (h = ctx_create(e->lc)) != hipSuccess) {
            g_create_error = std::string("HIP setup failed: ") + hipGetErrorString(h);
            gm_destroy(e);
            return GM_ERR_DEVICE;
        }
        e->num_cu = prop.multiProcessorCount;
        e->wall_khz = khz > 0 ? khz : 100000;
        if ((h = gm::scratch_area(device, &e->scratch)) != hipSuccess) {
            g_create_error = std::string("scratch arena lookup failed: ") + hipGetErrorString(h);
            gm_destroy(e);
            return GM_ERR_DEVICE;
        }
    }
    *out = e;
    return GM_OK;
}

void gm_destroy(gm_engine *e) {
    if (!e) return;
    if (e->device >= 0) {
        (void)hipSetDevice(e->device);
        ctx_destroy(e->lc);
        free_graph(e);
        for (int i = 0; i < 2; ++i)
            if (e->d_pool[i]) (void)hipFree(e->d_pool[i]);
        if (e->d_rows) (void)hipFree(e->d_rows);
        for (uint32_t *b : {e->d_vlen, e->d_vstart, e->d_voff, e->d_vtmp})
            if (b) (void)hipFree(b);
        for (int32_t *b : {e->d_cbits, e->d_crank, e->d_ctmp, e->d_clist, e->d_cedges, e->d_gbounds, e->d_gcol,
                           e->d_cmisc})
            if (b) (void)hipFree(b);
    }
    delete e;
}

gm_status gm_load_graph(gm_engine *e, int32_t n, const int64_t *row_ptr, const int32_t *col,
                        const int32_t *labels) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (n < 0) return e->fail(GM_ERR_ARG, "n must be >= 0");
    if (e->opt.candidate_graph && n > kSlimMaxVertices)
        return e->fail(GM_ERR_GRAPH, "the candidate-graph search holds vertex ids in 24 bits: at most 2^24 vertices");
    if (!row_ptr || (n > 0 && !labels)) return e->fail(GM_ERR_ARG, "row_ptr and labels must not be null");
    if (e->servers.load() > 0) return e->fail(GM_ERR_STATE, "a server is open on this engine");
    if (row_ptr[0] != 0) return e->fail(GM_ERR_GRAPH, "row_ptr[0] must be 0");
    const int64_t nnz64 = row_ptr[n];
    if (nnz64 < 0 || nnz64 >= (int64_t(1) << 32))
        return e->fail(GM_ERR_GRAPH, "row_ptr[n] must lie in [0, 2^32): at most 2^32 - 1 adjacency entries");
    if (nnz64 > 0 && !col) return e->fail(GM_ERR_ARG, "col is null");
    if (e->device < 0) {
        // host-only engine: the whole check on the host, then the planning tables
        gm_status st = check_graph(e, n, row_ptr, col, e->opt.skip_symmetry_check == 0);
        if (st) return st;
    } else {
        // the offsets must be sane before they size anything; the rows are checked on the device
        std::atomic<int> bad{0};
        parallel_ranges(n, [&](int64_t b, int64_t en) {
            for (int64_t v = b; v < en; ++v)
                if (row_ptr[v + 1] < row_ptr[v] || row_ptr[v + 1] - row_ptr[v] >= (int64_t(1) << 24)) bad = 1;
        });
        if (bad) return e->fail(GM_ERR_GRAPH, "row_ptr must be non-decreasing with every degree below 2^24");
    }
    HostGraph hg;
    hg.n = n;
    hg.nnz = static_cast<uint64_t>(nnz64);
    gm_status st = compact_labels(e, labels, n, hg);
    if (st) return st;
    hg.deg.resize(static_cast<size_t>(n));
    parallel_ranges(n, [&](int64_t b, int64_t en) {
        for (int64_t v = b; v < en; ++v) hg.deg[v] = static_cast<uint32_t>(row_ptr[v + 1] - row_ptr[v]);
    });
    if (e->device < 0) return install_host_only(e, hg);
    HIP_TRY(e, hipSetDevice(e->device));
    hipStream_t s = e->lc.stream;
    int64_t *d_rp = nullptr;
    int32_t *d_col = nullptr;
    uint8_t *d_clab = nullptr;
    auto release = [&]() {
        if (d_rp) (void)hipFree(d_rp);
        if (d_clab) (void)hipFree(d_clab);
    };
    hipError_t h = hipMalloc(reinterpret_cast<void **>(&d_rp), (static_cast<size_t>(n) + 1) * sizeof(int64_t));
    if (h == hipSuccess)
        h = hipMalloc(reinterpret_cast<void **>(&d_col), std::max<uint64_t>(hg.nnz, gm::kListWindow) * sizeof(int32_t));
    if (h == hipSuccess) h = hipMalloc(reinterpret_cast<void **>(&d_clab), std::max<size_t>(n, 1));
    if (h == hipSuccess) h = hipMemcpyAsync(d_rp, row_ptr, (static_cast<size_t>(n) + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (h == hipSuccess && hg.nnz) h = hipMemcpyAsync(d_col, col, hg.nnz * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (h == hipSuccess && n) h = hipMemcpyAsync(d_clab, hg.clab.data(), static_cast<size_t>(n), hipMemcpyHostToDevice, s);
    if (h != hipSuccess) {
        release();
        if (d_col) (void)hipFree(d_col);
        return e->fail(h == hipErrorOutOfMemory ? GM_ERR_NOMEM : GM_ERR_DEVICE,
                       std::string("graph upload: ") + hipGetErrorString(h));
    }
    st = install_device(e, hg, d_rp, 8, d_col, true, d_clab, s);  // takes d_col
    (void)hipStreamSynchronize(s);
    release();
    return st;
}

gm_status gm_load_graph_device(gm_engine *e, int32_t n, const void *row_ptr, int32_t row_ptr_bytes,
                               const int32_t *col, const uint8_t *labels, void *hip_stream) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->device < 0) return e->fail(GM_ERR_DEVICE, "a host-only engine cannot load device buffers");
    if (n < 0) return e->fail(GM_ERR_ARG, "n must be >= 0");
    if (e->opt.candidate_graph && n > kSlimMaxVertices)
        return e->fail(GM_ERR_GRAPH, "the candidate-graph search holds vertex ids in 24 bits: at most 2^24 vertices");
    if (row_ptr_bytes != 4 && row_ptr_bytes != 8) return e->fail(GM_ERR_ARG, "row_ptr_bytes must be 4 or 8");
    if (!row_ptr || (n > 0 && !labels)) return e->fail(GM_ERR_ARG, "row_ptr and labels must not be null");
    if (e->servers.load() > 0) return e->fail(GM_ERR_STATE, "a server is open on this engine");
    HIP_TRY(e, hipSetDevice(e->device));
    if (!device_buffer(e, row_ptr) || (n > 0 && !device_buffer(e, labels)))
        return e->fail(GM_ERR_ARG, "row_ptr and labels must be device memory of the engine's device");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // the offsets come to the host: they give the degrees and the size of col
    std::vector<int64_t> rp(static_cast<size_t>(n) + 1);
    if (row_ptr_bytes == 8) {
        HIP_TRY(e, hipMemcpyAsync(rp.data(), row_ptr, rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(e, hipStreamSynchronize(s));
    } else {
        std::vector<int32_t> rp32(rp.size());
        HIP_TRY(e, hipMemcpyAsync(rp32.data(), row_ptr, rp32.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(e, hipStreamSynchronize(s));
        for (size_t i = 0; i < rp.size(); ++i) rp[i] = rp32[i];
    }
    if (rp[0] != 0) return e->fail(GM_ERR_GRAPH, "row_ptr[0] must be 0");
    for (int32_t v = 0; v < n; ++v)
        if (rp[v + 1] < rp[v] || rp[v + 1] - rp[v] >= (int64_t(1) << 24))
            return e->fail(GM_ERR_GRAPH, "row_ptr must be non-decreasing with every degree below 2^24");
    if (rp[n] >= (int64_t(1) << 32)) return e->fail(GM_ERR_GRAPH, "at most 2^32 - 1 adjacency entries");
    HostGraph hg;
    hg.n = n;
    hg.nnz = static_cast<uint64_t>(rp[n]);
    if (hg.nnz > 0 && (!col || !device_buffer(e, col)))
        return e->fail(GM_ERR_ARG, "col must be device memory of the engine's device");
    hg.deg.resize(static_cast<size_t>(n));
    for (int32_t v = 0; v < n; ++v) hg.deg[v] = static_cast<uint32_t>(rp[v + 1] - rp[v]);
    // labels: a histogram on the device gives the values present; compact ids in value order
    unsigned int *d_hist = nullptr;
    uint8_t *d_clab = nullptr;
    auto release = [&]() {
        if (d_hist) (void)hipFree(d_hist);
        if (d_clab) (void)hipFree(d_clab);
    };
    hipError_t h = hipMalloc(reinterpret_cast<void **>(&d_hist), 256 * sizeof(unsigned int));
    if (h == hipSuccess) h = hipMalloc(reinterpret_cast<void **>(&d_clab), std::max<size_t>(n, 1));
    if (h == hipSuccess) h = hipMemsetAsync(d_hist, 0, 256 * sizeof(unsigned int), s);
    if (h == hipSuccess) h = gm::launch_label_hist(labels, n, d_hist, e->num_cu, s);
    unsigned int hist[256] = {};
    if (h == hipSuccess) h = hipMemcpyAsync(hist, d_hist, sizeof(hist), hipMemcpyDeviceToHost, s);
    if (h == hipSuccess) h = hipStreamSynchronize(s);
    uint8_t map[256] = {};
    int32_t used = 0;
    for (int32_t c = 0; c < 256 && h == hipSuccess; ++c) {
        if (!hist[c]) continue;
        if (used >= 255) {
            release();
            return e->fail(GM_ERR_GRAPH, "more than 255 distinct vertex labels");
        }
        map[c] = static_cast<uint8_t>(used);
        hg.ids.emplace(c, used++);
    }
    hg.labels_used = used;
    hg.clab.resize(static_cast<size_t>(n));
    if (h == hipSuccess) h = gm::launch_label_map(labels, n, map, d_clab, e->num_cu, s);
    if (h == hipSuccess && n) h = hipMemcpyAsync(hg.clab.data(), d_clab, static_cast<size_t>(n), hipMemcpyDeviceToHost, s);
    if (h == hipSuccess) h = hipStreamSynchronize(s);
    if (h != hipSuccess) {
        release();
        return hip_fail(e, h, "label compaction");
    }
    // the membership test reads windows of gm::kListWindow entries: a shorter array
    // is copied into one of the engine's own that long
    int32_t *d_col = const_cast<int32_t *>(col);
    bool owned = false;
    if (hg.nnz < gm::kListWindow) {
        h = hipMalloc(reinterpret_cast<void **>(&d_col), gm::kListWindow * sizeof(int32_t));
        if (h == hipSuccess) {
            owned = true;
            h = hipMemsetAsync(d_col, 0, gm::kListWindow * sizeof(int32_t), s);
        }
        if (h == hipSuccess && hg.nnz)
            h = hipMemcpyAsync(d_col, col, hg.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
        if (h != hipSuccess) {
            if (owned) (void)hipFree(d_col);
            release();
            return hip_fail(e, h, "adjacency copy");
        }
    }
    gm_status st = install_device(e, hg, row_ptr, row_ptr_bytes, d_col, owned, d_clab, s);
    (void)hipStreamSynchronize(s);
    release();
    return st;
}

gm_status gm_load_query(gm_engine *e, int32_t k, int32_t m, const int32_t *edges, const int32_t *labels,
                        int32_t *qid_out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!qid_out || !labels || (m > 0 && !edges)) return e->fail(GM_ERR_ARG, "null argument");
    if (k < 1 || k > kMaxK) return e->fail(GM_ERR_QUERY, "query must have 1..32 vertices");
    if (m < 0) return e->fail(GM_ERR_QUERY, "negative edge count");
    QueryRec q;
    q.live = true;
    q.k = k;
    q.labels.assign(labels, labels + k);
    for (int32_t i = 0; i < m; ++i) {
        const int32_t a = edges[2 * i], b = edges[2 * i + 1];
        if (a < 0 || a >= k || b < 0 || b >= k || a == b)
            return e->fail(GM_ERR_QUERY, "query edge " + std::to_string(i) + " is a self-loop or out of range");
        if ((q.adj[a] >> b) & 1u) return e->fail(GM_ERR_QUERY, "duplicate query edge " + std::to_string(i));
        q.adj[a] |= 1u << b;
        q.adj[b] |= 1u << a;
    }
    // connectivity: grow from vertex 0
    uint32_t seen = 1u, frontier = 1u;
    while (frontier) {
        uint32_t next = 0;
        for (uint32_t f = frontier; f; f &= f - 1) next |= q.adj[__builtin_ctz(f)];
        frontier = next & ~seen;
        seen |= next;
    }
    const uint32_t all = k == 32 ? 0xffffffffu : ((1u << k) - 1u);
    if (seen != all) return e->fail(GM_ERR_QUERY, "query graph is not connected");
    q.order = ri_order(k, q.adj);
    *qid_out = static_cast<int32_t>(e->queries.size());
    e->queries.push_back(std::move(q));
    return GM_OK;
}

gm_status gm_set_order(gm_engine *e, int32_t qid, const int32_t *order) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    const QueryRec *cq = nullptr;
    gm_status st = get_query(e, qid, &cq);
    if (st) return st;
    QueryRec &q = e->queries[qid];
    if (!order) {
        q.order = ri_order(q.k, q.adj);
        return GM_OK;
    }
    if (!connected_order(q.k, q.adj, order))
        return e->fail(GM_ERR_ORDER, "order must be a permutation where each vertex after the first has an earlier neighbour");
    q.order.assign(order, order + q.k);
    return GM_OK;
}

gm_status gm_get_order(const gm_engine *e, int32_t qid, int32_t *order_out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!order_out) return e->fail(GM_ERR_ARG, "order_out is null");
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    std::copy(q->order.begin(), q->order.end(), order_out);
    return GM_OK;
}

gm_status gm_count(gm_engine *e, int32_t qid, uint64_t cap, double time_limit_s, gm_result *out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!out) return e->fail(GM_ERR_ARG, "out is null");
    return run_search(e, qid, cap, time_limit_s, nullptr, out);
}

gm_status gm_enumerate(gm_engine *e, int32_t qid, int32_t *rows, uint64_t cap, double time_limit_s,
                       gm_result *out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!out) return e->fail(GM_ERR_ARG, "out is null");
    if (!rows || cap == 0) return e->fail(GM_ERR_BUFFER, "enumerate needs a row buffer and cap >= 1");
    return run_search(e, qid, cap, time_limit_s, rows, out);
}

gm_status gm_count_batch(gm_engine *e, int32_t nq, const int32_t *qids, uint64_t cap, double time_limit_s,
                         gm_result *out, gm_batch_info *info) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->opt.candidate_graph)
        return e->fail(GM_ERR_STATE, "the candidate graph is built per query: use gm_count or gm_enumerate");
    return run_batch(e, nq, qids, cap, time_limit_s, out, info);
}

gm_status gm_count_noalloc(gm_engine *e, int32_t qid, uint64_t cap, double time_limit_s, gm_result *out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!out) return e->fail(GM_ERR_ARG, "out is null");
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    if (!e->has_graph) return e->fail(GM_ERR_STATE, "no data graph loaded");
    if (e->device < 0) return e->fail(GM_ERR_DEVICE, "host-only engine (created with device -1) cannot search");
    if (e->opt.candidate_graph) return e->fail(GM_ERR_STATE, "the candidate graph is built per call; it allocates");
    if (!e->scratch) return e->fail(GM_ERR_DEVICE, "no scratch arena on this device");
    HIP_TRY(e, hipSetDevice(e->device));
    const auto t_start = std::chrono::steady_clock::now();
    std::memset(out, 0, sizeof(*out));
    // the plan of gm_count_batch for one query: first-vertex candidates as the pool
    bool missing = false;
    Plan p = make_plan(e, *q, &missing);
    p.cap = cap;
    p.flush = flush_for_cap(e, cap);
    p.depth = 1;
    p.budget = time_limit_s > 0 ? std::max<unsigned long long>(1, static_cast<unsigned long long>(
                                                                       time_limit_s * 1000.0 * static_cast<double>(e->wall_khz)))
                                : 0ull;
    if (!missing) root_share(e, p, &p.row0, &p.rows);
    p.perm_mul = root_order(p.rows);
    p.item0 = 0;
    p.item_end = items_of(p.rows);
    out->pool_depth = 1;
    out->pool_rows = p.rows;
    out->outcome = GM_DONE;
    auto elapsed_ms = [&]() {
        std::chrono::duration<double, std::milli> el = std::chrono::steady_clock::now() - t_start;
        return el.count();
    };
    if (p.item_end == 0) {  // no candidate for the first query vertex: no match, no launch
        out->search_ms = elapsed_ms();
        return GM_OK;
    }
    // arena layout: control block, plan, result block, work stream, idle bitmap,
    // then per wavefront a mailbox (with stealing) and its parked task groups
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const bool steal = e->opt.disable_stealing == 0;
    const size_t off_plan = up(sizeof(Control));
    const size_t off_qctl = off_plan + up(sizeof(Plan));
    const size_t off_sc = off_qctl + up(sizeof(gm::QCtl));
    const size_t off_idle = off_sc + up(sizeof(gm::StreamCtl));
    const size_t max_waves = static_cast<size_t>(e->num_cu) * 32;
    const size_t off_mail = off_idle + up((max_waves + 63) / 64 * sizeof(unsigned long long));
    const size_t per_wave = (steal ? sizeof(gm::Mailbox) : 0) + static_cast<size_t>(p.k) * gm::kWave * sizeof(uint2);
    if (off_mail + per_wave > gm::kScratchBytes)
        return e->fail(GM_ERR_BUFFER, "the scratch arena (" + std::to_string(gm::kScratchBytes >> 20) +
                                          " MiB) cannot hold the state of one wavefront");
    const size_t fit = (gm::kScratchBytes - off_mail) / per_wave;
    const int32_t waves = static_cast<int32_t>(std::min<size_t>({fit, max_waves}));
    const size_t off_parked = up(off_mail + (steal ? static_cast<size_t>(waves) * sizeof(gm::Mailbox) : 0));
    if (off_parked + static_cast<size_t>(waves) * p.k * gm::kWave * sizeof(uint2) > gm::kScratchBytes)
        return e->fail(GM_ERR_BUFFER, "scratch arena layout overflow");
    uint8_t *base = static_cast<uint8_t *>(e->scratch);
    hipStream_t s = e->lc.stream;
    gm::StreamCtl sc{};
    sc.items = p.item_end;
    sc.plan0 = 0;
    sc.plan1 = 1;
    // the previous call's contents stay in the arena: the counters start at zero
    HIP_TRY(e, gm::launch_zero_words(base, off_idle / 4, s));
    HIP_TRY(e, hipMemcpyAsync(base + off_plan, &p, sizeof(Plan), hipMemcpyHostToDevice, s));
    HIP_TRY(e, hipMemcpyAsync(base + off_sc, &sc, sizeof(gm::StreamCtl), hipMemcpyHostToDevice, s));
    SearchArgs a = graph_args(e, e->lc);
    a.ctl = reinterpret_cast<Control *>(base);
    a.plans = reinterpret_cast<Plan *>(base + off_plan);
    a.qctl = reinterpret_cast<gm::QCtl *>(base + off_qctl);
    a.streams = reinterpret_cast<gm::StreamCtl *>(base + off_sc);
    a.nq = 1;
    a.nstreams = 1;
    a.levels = p.k;
    a.pool = e->d_bylabel;
    a.slim = use_slim(e, p.k) ? 1 : 0;
    a.sb = has_sb(p) ? 1 : 0;
    a.budget = 0;  // the limit is the query's own (plan budget)
    a.steal_threshold = e->opt.steal_threshold > 0 ? e->opt.steal_threshold : 128;
    a.mail = steal ? reinterpret_cast<gm::Mailbox *>(base + off_mail) : nullptr;
    a.idle_bits = steal ? reinterpret_cast<unsigned long long *>(base + off_idle) : nullptr;
    a.steal_slots = steal ? waves : 0;
    a.parked = reinterpret_cast<uint2 *>(base + off_parked);
    a.park_waves = waves;
    if (steal) HIP_TRY(e, gm::launch_steal_init(a.mail, a.idle_bits, waves, s));
    HIP_TRY(e, gm::launch_start_clock(a.ctl, s));
    int grid_waves = 0;
    HIP_TRY(e, hipEventRecord(e->lc.ev0, s));
    HIP_TRY(e, gm::launch_search(a, false, e->num_cu, e->opt.waves_per_cu, s, &grid_waves));
    HIP_TRY(e, hipEventRecord(e->lc.ev1, s));
    gm::QCtl qc{};
    Control c{};
    HIP_TRY(e, hipMemcpyAsync(&qc, a.qctl, sizeof(gm::QCtl), hipMemcpyDeviceToHost, s));
    HIP_TRY(e, hipMemcpyAsync(&sc, a.streams, sizeof(gm::StreamCtl), hipMemcpyDeviceToHost, s));
    HIP_TRY(e, hipMemcpyAsync(&c, a.ctl, sizeof(Control), hipMemcpyDeviceToHost, s));
    HIP_TRY(e, hipStreamSynchronize(s));
    float kernel_ms = 0.f;
    HIP_TRY(e, hipEventElapsedTime(&kernel_ms, e->lc.ev0, e->lc.ev1));
    if (p.cap && qc.count >= p.cap) {
        out->count = p.cap;
        out->outcome = GM_CAPPED;
    } else {
        out->count = qc.count;
        out->outcome = qc.abort != gm::kAbortTime && query_finished(p, qc, sc) ? GM_DONE : GM_TIMEOUT;
    }
    out->groups = out->kernel_groups = qc.groups;
    out->tasks = out->kernel_tasks = qc.tasks;
    out->lanes_active = qc.lanes_active;
    out->lanes_issued = qc.lanes_issued;
    out->probes = out->kernel_probes = qc.probes;
    out->steals = qc.steals;
    out->scanned = out->kernel_scanned = qc.scanned;
    out->kernel_lookups = qc.lookups;
    out->kernel_bytes = qc.bytes;
    out->kernel_bytes_late = qc.bytes_late;
    out->kernel_ms = kernel_ms;
    out->grid_waves = grid_waves;
    out->search_ms = elapsed_ms();
    return GM_OK;
}

gm_status gm_tune_batch(gm_engine *e, int32_t nq, const int32_t *qids, uint64_t cap, double time_limit_s,
                        gm_tuning *out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!out) return e->fail(GM_ERR_ARG, "out is null");
    if (e->servers.load() > 0) return e->fail(GM_ERR_STATE, "a server is open on this engine");
    if (e->opt.candidate_graph)
        return e->fail(GM_ERR_STATE, "the candidate graph is built per query: use gm_count or gm_enumerate");
    return run_tune(e, nq, qids, cap, time_limit_s, out);
}

gm_status gm_candidate_sets(gm_engine *e, int32_t qid, uint32_t *bits, uint64_t *edges_out, int32_t *rounds_out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!bits) return e->fail(GM_ERR_ARG, "bits is null");
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    if (!e->has_graph) return e->fail(GM_ERR_STATE, "no data graph loaded");
    if (e->device < 0) return e->fail(GM_ERR_DEVICE, "host-only engine (created with device -1) cannot search");
    HIP_TRY(e, hipSetDevice(e->device));
    const size_t W = (static_cast<size_t>(e->n) + 31) / 32;
    std::memset(bits, 0, W * q->k * sizeof(uint32_t));
    if (edges_out) *edges_out = 0;
    if (rounds_out) *rounds_out = 0;
    bool label_missing = false;
    Plan p = make_plan(e, *q, &label_missing);
    if (e->n == 0 || label_missing) return GM_OK;  // some query label is not in G: every set is empty
    CandInfo ci;
    st = build_candidate_graph(e, p, &ci, p.gslot);
    if (st) return st;
    const unsigned long long wp = gm::cand_bitmap_words(e->n);
    for (int l = 0; l < q->k; ++l)
        HIP_TRY(e, hipMemcpyAsync(bits + static_cast<size_t>(p.phi[l]) * W, e->d_cbits + static_cast<size_t>(l) * wp,
                                  W * sizeof(uint32_t), hipMemcpyDeviceToHost, e->lc.stream));
    HIP_TRY(e, hipStreamSynchronize(e->lc.stream));
    if (edges_out) *edges_out = ci.edges;
    if (rounds_out) *rounds_out = ci.rounds;
    return GM_OK;
}

gm_status gm_get_options(const gm_engine *e, gm_options *out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!out) return e->fail(GM_ERR_ARG, "out is null");
    *out = e->opt;
    return GM_OK;
}

gm_status gm_serve_open(gm_engine *e, const gm_serve_options *opt, gm_server **out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!out) return e->fail(GM_ERR_ARG, "out is null");
    *out = nullptr;
    gm_serve_options o{};
    if (opt) o = *opt;
    if (o.slots < 0 || o.slots > 16 || o.max_batch < 0 || o.waves_per_cu < 0 || o.batch_streams < 0 ||
        o.max_pending < 0 || o.memory_mib < 0)
        return e->fail(GM_ERR_ARG, "serve option out of range");
    if (!e->has_graph) return e->fail(GM_ERR_STATE, "no data graph loaded");
    if (e->device < 0) return e->fail(GM_ERR_DEVICE, "host-only engine (created with device -1) cannot serve");
    if (e->opt.candidate_graph)
        return e->fail(GM_ERR_STATE, "the candidate graph is built per query: use gm_count or gm_enumerate");
    if (o.slots == 0) o.slots = 2;
    if (o.max_batch == 0) o.max_batch = 256;
    HIP_TRY(e, hipSetDevice(e->device));
    gm_server *s = new (std::nothrow) gm_server();
    if (!s) return e->fail(GM_ERR_NOMEM, "out of host memory");
    s->e = e;
    s->opt = o;
    s->budget = static_cast<size_t>(o.memory_mib > 0 ? o.memory_mib : 1024) << 20;
    s->slots.resize(static_cast<size_t>(o.slots));
    for (gm_server::Slot &sl : s->slots) {
        const hipError_t h = ctx_create(sl.c);
        if (h != hipSuccess) {
            for (gm_server::Slot &x : s->slots) ctx_destroy(x.c);
            delete s;
            return hip_fail(e, h, "server slot setup");
        }
    }
    e->servers.fetch_add(1);
    s->worker = std::thread(serve_loop, s);
    *out = s;
    return GM_OK;
}

gm_status gm_serve_submit(gm_server *s, int32_t qid, uint64_t cap, double time_limit_s, uint64_t *ticket) {
    if (!s) return GM_ERR_ARG;
    gm_engine *e = s->e;
    if (!ticket) return e->fail(GM_ERR_ARG, "ticket is null");
    gm_server::Request r;
    r.qid = qid;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        const QueryRec *q = nullptr;
        gm_status st = get_query(e, qid, &q);
        if (st) return st;
        bool missing = false;
        Plan p = make_plan(e, *q, &missing);
        p.cap = cap;
        p.flush = flush_for_cap(e, cap);
        p.depth = 1;
        if (time_limit_s > 0)
            p.budget = std::max<unsigned long long>(
                1, static_cast<unsigned long long>(time_limit_s * 1000.0 * static_cast<double>(e->wall_khz)));
        if (!missing) root_share(e, p, &p.row0, &p.rows);
        p.perm_mul = root_order(p.rows);
        r.plan = p;
        const size_t need = launch_state_bytes(s, 1, p.k);
        if (need > s->budget)
            return e->fail(GM_ERR_BUFFER, "request needs " + std::to_string(need >> 20) + " MiB of launch state, "
                                              "more than the server's memory budget of " +
                                              std::to_string(s->budget >> 20) + " MiB");
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->error) return e->fail(s->error, "server failed earlier: " + s->err);
        if (s->opt.max_pending && static_cast<int64_t>(s->pending.size()) >= s->opt.max_pending)
            return e->fail(GM_ERR_BUFFER, "server queue is full");
        r.ticket = s->next_ticket++;
        r.submit_ms = s->now_ms();
        *ticket = r.ticket;
        s->pending.push_back(r);
    }
    s->wake.notify_one();
    return GM_OK;
}

gm_status gm_serve_poll(gm_server *s, gm_serve_result *out, int32_t max_results, double wait_s, int32_t *n_out) {
    if (!s) return GM_ERR_ARG;
    if (!n_out || max_results < 0 || (max_results > 0 && !out)) return s->e->fail(GM_ERR_ARG, "bad poll arguments");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->ready.empty() && wait_s > 0)
        s->ready_cv.wait_for(lk, std::chrono::duration<double>(wait_s), [s] { return !s->ready.empty() || s->error; });
    int32_t n = 0;
    while (n < max_results && !s->ready.empty()) {
        out[n++] = s->ready.front();
        s->ready.pop_front();
    }
    *n_out = n;
    if (s->error && n == 0) return s->e->fail(s->error, "server failed: " + s->err);
    return GM_OK;
}

gm_status gm_serve_request_bytes(gm_server *s, int32_t qid, int64_t *bytes) {
    if (!s) return GM_ERR_ARG;
    gm_engine *e = s->e;
    if (!bytes) return e->fail(GM_ERR_ARG, "bytes is null");
    std::lock_guard<std::mutex> lk(e->mu);
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    *bytes = static_cast<int64_t>(launch_state_bytes(s, 1, q->k));
    return GM_OK;
}

gm_status gm_serve_stats(gm_server *s, int64_t *pending, int64_t *running, int64_t *ready) {
    if (!s) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (pending) *pending = static_cast<int64_t>(s->pending.size());
    if (running) *running = s->running;
    if (ready) *ready = static_cast<int64_t>(s->ready.size());
    return GM_OK;
}

gm_status gm_serve_close(gm_server *s) {
    if (!s) return GM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->wake.notify_all();
    if (s->worker.joinable()) s->worker.join();
    gm_engine *e = s->e;
    (void)hipSetDevice(e->device);
    for (gm_server::Slot &sl : s->slots) ctx_destroy(sl.c);
    const gm_status st = s->error;
    e->servers.fetch_sub(1);
    delete s;
    return st;
}

gm_status gm_order_features(gm_engine *e, int32_t qid, const int32_t *order, float *out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!out) return e->fail(GM_ERR_ARG, "out is null");
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    if (!e->has_graph) return e->fail(GM_ERR_STATE, "no data graph loaded");
    if (order && !connected_order(q->k, q->adj, order))
        return e->fail(GM_ERR_ORDER, "order must be a connected permutation");
    order_features(e, *q, order ? order : q->order.data(), out);
    return GM_OK;
}

gm_status gm_candidate_orders(gm_engine *e, int32_t qid, int32_t max_orders, uint64_t seed, int32_t *orders,
                              int32_t *n_out) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!orders || !n_out || max_orders < 1) return e->fail(GM_ERR_ARG, "bad arguments");
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    if (!e->has_graph) return e->fail(GM_ERR_STATE, "no data graph loaded");
    const auto cands = candidate_orders(e, *q, max_orders, seed);
    for (size_t i = 0; i < cands.size(); ++i) std::copy(cands[i].begin(), cands[i].end(), orders + i * q->k);
    *n_out = static_cast<int32_t>(cands.size());
    return GM_OK;
}

gm_status gm_choose_order(gm_engine *e, gm_model *model, int32_t qid, int32_t max_orders, uint64_t seed, float margin,
                          int32_t *chosen, float *predicted) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!model || !chosen || max_orders < 1) return e->fail(GM_ERR_ARG, "bad arguments");
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    if (!e->has_graph) return e->fail(GM_ERR_STATE, "no data graph loaded");
    const auto cands = candidate_orders(e, *q, max_orders, seed);
    std::vector<float> x(cands.size() * GM_ORDER_FEATURES), y(cands.size());
    for (size_t i = 0; i < cands.size(); ++i) order_features(e, *q, cands[i].data(), x.data() + i * GM_ORDER_FEATURES);
    st = gm_model_predict(model, x.data(), static_cast<int32_t>(cands.size()), GM_ORDER_FEATURES, y.data());
    if (st) return e->fail(st, std::string("model: ") + gm_model_last_error(model));
    size_t best = 0;
    for (size_t i = 1; i < cands.size(); ++i)
        if (y[i] < y[best]) best = i;
    if (!(y[best] < y[0] - margin)) best = 0;  // keep the heuristic order unless clearly beaten
    e->queries[qid].order = cands[best];
    *chosen = static_cast<int32_t>(best);
    if (predicted) std::copy(y.begin(), y.end(), predicted);
    return GM_OK;
}

gm_status gm_set_split(gm_engine *e, int32_t qid, int32_t split) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (split < 0 || split > (1 << 24)) return e->fail(GM_ERR_ARG, "split must lie in [0, 2^24]");
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    e->queries[qid].split = split;
    return GM_OK;
}

gm_status gm_get_split(const gm_engine *e, int32_t qid, int32_t *split) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!split) return e->fail(GM_ERR_ARG, "split is null");
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    *split = query_split(e, *q);
    return GM_OK;
}

gm_status gm_choose_plan(gm_engine *e, gm_model *model, int32_t qid, int32_t max_orders, uint64_t seed,
                         const int32_t *splits, int32_t nsplits, float margin, uint64_t probe_cap,
                         double probe_limit_s, int32_t *chosen_order, int32_t *chosen_split, float *predicted,
                         double *probe_ms) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (!model || !chosen_order || !chosen_split || max_orders < 1 || nsplits < 1 || !splits)
        return e->fail(GM_ERR_ARG, "bad arguments");
    for (int32_t j = 0; j < nsplits; ++j)
        if (splits[j] < 1 || splits[j] > (1 << 24)) return e->fail(GM_ERR_ARG, "splits must lie in [1, 2^24]");
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    if (!e->has_graph) return e->fail(GM_ERR_STATE, "no data graph loaded");
    QueryRec &rec = e->queries[qid];
    const int32_t split0 = query_split(e, rec);  // the fallback keeps the current split
    const auto cands = candidate_orders(e, *q, max_orders, seed);
    // candidate 0: heuristic order with the current split; then every (order, split) pair
    std::vector<std::pair<int32_t, int32_t>> plan{{0, split0}};
    for (int32_t o = 0; o < static_cast<int32_t>(cands.size()); ++o)
        for (int32_t j = 0; j < nsplits; ++j)
            if (!(o == 0 && splits[j] == split0)) plan.emplace_back(o, splits[j]);
    std::vector<float> x(plan.size() * GM_ORDER_FEATURES), y(plan.size());
    const int32_t saved = rec.split;
    for (size_t i = 0; i < plan.size(); ++i) {
        rec.split = plan[i].second;
        order_features(e, rec, cands[plan[i].first].data(), x.data() + i * GM_ORDER_FEATURES);
    }
    rec.split = saved;
    st = gm_model_predict(model, x.data(), static_cast<int32_t>(plan.size()), GM_ORDER_FEATURES, y.data());
    if (st) return e->fail(st, std::string("model: ") + gm_model_last_error(model));
    size_t best = 0;
    for (size_t i = 1; i < plan.size(); ++i)
        if (y[i] < y[best]) best = i;
    if (!(y[best] < y[0] - margin)) best = 0;  // keep the heuristic plan unless clearly beaten
    if (predicted) std::copy(y.begin(), y.end(), predicted);
    if (probe_ms) *probe_ms = 0.0;
    if (best != 0 && probe_cap > 0) {
        // measured runtime as the judge: both plans counted up to probe_cap; the
        // model's plan is kept only if it reached that point faster
        if (e->device < 0) return e->fail(GM_ERR_DEVICE, "host-only engine cannot measure plans");
        const std::vector<int32_t> order0 = rec.order;
        double ms[2] = {0.0, 0.0};
        for (int32_t which = 0; which < 2; ++which) {
            const size_t c = which == 0 ? 0 : best;
            rec.order = cands[plan[c].first];
            rec.split = c == 0 ? saved : plan[c].second;
            gm_result r{};
            st = run_search(e, qid, probe_cap, probe_limit_s, nullptr, &r);
            if (st) {
                rec.order = order0;
                rec.split = saved;
                return st;
            }
            ms[which] = r.search_ms;
        }
        if (probe_ms) *probe_ms = ms[0] + ms[1];
        if (!(ms[1] < ms[0])) best = 0;
    }
    rec.order = cands[plan[best].first];
    rec.split = best == 0 ? saved : plan[best].second;
    *chosen_order = plan[best].first;
    *chosen_split = plan[best].second;
    return GM_OK;
}

gm_status gm_set_symmetry_breaking(gm_engine *e, int32_t qid, int32_t enable, uint64_t *aut_size) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    const QueryRec *cq = nullptr;
    gm_status st = get_query(e, qid, &cq);
    if (st) return st;
    QueryRec &q = e->queries[qid];
    if (!symmetry_conditions(q)) {
        q.sb = false;
        std::fill(q.less, q.less + kMaxK, 0u);
        return e->fail(GM_ERR_QUERY, "automorphism search of the query exceeded its budget");
    }
    q.sb = enable != 0;
    if (aut_size) *aut_size = q.aut;
    return GM_OK;
}

gm_status gm_free_query(gm_engine *e, int32_t qid) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    const QueryRec *q = nullptr;
    gm_status st = get_query(e, qid, &q);
    if (st) return st;
    e->queries[qid] = QueryRec();
    return GM_OK;
}

const char *gm_last_error(const gm_engine *e) {
    if (!e) return g_create_error.c_str();
    thread_local std::string copy;  // valid until this thread's next call
    copy = e->last_error();
    return copy.c_str();
}

}  // extern "C"
