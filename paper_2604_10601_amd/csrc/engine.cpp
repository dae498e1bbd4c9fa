// Host side of the C ABI declared in include/gmatch.h: input checks, the
// matching-order plan, device buffers and the launch sequence of one search
// (root candidates -> breadth-first pool up to tau -> persistent depth-first
// search), following Alg. 2 of the gMatch paper.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
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

struct QueryRec {
    bool live = false;
    int32_t k = 0;
    std::vector<int32_t> labels;
    uint32_t adj[kMaxK] = {};
    std::vector<int32_t> order;
};

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
    int32_t *d_lcol = nullptr;     // lists ordered by (label, id); aliases d_col when not partitioned
    uint32_t *d_loff = nullptr;    // label slice bounds
    int32_t loff_stride = 1;
    std::unordered_map<int32_t, int32_t> label_id;  // G's label value -> compact id

    std::vector<QueryRec> queries;

    int32_t *d_pool[2] = {nullptr, nullptr};
    size_t pool_cap[2] = {0, 0};  // in int32
    int32_t *d_rows = nullptr;
    size_t rows_cap = 0;           // in int32
    Control *d_ctl = nullptr;
    gm::Mailbox *d_mail = nullptr;
    unsigned long long *d_idle_bits = nullptr;
    int32_t steal_slots = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int num_cu = 0;
    long long wall_khz = 0;

    gm_status fail(gm_status s, const std::string &msg) const {
        err = msg;
        return s;
    }
};

namespace {

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
        hipFree(*buf);
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

void free_graph(gm_engine *e) {
    if (e->d_vinfo) hipFree(e->d_vinfo);
    if (e->d_lcol && e->d_lcol != e->d_col) hipFree(e->d_lcol);
    if (e->d_col) hipFree(e->d_col);
    if (e->d_loff) hipFree(e->d_loff);
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
bool use_slim(const gm_engine *e, int32_t k) {
    (void)k;
    return e->opt.stack_layout != 1;
}

// tau (Sec. 4.3): the option, or by default one full batch of 64 pool rows for
// every wavefront the search launch keeps resident (about 2.5e5 on MI355X).
int64_t option_tau(const gm_engine *e, int32_t k) {
    if (e->opt.tau != 0) return e->opt.tau;
    return 64LL * gm::search_waves(k, e->num_cu, e->opt.waves_per_cu, use_slim(e, k));
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

gm_status get_query(const gm_engine *e, int32_t qid, const QueryRec **q) {
    if (qid < 0 || qid >= static_cast<int32_t>(e->queries.size()) || !e->queries[qid].live)
        return e->fail(GM_ERR_STATE, "unknown or freed query id " + std::to_string(qid));
    *q = &e->queries[qid];
    return GM_OK;
}

gm_status read_ctl(gm_engine *e, Control *host) {
    HIP_TRY(e, hipMemcpyAsync(host, e->d_ctl, sizeof(Control), hipMemcpyDeviceToHost, e->stream));
    HIP_TRY(e, hipStreamSynchronize(e->stream));
    return GM_OK;
}

// Empty idle bitmap and mailboxes, zero busy and idle counts before a launch that steals.
gm_status reset_stealing(gm_engine *e, const SearchArgs &a) {
    if (!a.mail) return GM_OK;
    HIP_TRY(e, hipMemsetAsync(&e->d_ctl->busy, 0, sizeof(int), e->stream));
    HIP_TRY(e, hipMemsetAsync(&e->d_ctl->idle_count, 0, sizeof(int), e->stream));
    HIP_TRY(e, gm::launch_steal_init(a.mail, a.idle_bits, a.steal_slots, e->stream));
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

    Plan plan{};
    plan.k = q->k;
    bool label_missing = false;
    for (int32_t i = 0; i < q->k; ++i) {
        const int32_t u = q->order[i];
        plan.phi[i] = u;
        auto it = e->label_id.find(q->labels[u]);
        plan.lab[i] = it == e->label_id.end() ? 255 : it->second;
        label_missing |= it == e->label_id.end();
        plan.qdeg[i] = popcount(q->adj[u]);
        uint32_t b = 0;
        for (int32_t j = 0; j < i; ++j)
            if ((q->adj[u] >> q->order[j]) & 1u) b |= 1u << j;
        plan.bwd[i] = b;
    }
    const bool enumerate = rows != nullptr;
    if (label_missing || e->n == 0) {
        out->outcome = GM_DONE;
        return GM_OK;
    }

    const auto t_start = std::chrono::steady_clock::now();
    const long long budget_ticks =
        time_limit_s > 0 ? static_cast<long long>(time_limit_s * 1000.0 * static_cast<double>(e->wall_khz)) : 0;
    auto timed_out_host = [&]() {
        if (time_limit_s <= 0) return false;
        std::chrono::duration<double> el = std::chrono::steady_clock::now() - t_start;
        return el.count() > time_limit_s;
    };

    HIP_TRY(e, hipMemsetAsync(e->d_ctl, 0, sizeof(Control), e->stream));
    st = ensure_buffer(e, &e->d_pool[0], &e->pool_cap[0], static_cast<size_t>(e->n));
    if (st) return st;
    // the root scan also bounds the next level: each root's label slice for position 1
    const int32_t lab1 = q->k >= 2 ? (e->loff_stride > 1 ? plan.lab[1] : 0) : -1;
    HIP_TRY(e, gm::launch_root_scan(e->d_vinfo, e->n, plan.lab[0], plan.qdeg[0], e->d_pool[0], e->d_loff,
                                    e->loff_stride, lab1, e->d_ctl, e->num_cu, e->stream));
    Control c{};
    st = read_ctl(e, &c);
    if (st) return st;
    uint64_t pool_rows = c.out_rows;
    uint64_t bound = c.measure;  // upper bound on the rows of the next level
    int cur = 0;
    int32_t depth = 1;

    SearchArgs a{};
    a.vinfo = e->d_vinfo;
    a.col = e->d_col;
    a.lcol = e->d_lcol;
    a.loff = e->d_loff;
    a.loff_stride = e->loff_stride;
    a.ctl = e->d_ctl;
    a.cap = cap;
    a.flush = ~0ull;
    a.budget = static_cast<unsigned long long>(budget_ticks);
    a.slim = use_slim(e, q->k) ? 1 : 0;
    a.mail = nullptr;
    a.idle_bits = nullptr;
    a.steal_slots = 0;
    if (!e->opt.disable_stealing) {
        if (!e->d_mail) {
            // one mailbox per wavefront that can be resident (at most 32 per CU)
            const int32_t slots = e->num_cu * 32;
            hipError_t h = hipMalloc(reinterpret_cast<void **>(&e->d_mail), sizeof(gm::Mailbox) * slots);
            if (h == hipSuccess)
                h = hipMalloc(reinterpret_cast<void **>(&e->d_idle_bits), sizeof(unsigned long long) * ((slots + 63) / 64));
            if (h != hipSuccess) {
                if (e->d_mail) hipFree(e->d_mail);
                e->d_mail = nullptr;
                e->d_idle_bits = nullptr;
                return e->fail(GM_ERR_NOMEM, "work-stealing mailbox allocation failed");
            }
            e->steal_slots = slots;
        }
        a.mail = e->d_mail;
        a.idle_bits = e->d_idle_bits;
        a.steal_slots = e->steal_slots;
    }
    a.steal_threshold = e->opt.steal_threshold > 0 ? e->opt.steal_threshold : 128;
    a.plan = plan;

    if (q->k == 1) {
        // a single query vertex: its candidates are the matches
        const uint64_t cnt = pool_rows;
        out->count = cap && cnt >= cap ? cap : cnt;
        out->outcome = cap && cnt >= cap ? GM_CAPPED : GM_DONE;
        out->pool_rows = pool_rows;
        out->pool_depth = 1;
        if (enumerate && out->count) {
            HIP_TRY(e, hipMemcpyAsync(rows, e->d_pool[0], out->count * sizeof(int32_t), hipMemcpyDeviceToHost,
                                      e->stream));
            HIP_TRY(e, hipStreamSynchronize(e->stream));
            out->rows = out->count;
        }
        std::chrono::duration<double, std::milli> ms = std::chrono::steady_clock::now() - t_start;
        out->search_ms = ms.count();
        return GM_OK;
    }

    // Initialisation phase (Sec. 4.3): breadth-first levels until >= tau rows.
    const int64_t tau = option_tau(e, q->k);
    const int64_t row_limit = e->opt.pool_row_limit > 0 ? e->opt.pool_row_limit : 64 * std::max<int64_t>(tau, 1);
    bool aborted = false;
    while (tau > 0 && pool_rows > 0 && pool_rows < static_cast<uint64_t>(tau) && depth < q->k - 1) {
        a.plan.depth = depth;
        a.pool = e->d_pool[cur];
        a.pool_rows = pool_rows;
        if (bound > static_cast<uint64_t>(row_limit)) break;
        st = ensure_buffer(e, &e->d_pool[cur ^ 1], &e->pool_cap[cur ^ 1], bound * static_cast<size_t>(depth + 1));
        if (st) return st;
        HIP_TRY(e, hipMemsetAsync(&e->d_ctl->pool_next, 0, sizeof(unsigned long long), e->stream));
        HIP_TRY(e, hipMemsetAsync(&e->d_ctl->out_rows, 0, sizeof(unsigned long long), e->stream));
        HIP_TRY(e, hipMemsetAsync(&e->d_ctl->measure, 0, sizeof(unsigned long long), e->stream));
        a.out = e->d_pool[cur ^ 1];
        a.out_cap = bound;
        a.measure_next = depth + 1 < q->k - 1 ? 1 : 0;  // bound of the level after this one
        st = reset_stealing(e, a);
        if (st) return st;
        HIP_TRY(e, gm::launch_expand(a, e->num_cu, e->stream));
        st = read_ctl(e, &c);
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
    Control before = c;
    if (!aborted && pool_rows > 0) {
        if (enumerate) {
            st = ensure_buffer(e, &e->d_rows, &e->rows_cap, static_cast<size_t>(cap) * q->k);
            if (st) return st;
        }
        a.plan.depth = depth;
        a.pool = e->d_pool[cur];
        a.pool_rows = pool_rows;
        a.out = enumerate ? e->d_rows : nullptr;
        a.out_cap = enumerate ? cap : 0;
        if (cap) {
            const unsigned long long per = cap / (static_cast<unsigned long long>(e->num_cu) * 64ull);
            a.flush = std::max<unsigned long long>(1, std::min<unsigned long long>(4096, per));
        }
        HIP_TRY(e, hipMemsetAsync(&e->d_ctl->pool_next, 0, sizeof(unsigned long long), e->stream));
        HIP_TRY(e, hipMemsetAsync(&e->d_ctl->out_rows, 0, sizeof(unsigned long long), e->stream));
        st = reset_stealing(e, a);
        if (st) return st;
        before = c;
        HIP_TRY(e, hipEventRecord(e->ev0, e->stream));
        HIP_TRY(e, gm::launch_search(a, enumerate, e->num_cu, e->opt.waves_per_cu, e->stream, &grid_waves));
        HIP_TRY(e, hipEventRecord(e->ev1, e->stream));
        st = read_ctl(e, &c);
        if (st) return st;
        HIP_TRY(e, hipEventElapsedTime(&kernel_ms, e->ev0, e->ev1));
    }

    const uint64_t total = c.count;
    if (cap && total >= cap) {
        out->count = cap;
        out->outcome = GM_CAPPED;
    } else {
        out->count = total;
        out->outcome = (aborted || c.abort == gm::kAbortTime) ? GM_TIMEOUT : GM_DONE;
    }
    out->pool_rows = pool_rows;
    out->pool_depth = depth;
    out->groups = c.groups;
    out->tasks = c.tasks;
    out->lanes_active = c.lanes_active;
    out->lanes_issued = c.lanes_issued;
    out->probes = c.probes;
    out->steals = c.steals;
    out->kernel_ms = kernel_ms;
    out->grid_waves = grid_waves;
    out->kernel_tasks = c.tasks - before.tasks;
    out->kernel_probes = c.probes - before.probes;
    out->kernel_groups = c.groups - before.groups;
    out->scanned = c.scanned;
    out->kernel_scanned = c.scanned - before.scanned;
    out->kernel_lookups = c.lookups - before.lookups;
    if (enumerate) {
        const uint64_t nrows = std::min<uint64_t>(out->count, std::min<uint64_t>(c.out_rows, cap));
        if (nrows) {
            HIP_TRY(e, hipMemcpyAsync(rows, e->d_rows, nrows * q->k * sizeof(int32_t), hipMemcpyDeviceToHost,
                                      e->stream));
            HIP_TRY(e, hipStreamSynchronize(e->stream));
        }
        out->rows = nrows;
    }
    std::chrono::duration<double, std::milli> ms = std::chrono::steady_clock::now() - t_start;
    out->search_ms = ms.count();
    return GM_OK;
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
        o.pool_row_limit < 0) {
        g_create_error = "option out of range";
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
            (h = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking)) != hipSuccess ||
            (h = hipEventCreate(&e->ev0)) != hipSuccess || (h = hipEventCreate(&e->ev1)) != hipSuccess ||
            (h = hipMalloc(reinterpret_cast<void **>(&e->d_ctl), sizeof(Control))) != hipSuccess) {
            g_create_error = std::string("HIP setup failed: ") + hipGetErrorString(h);
            gm_destroy(e);
            return GM_ERR_DEVICE;
        }
        e->num_cu = prop.multiProcessorCount;
        e->wall_khz = khz > 0 ? khz : 100000;
    }
    *out = e;
    return GM_OK;
}

void gm_destroy(gm_engine *e) {
    if (!e) return;
    if (e->device >= 0) {
        hipSetDevice(e->device);
        if (e->stream) hipStreamSynchronize(e->stream);
        free_graph(e);
        for (int i = 0; i < 2; ++i)
            if (e->d_pool[i]) hipFree(e->d_pool[i]);
        if (e->d_rows) hipFree(e->d_rows);
        if (e->d_ctl) hipFree(e->d_ctl);
        if (e->d_mail) hipFree(e->d_mail);
        if (e->d_idle_bits) hipFree(e->d_idle_bits);
        if (e->ev0) hipEventDestroy(e->ev0);
        if (e->ev1) hipEventDestroy(e->ev1);
        if (e->stream) hipStreamDestroy(e->stream);
    }
    delete e;
}

gm_status gm_load_graph(gm_engine *e, int32_t n, const int64_t *row_ptr, const int32_t *col,
                        const int32_t *labels) {
    if (!e) return GM_ERR_ARG;
    std::lock_guard<std::mutex> lk(e->mu);
    if (n < 0) return e->fail(GM_ERR_ARG, "n must be >= 0");
    if (!row_ptr || (n > 0 && !labels)) return e->fail(GM_ERR_ARG, "row_ptr and labels must not be null");
    gm_status st = check_graph(e, n, row_ptr, col, e->opt.skip_symmetry_check == 0);
    if (st) return st;
    std::unordered_map<int32_t, int32_t> ids;
    std::vector<VInfo> vinfo(static_cast<size_t>(n));
    for (int32_t v = 0; v < n; ++v) {
        auto it = ids.find(labels[v]);
        int32_t id;
        if (it == ids.end()) {
            id = static_cast<int32_t>(ids.size());
            if (id >= 255) return e->fail(GM_ERR_GRAPH, "more than 255 distinct vertex labels");
            ids.emplace(labels[v], id);
        } else {
            id = it->second;
        }
        const uint64_t deg = static_cast<uint64_t>(row_ptr[v + 1] - row_ptr[v]);
        vinfo[v].x = static_cast<uint32_t>(row_ptr[v]);
        vinfo[v].y = static_cast<uint32_t>(deg << 8) | static_cast<uint32_t>(id);
    }
    const uint64_t nnz = static_cast<uint64_t>(row_ptr[n]);
    // Label-partitioned copy of the lists: N(v) ordered by (label, id), with the
    // bounds of every label slice, so a task group scans only candidates that
    // carry its query vertex's label.  Skipped when asked, when there is one
    // label, or when the bounds table would exceed 8 GiB.
    const int32_t labels_used = static_cast<int32_t>(ids.size());
    int32_t stride = labels_used + 1;
    if (e->opt.disable_label_index || labels_used <= 1 ||
        static_cast<uint64_t>(n) * static_cast<uint64_t>(stride) * 4ull > (8ull << 30))
        stride = 1;
    std::vector<uint32_t> loff;
    std::vector<int32_t> lcol;
    if (stride == 1) {
        loff.resize(static_cast<size_t>(n) + 1);
        for (int32_t v = 0; v <= n; ++v) loff[v] = static_cast<uint32_t>(row_ptr[v]);
    } else {
        loff.resize(static_cast<size_t>(n) * stride);
        lcol.resize(nnz);
        parallel_ranges(n, [&](int64_t b, int64_t end) {
            std::vector<uint32_t> cnt(stride);
            for (int64_t v = b; v < end; ++v) {
                std::fill(cnt.begin(), cnt.end(), 0u);
                for (int64_t p = row_ptr[v]; p < row_ptr[v + 1]; ++p) ++cnt[(vinfo[col[p]].y & 0xffu) + 1];
                uint32_t *o = &loff[static_cast<size_t>(v) * stride];
                o[0] = static_cast<uint32_t>(row_ptr[v]);
                for (int32_t c = 1; c < stride; ++c) o[c] = o[c - 1] + cnt[c];
                for (int32_t c = 0; c + 1 < stride; ++c) cnt[c] = o[c];  // fill cursors
                for (int64_t p = row_ptr[v]; p < row_ptr[v + 1]; ++p) lcol[cnt[vinfo[col[p]].y & 0xffu]++] = col[p];
            }
        });
    }
    if (e->device >= 0) {
        HIP_TRY(e, hipSetDevice(e->device));
        free_graph(e);
        hipError_t h = hipMalloc(reinterpret_cast<void **>(&e->d_vinfo), std::max<size_t>(n, 1) * sizeof(VInfo));
        if (h == hipSuccess)
            h = hipMalloc(reinterpret_cast<void **>(&e->d_col), std::max<uint64_t>(nnz, 1) * sizeof(int32_t));
        if (h == hipSuccess)
            h = hipMalloc(reinterpret_cast<void **>(&e->d_loff), std::max<size_t>(loff.size(), 1) * sizeof(uint32_t));
        if (h == hipSuccess && stride > 1)
            h = hipMalloc(reinterpret_cast<void **>(&e->d_lcol), std::max<uint64_t>(nnz, 1) * sizeof(int32_t));
        if (h != hipSuccess) {
            free_graph(e);
            return e->fail(GM_ERR_NOMEM, std::string("graph upload: ") + hipGetErrorString(h));
        }
        if (stride == 1) e->d_lcol = e->d_col;
        e->loff_stride = stride;
        if (n) HIP_TRY(e, hipMemcpy(e->d_vinfo, vinfo.data(), static_cast<size_t>(n) * sizeof(VInfo), hipMemcpyHostToDevice));
        if (nnz) HIP_TRY(e, hipMemcpy(e->d_col, col, nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_TRY(e, hipMemcpy(e->d_loff, loff.data(), loff.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        if (stride > 1 && nnz) HIP_TRY(e, hipMemcpy(e->d_lcol, lcol.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
    } else {
        free_graph(e);
        e->loff_stride = stride;
    }
    e->label_id = std::move(ids);
    e->n = n;
    e->nnz = nnz;
    e->has_graph = true;
    return GM_OK;
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
    return e->err.c_str();
}

}  // extern "C"
