/*
 * gmatch.h -- C ABI of the MI355X (gfx950) subgraph-matching engine.
 *
 * Problem (gMatch paper, Sec. 2.1, Def. 1): given an undirected vertex-labelled
 * data graph G and a connected query graph Q, find every injective map
 * M: V(Q) -> V(G) with L(u) = L(M[u]) for all query vertices u and
 * (M[u], M[u']) in E(G) for every query edge (u, u').  Matching is
 * non-induced and every map is counted (no symmetry breaking).  Algorithm 2's
 * interface takes Q, G, a matching order phi and the initial pool size tau and
 * outputs all matches; the calls below expose exactly that, with a result cap
 * and a time limit added.
 *
 * Conventions shared by every call:
 *   - Every call returns gm_status: GM_OK (0) or a negative error.  Nothing
 *     throws across the ABI.  gm_last_error() returns a message for the last
 *     failing call on an engine (or, with NULL, on this thread's gm_create).
 *   - Host pointers are only read during the call; the caller keeps ownership.
 *   - One engine holds one resident data graph on one GPU.  Calls on one engine
 *     are serialised by an internal mutex; engines are independent.
 *   - Counts are uint64.  Vertex ids are int32 in [0, n).
 */
#ifndef GMATCH_H
#define GMATCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GM_OK = 0,
    GM_ERR_ARG = -1,    /* null pointer, negative size, bad option value */
    GM_ERR_GRAPH = -2,  /* G is not a simple undirected CSR graph, or exceeds layout limits */
    GM_ERR_QUERY = -3,  /* Q is empty, larger than 32 vertices, not simple or not connected */
    GM_ERR_ORDER = -4,  /* order is not a permutation or not connected (Sec. 2.2) */
    GM_ERR_NOMEM = -5,  /* host or device allocation failed */
    GM_ERR_DEVICE = -6, /* HIP runtime error, or the engine has no GPU */
    GM_ERR_BUFFER = -7, /* output buffer missing or too small */
    GM_ERR_STATE = -8   /* no graph loaded, or unknown / freed query id */
} gm_status;

typedef enum {
    GM_DONE = 0,    /* search finished: count is exact */
    GM_CAPPED = 1,  /* the count reached the cap: count == cap (the true number is >= cap) */
    GM_TIMEOUT = 2  /* time limit hit first: count is a lower bound (an unsolved query, Sec. 6.1) */
} gm_outcome;

typedef struct gm_engine gm_engine;

/* Engine options.  A zero-initialised struct selects every default. */
typedef struct {
    /* Initial task pool (Sec. 4.3, "Initialization Phase").
     * 0 = default: a two-phase pool at position 1, with no breadth-first launch
     * and no host round trip.  First-phase work items hold 64 candidates of the
     * first query vertex each, every one with at most pool_hub_cut of its tasks
     * at position 1, so each candidate is sampled early and a hub holds up one
     * wavefront only.  The rest of the hubs' tasks are laid out as one list by a
     * prefix sum; second-phase items are 64 consecutive tasks of it, so a hub's
     * work spreads over many wavefronts, and wavefronts with no first-phase item
     * start on them at once.
     * > 0 = the paper's scheme: breadth-first expansion up to the first level
     * holding >= tau partial matches (the paper's own setting is 1e6).
     * < 0 = no expansion: the pool is the candidate set of the first query vertex,
     * 64 candidates per work item (the BFS-disabled mode of Sec. 6.2). */
    int64_t tau;
    /* Largest pool the expansion may build, in rows; 0 = default 64 * tau. */
    int64_t pool_row_limit;
    /* 0 = idle wavefronts steal work from busy ones (Sec. 4.3, "Dynamic Balancing
     * Phase"); 1 = no stealing. */
    int32_t disable_stealing;
    /* A busy wavefront donates work only from a level with at least this many
     * unscattered tasks.  0 = default 128. */
    int32_t steal_threshold;
    /* Wavefronts launched per compute unit; 0 = as many as fit. */
    int32_t waves_per_cu;
    /* 1 = skip the symmetry check of gm_load_graph (trusted input). */
    int32_t skip_symmetry_check;
    /* Per-wavefront stack layout in LDS: 1 = full (12 B per level and lane;
     * entries cache their neighbour-list range), 2 = slim (4 B: vertex and
     * parent lane in one word; membership tests bisect label slices, whose
     * bounds cost one load), 0 = default (slim: it keeps more wavefronts per CU
     * and bisects shorter ranges).  The slim layout holds vertex ids below
     * 2^24; on a graph with more vertices every search uses the full layout,
     * and a candidate-graph engine (which needs slim) refuses to load it. */
    int32_t stack_layout;
    /* 1 = do not build label-partitioned neighbour lists (every task group then
     * scans its whole list and the label filter rejects the rest). */
    int32_t disable_label_index;
    /* gm_count_batch: 0 = one persistent launch per stack-depth class (queries
     * whose stacks allow the same number of resident wavefronts share a launch),
     * 1 = a single launch sized for the largest query of the batch. */
    int32_t batch_single_launch;
    /* gm_count_batch: work-item streams per launch, i.e. queries in flight at
     * once.  Every wavefront serves its home stream's queries in order and
     * helps the next stream once its own runs dry.  0 = default 64. */
    int32_t batch_streams;
    /* Default pool (tau = 0): position-1 tasks a first-vertex candidate keeps
     * in its first-phase work item; the rest of a hub's tasks go to the second
     * phase.  0 = default 1, or 8 for a query whose first-phase items hold
     * one root each (fewer roots than resident wavefronts). */
    int32_t pool_hub_cut;
    /* 1 = no adjacency bitmaps.  By default gm_load_graph keeps one bit per
     * vertex of G for each of the highest-degree vertices (at least 256
     * neighbours; at most 4096 of them and hub_bitmap_mib in all), and a
     * membership test in such a list (slim stack layout) reads one bit instead
     * of bisecting. */
    int32_t disable_hub_bitmaps;
    /* Device memory for the adjacency bitmaps, in MiB (each takes |V(G)| / 8
     * bytes).  0 = default 1024. */
    int32_t hub_bitmap_mib;
    /* 1 = search on a candidate graph G' (the paper does so when it compares
     * with EGSM, whose G' it adopts: Sec. 6.1; App. C describes G' as built by
     * a light filter over labels and query structure).  Each gm_count /
     * gm_enumerate call first keeps, for every query vertex u, the largest set
     * C(u) of vertices with u's label and at least u's degree in which every
     * vertex has a neighbour in C(u') for each query neighbour u' of u, then
     * lists, for each query edge, the neighbours of every candidate that lie in
     * the other end's set; the search reads those lists instead of G's.
     * Counts are the same as on G.  The build runs on the device (a few sweeps
     * over G) and is part of the call's search_ms.  Requires tau = 0 and the
     * slim stack layout (stack_layout 0 or 2); gm_count_batch, gm_tune_batch
     * and gm_serve_open return GM_ERR_STATE while it is on.  Device memory:
     * |E(Q)| * (|V(G)| + 1) * 4 bytes of list bounds plus the lists. */
    int32_t candidate_graph;
    /* Default pool (tau = 0): first-vertex candidates per first-phase work
     * item, 1..64.  0 = automatic: 1 when a query has fewer candidates than
     * the launch has resident wavefronts (each starts on a root of its own),
     * else 64. */
    int32_t pool_roots_per_item;
    /* Membership tests (Sec. 5.2, "Time Cost"; Alg. 2 Process): the candidates
     * a parent hands out in one scatter round form an ascending run, and each of
     * them is tested against the same backward neighbour lists.  A list of
     * length n tested by a run of r candidates is staged into LDS by the run's
     * lanes and intersected there by merge path when n <= merge_ratio * r (it
     * must also fit the run's share of the staging buffer, 8 entries per lane);
     * longer lists are bisected in device memory by each lane (or answered by a
     * hub bitmap).  0 = default: ratio 1 unless the staging area would lower
     * the wavefronts a CU keeps resident (the deepest queries, about 29
     * vertices and more, where LDS bounds residency; those then never stage);
     * -1 = never stage; 1..8 = that ratio, always. */
    int32_t merge_ratio;
    int32_t reserved[2];
} gm_options;

/* Result of one count or enumerate call. */
typedef struct {
    uint64_t count;        /* min(#matches, cap) */
    int32_t outcome;       /* gm_outcome */
    int32_t pool_depth;    /* matched positions per initial-pool row (1 for the virtual pool:
                              its rows are the first vertex's candidates) */
    double search_ms;      /* wall time of the search on the device: from the first
                              launch to the result being back on the host */
    uint64_t pool_rows;    /* size of the initial task pool */
    uint64_t groups;       /* task groups: valid partial matches of length 1..k-1 extended (Sec. 4.1) */
    uint64_t tasks;        /* tasks: local candidates examined, sum of |C^L| over groups (Sec. 4.1) */
    uint64_t lanes_active; /* lanes that held a task, summed over scatter rounds */
    uint64_t lanes_issued; /* 64 x scatter rounds; idle rate = 1 - active/issued (Sec. 2.3) */
    uint64_t probes;       /* 4-byte neighbour-list reads made by membership tests */
    uint64_t steals;       /* work donations taken by idle wavefronts */
    uint64_t rows;         /* enumerate: rows written */
    double kernel_ms;      /* device time of the depth-first search launch alone (HIP events) */
    int32_t grid_waves;    /* wavefronts in that launch */
    int32_t candidate_rounds; /* candidate graph: filter sweeps up to the first that dropped
                                 nothing (0 when off) */
    uint64_t kernel_tasks;  /* tasks, probes and matches of that launch alone (the pool */
    uint64_t kernel_probes; /* expansion before it is excluded) */
    uint64_t kernel_groups;
    uint64_t scanned;        /* candidates actually read: with label-partitioned neighbour
                                lists a task group scans only the slice of its list whose
                                label is the query vertex's label (<= tasks) */
    uint64_t kernel_scanned; /* ... of the depth-first search launch alone */
    uint64_t kernel_lookups; /* label-slice bound lookups (8 B each) of that launch */
    double candidate_ms;     /* candidate graph: host wall time of its build (inside search_ms) */
    uint64_t candidate_edges; /* candidate graph: list entries, summed over query edges */
    uint64_t kernel_bytes;   /* device-memory bytes the depth-first search launch requested for
                                this query: every load it issued (list entries, vertex records,
                                slice bounds, bisection and tail probes, bitmap words, pool rows)
                                and every row it wrote, counted where issued */
    double query_ms;         /* batched launches: device time from the query's first work item to
                                the last time a wavefront reported work on it (0 elsewhere) */
    uint64_t kernel_bytes_late; /* part of kernel_bytes from the last 32-round window of each
                                wavefront that saw the cap or time limit: an upper bound on the
                                bytes spent after the query was decided */
} gm_result;

/* Create an engine on HIP device `device` (>= 0).  device = -1 creates a
 * host-only engine: graphs and queries are checked and planned, but count and
 * enumerate return GM_ERR_DEVICE.  opt may be NULL (all defaults). */
gm_status gm_create(int32_t device, const gm_options *opt, gm_engine **out);

/* Free the engine, its device memory and its queries.  NULL is ignored. */
void gm_destroy(gm_engine *engine);

/* Load G from host CSR arrays, replacing any previous graph (and keeping the
 * loaded queries).  row_ptr[n+1] (row_ptr[0] = 0, non-decreasing),
 * col[row_ptr[n]] with every row strictly ascending, ids in [0, n), no
 * self-loops, and every edge stored in both directions (Sec. 2.1: undirected).
 * labels[n]: any int32 values; at most 255 distinct values.  Layout limits:
 * row_ptr[n] < 2^32 and every degree < 2^24.  Violations: GM_ERR_GRAPH. */
gm_status gm_load_graph(gm_engine *engine, int32_t n, const int64_t *row_ptr, const int32_t *col,
                        const int32_t *labels);

/* Load G from CSR arrays that already live in device memory of the engine's
 * device (for example tensors of a framework that owns the GPU's memory and
 * streams), replacing any previous graph.  Same graph as gm_load_graph (Def. 1,
 * Sec. 2.1), same checks and GM_ERR_GRAPH cases, with these layouts:
 *   row_ptr: n + 1 offsets of row_ptr_bytes bytes each (4: int32, 8: int64);
 *   col:     row_ptr[n] int32 neighbour ids, every row strictly ascending;
 *   labels:  n uint8 label values (at most 255 distinct).
 * Ownership: col is NOT copied.  The engine searches the caller's col in place
 * until the graph is replaced or the engine destroyed; the caller must keep it
 * alive and unchanged until then.  row_ptr and labels are read during the call
 * only.  The engine allocates and owns the structures it derives (vertex
 * records, label-sorted lists, hub bitmaps).
 * hip_stream: the HIP stream (hipStream_t; NULL = the null stream) on which the
 * caller produced the arrays; the load's copies and kernels run on it after the
 * caller's queued work, and the call returns once they are done.
 * Errors: GM_ERR_ARG for a pointer that is not device memory of this engine's
 * device or a row_ptr_bytes other than 4 or 8, GM_ERR_DEVICE on a host-only
 * engine, GM_ERR_STATE while a server is open. */
gm_status gm_load_graph_device(gm_engine *engine, int32_t n, const void *row_ptr, int32_t row_ptr_bytes,
                               const int32_t *col, const uint8_t *labels, void *hip_stream);

/* Load Q: k vertices (1..32), m undirected edges given as pairs
 * edges[2e], edges[2e+1], labels[k].  Q must be simple and connected.  On
 * success *qid_out receives a handle; its matching order is the heuristic
 * order (see gm_set_order). */
gm_status gm_load_query(gm_engine *engine, int32_t k, int32_t m, const int32_t *edges,
                        const int32_t *labels, int32_t *qid_out);

/* Set the matching order phi of a query (Sec. 2.2): order[i] is the query
 * vertex mapped i-th.  It must be a permutation in which every vertex after the
 * first has an earlier neighbour.  order = NULL restores the heuristic order:
 * RI's greatest-constraint-first rule (Sec. 3 uses RI): start from the largest
 * query degree, then repeatedly take the vertex with the most already-ordered
 * neighbours, then the most ordered vertices adjacent to its unordered
 * neighbours, then the most unordered neighbours with no ordered neighbour;
 * ties go to the smaller vertex id. */
gm_status gm_set_order(gm_engine *engine, int32_t qid, const int32_t *order);

/* Copy the current matching order of a query into order_out[k]. */
gm_status gm_get_order(const gm_engine *engine, int32_t qid, int32_t *order_out);

/* Count the matches of query qid in the loaded graph (Alg. 2 with counting as
 * its output).  cap = 0: no cap.  time_limit_s <= 0: no limit.  out receives
 * the count, the outcome and the work counters. */
gm_status gm_count(gm_engine *engine, int32_t qid, uint64_t cap, double time_limit_s, gm_result *out);

/* List matches: rows is a host buffer of cap * k int32 (cap >= 1); row r holds
 * the data vertex of query vertex 0..k-1 of the r-th match found.  Rows come in
 * no particular order.  At most cap rows are written; out->count follows
 * gm_count's rules with this cap and out->rows equals min(count, cap). */
gm_status gm_enumerate(gm_engine *engine, int32_t qid, int32_t *rows, uint64_t cap, double time_limit_s,
                       gm_result *out);

/* The candidate sets of query qid (see gm_options.candidate_graph), built for
 * its current order whether or not the option is on.  bits: host buffer of
 * k * ((n + 31) / 32) words, n = |V(G)|; bit (v % 32) of bits[u * ((n + 31) /
 * 32) + v / 32] is set iff v is in C(u), u a query vertex.  edges_out (may be
 * NULL): list entries of G', summed over the query's edges.  rounds_out (may
 * be NULL): filter sweeps up to the first one that dropped nothing.  Errors:
 * GM_ERR_STATE without a graph, GM_ERR_DEVICE on a host-only engine. */
gm_status gm_candidate_sets(gm_engine *engine, int32_t qid, uint32_t *bits, uint64_t *edges_out,
                            int32_t *rounds_out);

/* Summary of one gm_count_batch call. */
typedef struct {
    double total_ms;     /* host wall time of the call */
    double kernel_ms;    /* device time of its persistent search launches (HIP events), summed */
    int32_t launches;    /* search launches made */
    int32_t grid_waves;  /* wavefronts of the largest launch */
    uint64_t count;      /* sums over the queries of the per-query fields */
    uint64_t tasks;
    uint64_t scanned;
    uint64_t lookups;
    uint64_t probes;
    uint64_t groups;
    uint64_t steals;
    uint64_t bytes;      /* kernel_bytes and kernel_bytes_late of gm_result, summed */
    uint64_t bytes_late;
    uint64_t reserved[2];
} gm_batch_info;

/* Count several queries in shared persistent launches (Alg. 2 for many
 * queries at once; Sec. 4.3's persistent wavefronts and work stealing carry
 * over unchanged).  qids[nq] may repeat a query.  Each query's first-vertex
 * candidates (label and degree filter, Sec. 6.1) form its share of the pool,
 * 64 per work item, with no breadth-first expansion; idle wavefronts take work
 * from busy ones regardless of query, so a heavy query spreads over the GPU.
 * out[i] follows gm_count's rules for qids[i] with the same cap and time
 * limit: the same exact count when the search finishes, min(count, cap) with
 * GM_CAPPED, or a lower bound with GM_TIMEOUT.  Each query's time limit runs
 * from the moment its first work item is taken on the device, so waiting
 * behind other queries of the batch does not count.  out[i].search_ms is the
 * call's wall time, out[i].kernel_ms and grid_waves describe the launch that
 * held the query, pool_depth is 1 and pool_rows its candidate count; the
 * kernel_* counters equal the totals (there is no expansion launch).  info
 * may be NULL.  nq = 0 is allowed and does nothing. */
gm_status gm_count_batch(gm_engine *engine, int32_t nq, const int32_t *qids, uint64_t cap, double time_limit_s,
                         gm_result *out, gm_batch_info *info);

/* Count one query without allocating: for callers that cannot allocate device
 * memory while they run (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same result as gm_count_batch on the one
 * query qid (first-vertex candidates as the pool, cap and time limit as
 * gm_count), with every device buffer of its launch in a fixed arena that the
 * library holds on each GPU until the process ends: 64 MiB, a file-scope
 * device array, looked up once per device when an engine is created on it.
 * The call makes no hipMalloc, hipFree or other allocating call.  The arena
 * holds the query's control blocks and, per wavefront, a stealing mailbox and
 * the parked task groups of its levels; a launch uses at most as many
 * wavefronts as fit (all resident ones up to 16-vertex queries, about 2,700 at
 * 32 vertices), and GM_ERR_BUFFER is returned if not even one would fit.
 * The arena keeps the last call's contents; each call clears what must start
 * at zero.  Calls on one GPU share its arena, so calls that overlap on one GPU
 * (two threads, two engines, or two servers) race: serialise them.  Returns
 * GM_ERR_STATE with the candidate-graph option (its per-call build allocates). */
gm_status gm_count_noalloc(gm_engine *engine, int32_t qid, uint64_t cap, double time_limit_s, gm_result *out);

/* Settings chosen by gm_tune_batch. */
typedef struct {
    int32_t waves_per_cu;        /* resident wavefronts per CU (0 = as many as fit) */
    int32_t steal_threshold;     /* smallest level a busy wavefront splits for an idle one */
    int32_t stack_layout;        /* 1 = full, 2 = slim (LDS bytes per stack entry) */
    int32_t batch_single_launch; /* as in gm_options */
    int32_t batch_streams;       /* as in gm_options */
    int32_t trials;              /* settings measured */
    double best_ms;              /* device time of the chosen setting on the sample */
    double default_ms;           /* device time of the engine's settings before tuning */
    int32_t merge_ratio;         /* as in gm_options: LDS staging of short lists (0 = default, -1 = never) */
    int32_t reserved;
} gm_tuning;

/* Autotuner of the batched launch: runs gm_count_batch on the sample qids[nq]
 * and tunes one setting at a time, each over a fixed list, keeping the best
 * value before moving on: streams (queries in flight) over 1, 16, 64, 256;
 * wavefronts per CU over as-many-as-fit, 12, 8; stack layout (LDS bytes per
 * wavefront) slim, full; steal threshold 32, 128, 512; LDS staging of short
 * lists (merge_ratio: the default, none, or a staging buffer of 1, 2 or 4
 * entries per lane); launch grouping.  The
 * measure is the device time of the batch's launches.  The result stays in
 * the engine's options and is reported in *out.  Every setting must give the
 * same count for each query that finishes under both; a difference returns
 * GM_ERR_STATE (an engine defect) and restores the options. */
gm_status gm_tune_batch(gm_engine *engine, int32_t nq, const int32_t *qids, uint64_t cap, double time_limit_s,
                        gm_tuning *out);

/* Copy the engine's current options (after gm_tune_batch, its choices). */
gm_status gm_get_options(const gm_engine *engine, gm_options *out);

/* ------------------------------------------------------------------------
 * Serving: continuous batching over a resident graph.
 *
 * A server owns `slots` launch contexts (a HIP stream each, with its own
 * control block, plans, result blocks and stealing mailboxes) and a native
 * worker thread.  gm_serve_submit only queues a request (the query's plan is
 * built at once, so the query may be freed afterwards).  Whenever a slot is
 * free, the worker admits up to max_batch queued requests, oldest first, into
 * one persistent launch on that slot (the batched launch of gm_count_batch,
 * every query with its own cap and time limit); launches of different slots
 * run on the GPU at the same time, each with its share of the wavefronts, so
 * requests that arrive while others run are admitted as soon as a slot frees
 * up and their work overlaps with the work in flight.  Admission is bounded by
 * memory: a launch holds at most max_batch requests, its wavefronts' LDS stacks
 * are sized for its largest query, and the device memory of the launches in
 * flight (plans, result blocks, stealing mailboxes and parked task groups)
 * stays within memory_mib.  Results come back
 * through gm_serve_poll with their submit, start and completion times.
 * Each result equals what gm_count gives for the query with the same cap and
 * time limit (exact when it finishes; with GM_TIMEOUT a lower bound).
 * While a server is open, gm_load_graph and gm_tune_batch on its engine return
 * GM_ERR_STATE; other engine calls may run alongside it.  Close every server
 * before gm_destroy of its engine.
 * ------------------------------------------------------------------------ */
typedef struct gm_server gm_server;

typedef struct {
    int32_t slots;          /* concurrent launches; 0 = default 2 */
    int32_t max_batch;      /* requests admitted into one launch; 0 = default 256 */
    int32_t waves_per_cu;   /* wavefronts per CU of each launch; 0 = an equal share of what fits */
    int32_t batch_streams;  /* work-item streams per launch (queries in flight); 0 = the engine's */
    int64_t max_pending;    /* queued requests beyond which submit returns GM_ERR_BUFFER; 0 = no limit */
    /* Device memory for the working state of the launches in flight, in MiB;
     * 0 = default 1024.  A launch's state is its requests' plans and result
     * blocks and, for each of its wavefronts, a stealing mailbox and the parked
     * task groups of as many levels as its largest query has.  A free slot
     * admits the oldest requests while the launches in flight plus the new one
     * fit; a request that does not fit waits (in order) for memory to free up,
     * and one that could not fit even alone is refused by gm_serve_submit with
     * GM_ERR_BUFFER. */
    int64_t memory_mib;
    int32_t reserved[4];
} gm_serve_options;

typedef struct {
    uint64_t ticket;        /* as returned by gm_serve_submit */
    int32_t qid;
    int32_t slot;           /* slot whose launch ran it */
    double submit_ms;       /* times on the server's clock, ms since gm_serve_open */
    double start_ms;        /* launch of its batch queued */
    double done_ms;         /* its batch's results read back */
    gm_result result;
    int32_t status;         /* GM_OK, or the error that stopped its launch (result then invalid) */
    int32_t reserved;
} gm_serve_result;

/* Start a server on an engine with a loaded graph.  opt may be NULL. */
gm_status gm_serve_open(gm_engine *engine, const gm_serve_options *opt, gm_server **out);

/* Queue a count of query qid with its cap (0 = none) and time limit (<= 0 =
 * none; counted from the query's first work item on the device).  *ticket
 * identifies its result. */
gm_status gm_serve_submit(gm_server *server, int32_t qid, uint64_t cap, double time_limit_s, uint64_t *ticket);

/* Move up to max_results finished results into out[], oldest first, waiting
 * up to wait_s seconds for at least one if none is ready (0 = do not wait).
 * *n_out receives the number written. */
gm_status gm_serve_poll(gm_server *server, gm_serve_result *out, int32_t max_results, double wait_s,
                        int32_t *n_out);

/* Device memory (bytes) of the working state a launch holding only query qid
 * takes on this server: what admission charges a request that runs alone. */
gm_status gm_serve_request_bytes(gm_server *server, int32_t qid, int64_t *bytes);

/* Numbers of requests queued, running and finished-but-not-polled. */
gm_status gm_serve_stats(gm_server *server, int64_t *pending, int64_t *running, int64_t *ready);

/* Finish every queued and running request, stop the worker and free the
 * server; results not yet polled are dropped.  NULL is ignored. */
gm_status gm_serve_close(gm_server *server);

/* ------------------------------------------------------------------------
 * Learned matching order.
 *
 * The matching order decides the size of the search space (Sec. 2.2; the
 * paper takes RI's heuristic order, Sec. 3).  Any connected order gives the
 * same matches, so an order can be chosen for speed alone: a cost model
 * predicts the log2 search time of (query, order) pairs from features of the
 * query and of the data graph, and the engine runs the candidate predicted
 * cheapest, keeping the heuristic order unless another is predicted faster by
 * a margin.  The model is trained on search times the engine itself measures.
 * ------------------------------------------------------------------------ */

/* Length of a feature vector. */
#define GM_ORDER_FEATURES 192

/* Features of query qid under `order` (NULL = its current order) into
 * out[GM_ORDER_FEATURES]: for each position i < 32 of the order, five values
 * at out[5 i ..] (zeros past k): log2(1 + candidates of the query vertex in
 * G, by label and degree) / 24, its query degree / 8, its backward neighbours
 * / 8, log2(1 + the smallest candidate count among its backward neighbours) /
 * 24, and log2(1 + vertices of G with its label) / 24; then out[160] = k / 32,
 * out[161] = edges / 64 and 30 zeros. */
gm_status gm_order_features(gm_engine *engine, int32_t qid, const int32_t *order, float *out);

/* Candidate orders of query qid into orders[max_orders * k], *n_out of them:
 * the heuristic order first; then the connected order that always takes the
 * vertex with the fewest candidates among those adjacent to the placed ones
 * (starting from the fewest overall), if different; then random connected
 * orders (seeded by `seed`), without duplicates. */
gm_status gm_candidate_orders(gm_engine *engine, int32_t qid, int32_t max_orders, uint64_t seed, int32_t *orders,
                              int32_t *n_out);

/* The cost model: a perceptron with two hidden relu layers of `hidden` units
 * (a multiple of 32) and one output, bf16 weights and fp32 accumulation on the
 * matrix cores.  Inputs are padded to a multiple of 32.  Created on a HIP
 * device with weights drawn from `seed` (He initialisation). */
typedef struct gm_model gm_model;
gm_status gm_model_create(int32_t device, int32_t in_dim, int32_t hidden, uint64_t seed, gm_model **out);
void gm_model_destroy(gm_model *model);

/* Predictions for n rows of `dim` features (x[n * dim], host) into y[n]. */
gm_status gm_model_predict(gm_model *model, const float *x, int32_t n, int32_t dim, float *y);

/* Adam on the mean squared error against t[n] (host arrays), `epochs` passes
 * in shuffled minibatches of `batch` rows (seeded); *mean_loss (may be NULL)
 * receives the last pass's mean squared error. */
gm_status gm_model_train(gm_model *model, const float *x, const float *t, int32_t n, int32_t dim, int32_t epochs,
                         int32_t batch, float lr, uint64_t seed, float *mean_loss);

/* fp32 master weights: w1[in_dim_padded * hidden] (row-major, input-major),
 * b1[hidden], w2[hidden * hidden], b2[hidden], w3[hidden], b3[1].  Setting them
 * also resets the optimiser state. */
gm_status gm_model_get_params(const gm_model *model, float *w1, float *b1, float *w2, float *b2, float *w3, float *b3);
gm_status gm_model_set_params(gm_model *model, const float *w1, const float *b1, const float *w2, const float *b2,
                              const float *w3, const float *b3);
const char *gm_model_last_error(const gm_model *model);

/* Choose the order of query qid with the model: predict every candidate of
 * gm_candidate_orders(max_orders, seed); set the one predicted cheapest if its
 * prediction is below the heuristic order's by more than `margin` (log2
 * units), else keep the heuristic order.  *chosen receives the candidate's
 * index (0 = heuristic) and predicted[max_orders] (may be NULL) the
 * predictions. */
gm_status gm_choose_order(gm_engine *engine, gm_model *model, int32_t qid, int32_t max_orders, uint64_t seed,
                          float margin, int32_t *chosen, float *predicted);

/* Task split of query qid's initial pool (Sec. 4.3 splits the search into
 * tasks before the depth-first phase): with the default two-phase pool, the
 * number of a first-vertex candidate's position-1 tasks that stay with it in
 * its first-phase work item; the rest of them become second-phase items of 64
 * tasks that any wavefront can take.  0 = the engine's pool_hub_cut (default
 * 1, or 8 where a first-phase item holds one root).  Counts do not depend on it.  GM_ERR_ARG outside [0, 2^24]. */
gm_status gm_set_split(gm_engine *engine, int32_t qid, int32_t split);
/* The split a count of qid uses now (its own, else the engine's). */
gm_status gm_get_split(const gm_engine *engine, int32_t qid, int32_t *split);

/* Let the model pick query qid's plan: its matching order among
 * gm_candidate_orders(max_orders, seed) and its task split among
 * splits[nsplits].  Candidate 0 is the heuristic order with the current split;
 * then every (order, split) pair in order-major order.  The candidate
 * predicted cheapest is proposed if it beats candidate 0's prediction by more
 * than `margin` (log2 units), else candidate 0 stays.  With probe_cap > 0 the
 * measured runtime judges the proposal: the query is counted under both plans
 * up to probe_cap (and probe_limit_s, <= 0 = none), and the proposal is kept
 * only if it got there faster; *probe_ms (may be NULL) receives those runs'
 * search time.  *chosen_order receives the order's index (0 = heuristic),
 * *chosen_split the split, and predicted[1 + orders * nsplits] (may be NULL)
 * the predictions. */
gm_status gm_choose_plan(gm_engine *engine, gm_model *model, int32_t qid, int32_t max_orders, uint64_t seed,
                         const int32_t *splits, int32_t nsplits, float margin, uint64_t probe_cap,
                         double probe_limit_s, int32_t *chosen_order, int32_t *chosen_split, float *predicted,
                         double *probe_ms);

/* Opt-in symmetry breaking.  By default every injective map is counted (Def.
 * 1).  The paper's comparison runs give all systems the same symmetry-breaking
 * strategy (App. A); with enable = 1, query qid counts each class of matches
 * that differ only by an automorphism of Q (a permutation of V(Q) keeping its
 * labels and edges) once.  Conditions M(v) < M(u) chosen along a stabilizer
 * chain (Grochow and Kellis 2007) keep exactly one map per class, so the
 * count with it on times |Aut(Q)| is the count with it off (enumeration lists
 * one representative per class).  *aut_size (may be NULL) receives |Aut(Q)|,
 * saturating at 2^64 - 1.  GM_ERR_QUERY if the automorphism search of Q
 * exceeds its budget (then the mode stays off). */
gm_status gm_set_symmetry_breaking(gm_engine *engine, int32_t qid, int32_t enable, uint64_t *aut_size);

/* Forget a query; its id is not reused. */
gm_status gm_free_query(gm_engine *engine, int32_t qid);

/* Message describing the last failed call on this engine (NULL: the last failed
 * gm_create on this thread).  The text is copied for the calling thread; the
 * pointer stays valid until that thread calls gm_last_error again. */
const char *gm_last_error(const gm_engine *engine);

#ifdef __cplusplus
}
#endif

#endif /* GMATCH_H */
