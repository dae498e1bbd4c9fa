// Types shared by the host engine (engine.cpp) and the gfx950 kernels (kernels.hip).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace gm {

constexpr int kMaxK = 32;  // largest query supported
constexpr unsigned long long kScratchBytes = 64ull << 20;  // the allocation-free call's arena (per GPU)
constexpr int kMaxMergeSlots = 8;      // LDS-staged intersection: largest staging entries per lane
constexpr int kDefaultMergeSlots = 1;  // ... and the default (lists no longer than the run of candidates)
constexpr int kWave = 64;  // CDNA wavefront width
// The membership test reads the end of a list as one window of this many
// consecutive entries, so every adjacency array it searches (the adjacency, its
// label-sorted copy, the candidate graph's lists) is allocated with at least
// this many entries.
constexpr uint64_t kListWindow = 8;

// Packed per-vertex record, one 8-byte load per candidate:
//   x = first adjacency slot of v in col[], y = (degree << 8) | compact label.
using VInfo = uint2;

__host__ __device__ inline uint32_t vi_deg(VInfo a) { return a.y >> 8; }
__host__ __device__ inline uint32_t vi_lab(VInfo a) { return a.y & 0xffu; }

// Query along the matching order: position i maps query vertex phi[i].  Plans
// live in device memory (one per query of a launch); kernels read them through
// the constant address space, so a wavefront's plan fields come from scalar loads.
struct Plan {
    int32_t k;                // query size
    int32_t depth;            // matched positions per pool row (>= 1)
    int32_t phi[kMaxK];       // query vertex at position i
    int32_t lab[kMaxK];       // compact label of phi[i] (255 = absent from G)
    int32_t qdeg[kMaxK];      // query degree of phi[i] (degree filter)
    uint32_t bwd[kMaxK];      // bit j set: phi[j] (j < i) is a backward neighbour of phi[i]
    unsigned long long cap;   // 0 = none
    unsigned long long flush; // local matches kept by a wavefront before an atomic flush
    unsigned long long budget; // time limit of this query in device wall-clock ticks from
                               // its first work item, 0 = none
    // this query's share of the launch's pool: rows pool[row0 + r * depth ...],
    // r < rows, claimed as work items item0 .. item_end - 1 of 64 rows each
    unsigned long long row0;
    unsigned long long rows;
    unsigned long long item0;
    unsigned long long item_end;
    // two-phase pool (vmode = 1): the rows are roots (depth 1).  Items item0 ..
    // item_split - 1 hold 64 roots each, every root with at most its first hub_cut
    // tasks of position 1; items from item_split on hold 64 consecutive tasks of
    // the rest, taken from the concatenation of the roots' remaining slices: root
    // i's remainder starts at lcol[vstart[vrow0 + i]] and its first task has index
    // voff[vrow0 + i]; tasks1 such tasks in all
    int32_t vmode;
    uint32_t hub_cut;
    unsigned long long vrow0;
    unsigned long long tasks1;
    unsigned long long item_split;
    // order of a depth-1 share: root r is pool row row0 + (r * perm_mul) mod rows
    // (perm_mul coprime to rows; 0 = rows in stored order)
    unsigned long long perm_mul;
    // symmetry breaking (opt-in): bit j of sb_lt[i] requires M(phi[j]) < M(phi[i]),
    // bit j of sb_gt[i] requires M(phi[i]) < M(phi[j]), for j < i
    uint32_t sb_lt[kMaxK];
    uint32_t sb_gt[kMaxK];
    // rows per work item of the pool's first part (0 = 64, one per lane): fewer
    // when a query has few roots, so that more wavefronts start at once
    uint32_t rpi;
    uint32_t pad_rpi;
    // candidate graph (opt-in): the query edge from position i to position l
    // (i a backward neighbour) is list gslot[l] + (backward neighbours of l
    // before i) of SearchArgs::gbounds
    uint32_t gslot[kMaxK];
};

// Per-query results of a launch.  The count (atomics from every wavefront on
// the query) and the abort word (polled by them) sit on separate 128-byte
// lines: sharing one line costs about half the throughput of a single query.
struct alignas(128) QCtl {
    unsigned long long count;        // matches found (flushed by wavefronts)
    unsigned long long pad0[15];
    unsigned int abort;              // kAbortCap once the count reached the cap, kAbortTime
                                     // once work remained past the query's time limit
    unsigned int pad1;
    unsigned long long t_start;      // device wall clock when its first work item was claimed
    unsigned long long pad2[14];
    unsigned long long groups;
    unsigned long long tasks;
    unsigned long long scanned;      // candidates read from label slices
    unsigned long long lookups;      // label-slice bound lookups
    unsigned long long probes;
    unsigned long long lanes_active;
    unsigned long long lanes_issued;
    unsigned long long steals;
    // device wall clock of the last flush of this query's counters by any
    // wavefront (with t_start, the query's device time in a batched launch)
    unsigned long long t_last;
    // bytes the search kernel requested from device memory (reads and writes)
    // for this query; bytes_late: those of the last 32-round window of each
    // wavefront in which it saw the query's (or the launch's) abort word, an
    // upper bound on the work done after the cap or time limit was reached
    unsigned long long bytes;
    unsigned long long bytes_late;
    int live;                        // work units (items, donations) taken and not finished
    int pad3[9];
};

static_assert(sizeof(QCtl) == 384 && offsetof(QCtl, abort) == 128 && offsetof(QCtl, groups) == 256,
              "hot words of QCtl must sit on lines of their own");

// Device-resident control block of a launch.  Words that many wavefronts hit
// with atomics or polls live on cache lines of their own (128 B).
struct alignas(128) Control {
    unsigned long long out_rows;     // rows appended (root scan, expansion, enumerate)
    unsigned long long pad_rows[15];
    unsigned int abort;              // kAbortNone, or kAbortTime (stops the whole launch)
    unsigned int pad_abort[31];
    int busy;                        // wavefronts holding work (donations count from hand-over)
    int pad_busy[31];
    int idle_count;                  // wavefronts whose bit is set in the idle bitmap
    int pad_idle[31];
    // written once per launch or read by the host only
    unsigned long long measure;      // bound on the next pool level (sum of smallest label slices)
    unsigned long long t0;           // device wall clock at the start of the search
    unsigned long long pad_cold[14];
};

// A stream of work items: the items of queries plan0 .. plan1 - 1, one query
// after the other (each plan's item0 / item_end count from the stream's start).
// Every wavefront has a home stream and moves on to the next stream once its
// own runs dry, so a launch holds as many queries in flight as it has streams.
struct alignas(128) StreamCtl {
    unsigned long long next;         // next unclaimed item of this stream
    unsigned long long pad0[15];
    unsigned long long items;        // items in the stream
    int32_t plan0, plan1;            // its queries
    unsigned long long pad1[14];
};

static_assert(sizeof(StreamCtl) == 256, "StreamCtl: claim counter on a line of its own");

// Mailbox of one wavefront for dynamic balancing (Sec. 4.3): an idle wavefront
// sets its bit in the idle bitmap and polls only its own mailbox; a busy one
// claims a bit and writes the donated work here.  The work is the
// partial matches of the donor's parent lanes pi..ei at level `depth` and the
// task range from (pi, pj) up to, not including, (ei, ej) of that level's
// virtual task pool.
struct alignas(128) Mailbox {
    unsigned int status;             // kMailEmpty / kMailWaiting / kMailFull
    int32_t depth, pi, pj, ei, ej;
    unsigned long long lanes;        // parent lanes present
    int32_t qid;                     // query of the donated work
    int32_t pad[23];
    int32_t rows[kWave * kMaxK];     // rows[q * kMaxK + i] = image of position i for parent lane q
};

enum : unsigned int { kMailEmpty = 0, kMailWaiting = 1, kMailFull = 2 };

enum : unsigned int { kAbortNone = 0, kAbortCap = 1, kAbortTime = 2 };

// Arguments of every search kernel (passed by value in the kernarg segment).
struct SearchArgs {
    const VInfo *vinfo;        // [n]
    const int32_t *col;        // [nnz] neighbour lists, ids ascending (membership tests)
    const int32_t *lcol;       // [nnz] the same lists ordered by (label, id) (candidate scans)
    const uint32_t *loff;      // label slice bounds: N(v) with label c is
                               // lcol[loff[v*stride + c] .. loff[v*stride + c + 1])
    int32_t loff_stride;       // labels + 1, or 1 when lists are not partitioned (c = 0)
    const int32_t *hub_id;     // [n] index of v's adjacency bitmap, -1 if none (null: no bitmaps)
    const uint32_t *hub_bits;  // hub h's bitmap: bit u of hub_bits[h * hub_words ..] set iff u in N(v)
    unsigned long long hub_words;
    const Plan *plans;         // [nq] device copies of the query plans
    QCtl *qctl;                // [nq] per-query results
    int32_t nq;                // queries in this launch
    int32_t levels;            // stack levels per wavefront: the largest k of the launch
    const int32_t *pool;       // pool rows of every query (each plan gives its share)
    const uint32_t *voff;      // virtual level-1 pools: first task index of each root
    const uint32_t *vstart;    //   ... start of each root's candidate slice in lcol
    StreamCtl *streams;        // [nstreams] work-item streams
    int32_t nstreams;
    int32_t *out;              // expansion: next pool; enumerate: rows
    unsigned long long out_cap; // rows that fit in out
    Control *ctl;
    unsigned long long budget; // time limit in device wall-clock ticks from ctl->t0, 0 = none
    Mailbox *mail;             // one per wavefront (work stealing), or null
    unsigned long long *idle_bits; // bit w set: wavefront w waits for work
    int32_t steal_slots;       // number of mailboxes (>= wavefronts launched)
    int32_t steal_threshold;
    int32_t slim;              // 1: slim stack layout (membership tests on label slices)
    int32_t sb;                // 1: some plan of the launch has symmetry-breaking conditions
    int32_t cg;                // 1: search the candidate graph: lcol holds its lists, and the list of
                               // query edge e for vertex v is lcol[gbounds[2 * (e * gn + v)] ..
                               // gbounds[2 * (e * gn + v) + 1])
    const uint32_t *gbounds;
    unsigned long long gn;     // |V(G)|
    int32_t measure_next;      // expansion: add the next level's size bound to ctl->measure
    int32_t merge_slots;       // LDS-staged intersection: staging entries per lane, 0 = off (slim
                               // layout only); a run of r candidates stages a list of n <= slots * r
    int32_t merge_auto;        // 1: the launch drops the staging area where it costs residency
    // parked task groups: levels x 64 entries of 8 bytes per wavefront, for up to
    // park_waves wavefronts (a launch never has more)
    uint2 *parked;
    int32_t park_waves;
};

// Candidate graph of one query (candidate.hip).  Positions follow the
// matching order; adj[l] bit j: positions l and j are adjacent in Q.
struct CandQuery {
    int32_t k;
    int32_t lab[kMaxK];
    int32_t qdeg[kMaxK];
    uint32_t adj[kMaxK];
};

constexpr int kMaxCandEdges = kMaxK * (kMaxK - 1) / 2;

// Query edge e = (src, dst), src before dst in the order: its lists belong to
// the candidates clist[start .. start + len) of src, and their lengths and
// offsets sit at first .. first + len - 1 of the per-edge arrays.  One entry
// per query edge in a small device table.
struct CandEdge {
    int32_t src, dst;
    uint32_t start, len;
    uint32_t first;
    uint32_t pad[3];
};

// Words of one position's bitmap (a multiple of two: 64 vertices per wavefront).
unsigned long long cand_bitmap_words(int32_t n);
// Scratch words launch_exclusive_scan needs for m values.
unsigned long long cand_scan_temp_words(unsigned long long m);
// C0 of every position into bits (q.k rows of cand_bitmap_words(n) words).
hipError_t launch_cand_init(const VInfo *vinfo, int32_t n, const CandQuery &q, uint32_t *bits, int num_cu,
                            hipStream_t s);
// One sweep of the support filter; sets *changed to 1 if it cleared a bit.
hipError_t launch_cand_refine(const int32_t *lcol, const uint32_t *loff, int32_t stride, int32_t n,
                              const CandQuery &q, uint32_t *bits, uint32_t *changed, int num_cu, hipStream_t s);
// Candidate lists of all k positions, ids ascending, into clist; bounds[l] ..
// bounds[l + 1] is position l's (k + 1 words).  rank: k * cand_bitmap_words(n)
// words of scratch; tmp: prefix-sum scratch for as many values.
hipError_t launch_cand_lists(const uint32_t *bits, int32_t n, int32_t k, uint32_t *rank, uint32_t *tmp,
                             int32_t *clist, uint32_t *bounds, int num_cu, hipStream_t s);
// List lengths of the m query edges into cnt (most = the largest len) and their
// sum (added to *total).
hipError_t launch_cand_count(const int32_t *lcol, const uint32_t *loff, int32_t stride, int32_t n,
                             const CandQuery &q, const uint32_t *bits, const CandEdge *edges, int32_t m,
                             unsigned long long most, const int32_t *clist, uint32_t *cnt, unsigned long long *total,
                             int num_cu, hipStream_t s);
// The lists at offsets offs (the exclusive prefix sum of the lengths) and their
// bounds in gbounds (2 words per edge and vertex, m * n * 2 in all).
hipError_t launch_cand_fill(const int32_t *lcol, const uint32_t *loff, int32_t stride, int32_t n,
                            const CandQuery &q, const uint32_t *bits, const CandEdge *edges, int32_t m,
                            unsigned long long most, const int32_t *clist, const uint32_t *offs, int32_t *gcol,
                            uint32_t *gbounds, int num_cu, hipStream_t s);
// In-place exclusive prefix sum of m uint32 values whose total fits 32 bits;
// tmp holds cand_scan_temp_words(m) words.
hipError_t launch_exclusive_scan(uint32_t *x, unsigned long long m, uint32_t *tmp, hipStream_t s);

// Launchers implemented in kernels.hip.  All return hipSuccess or the launch error.
// measure_lab >= 0: also add up the candidates' label slices for position 1
// (label id measure_lab) into ctl->measure, the bound of the next pool level.
hipError_t launch_root_scan(const VInfo *vinfo, int32_t n, int32_t lab0, int32_t qdeg0, int32_t *pool,
                            const uint32_t *loff, int32_t loff_stride, int32_t measure_lab, Control *ctl, int num_cu,
                            hipStream_t s);
hipError_t launch_expand(const SearchArgs &a, int num_cu, hipStream_t s);
hipError_t launch_search(const SearchArgs &a, bool enumerate, int num_cu, int waves_per_cu, hipStream_t s,
                         int *grid_waves_out);
// Writes the device wall clock into ctl->t0 (start of a search's time budget).
hipError_t launch_start_clock(Control *ctl, hipStream_t s);
// Second phase of a two-phase pool: per root (roots in the order given by
// perm_mul), the part of its position-1 slice (label id lab1; the whole list
// when stride == 1) beyond its first hub_cut tasks: start in lcol and length;
// adds those candidates to qc->scanned.  Then voff = exclusive prefix sum of the
// lengths (tmp: R / 4096 + 2 words), and plan->tasks1, plan->item_end and
// sc->items are set from the total.
hipError_t launch_level1(const int32_t *roots, int32_t R, unsigned long long perm_mul, uint32_t hub_cut,
                         const uint32_t *loff, int32_t stride, int32_t lab1, uint32_t *lens, uint32_t *vstart,
                         uint32_t *voff, uint32_t *tmp, QCtl *qc, Plan *plan, StreamCtl *sc, int num_cu,
                         hipStream_t s);
// Wavefronts a depth-first search launch for a query of `levels` positions keeps resident.
int search_waves(int levels, int num_cu, int waves_per_cu, bool slim, int merge_slots, bool merge_auto);
hipError_t launch_steal_init(Mailbox *mail, unsigned long long *idle_bits, int32_t n, hipStream_t s);

// Allocation-free count (scratch.hip): device address of this device's
// kScratchBytes arena (looked up once per device, which must be current), and
// a kernel that zeroes words of it.
hipError_t scratch_area(int device, void **out);
hipError_t launch_zero_words(void *p, unsigned long long words, hipStream_t s);

// Graph load (graph_build.hip).  Error bits of the checks:
enum : unsigned int { kGraphBadRowPtr = 1, kGraphBadEntry = 2, kGraphBadDegree = 4, kGraphAsymmetric = 8 };
// entries = false: row offsets (start at 0, non-decreasing, degrees < 2^24);
// entries = true (only after the offsets passed): ids in [0, n), rows strictly
// ascending, no self-loops, and symmetry if asked.  ORs error bits into *err.
hipError_t launch_graph_check(const void *row_ptr, int row_ptr_bytes, const int32_t *col, int32_t n, bool symmetric,
                              unsigned int *err, bool entries, int num_cu, hipStream_t s);
// hist256[c] += number of vertices with label value c.
hipError_t launch_label_hist(const uint8_t *labels, int32_t n, unsigned int *hist256, int num_cu, hipStream_t s);
// clab[v] = map256[labels[v]] (compact label ids).
hipError_t launch_label_map(const uint8_t *labels, int32_t n, const uint8_t *map256, uint8_t *clab, int num_cu,
                            hipStream_t s);
// Vertex records; with stride > 1 the label slices (loff [n * stride], lcol [nnz]),
// else loff [n + 1] = the row offsets as 32-bit values (lcol unused).
hipError_t launch_graph_build(const void *row_ptr, int row_ptr_bytes, const int32_t *col, const uint8_t *clab,
                              int32_t n, int32_t stride, VInfo *vinfo, uint32_t *loff, int32_t *lcol, int num_cu,
                              hipStream_t s);
// Adjacency bitmaps of the hubs hubs[0 .. nh) (bits cleared beforehand) and
// hub_id[hubs[h]] = h (hub_id set to -1 beforehand).
hipError_t launch_hub_bitmaps(const VInfo *vinfo, const int32_t *col, const int32_t *hubs, int32_t nh, uint32_t *bits,
                              unsigned long long words, int32_t *hub_id, int num_cu, hipStream_t s);

}  // namespace gm
