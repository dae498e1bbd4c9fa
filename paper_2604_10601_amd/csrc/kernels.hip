// gfx950 (CDNA4) kernels of the matching engine.
//
// Method (gMatch paper, arXiv 2604.10601):
//   * Fine-grained tasks (Sec. 4.1): extending a partial match M by the next query
//     vertex u is split into one task per local candidate v in C^L_M(u), the
//     neighbour list of the backward neighbour whose image has the fewest
//     neighbours.  One lane validates one task.
//   * Batch exploration (Sec. 4.2, Alg. 2): a wavefront keeps up to 64 partial
//     matches per level in an LDS stack S[level][lane] = {v, parent lane}; the
//     task groups of all of them form one virtual task pool that two cursors
//     (parent lane, offset in its list) walk 64 tasks at a time.  Partial
//     matches are rebuilt by following parent pointers down the stack.
//   * Initial pool (Sec. 4.3): wavefronts claim work items with an atomic
//     counter.  By default the pool is two-phase: first-phase items hold 64
//     candidates of the first query vertex, each with at most its first
//     hub_cut tasks at position 1; second-phase items are 64 consecutive tasks
//     of the rest of those position-1 lists, laid out by a prefix sum.  With
//     tau > 0 the paper's own scheme runs instead: breadth-first expansion
//     until a level holds at least tau partial matches, then rows of it.
//
// gfx950 design, which differs from the paper's 32-lane CUDA design:
//   * 64-lane wavefronts: the stack is K x 64, ballots are 64-bit.
//   * ScatterTask is done by the whole wavefront at once instead of a serial
//     loop on one lane: an exclusive scan of the per-parent remaining list
//     lengths (clamped to 64, so seven ballots + mbcnt give the scan), a start
//     marker per parent in LDS, and a find-last-set per lane give every lane
//     its parent and offset.
//   * A wavefront claims 64 pool rows at a time, one per lane, so the first
//     level is already a full batch.
//   * Two stack layouts: the slim default keeps only each entry's vertex and
//     parent lane, and membership tests bisect label slices of N(w) whose
//     bounds cost one lookup; the full layout also caches each entry's list
//     start and degree, so tests bisect the id-sorted lists with no lookup.
//   * Per-vertex data is one packed 8-byte record (list start, degree, label):
//     a single load decides the label and degree filters.
//   * Membership is bisection while the remaining range is longer than a few
//     entries, then one batch of independent loads (fewer dependent round trips).
//   * The search is one persistent launch; waves exit when the pool is empty,
//     or when the cap or the time limit sets the abort word.
#include <hip/hip_runtime.h>

#include "gm_internal.h"

namespace gm {

namespace {

constexpr int kWavesPerBlock = 1;
constexpr int kBlock = kWave * kWavesPerBlock;

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

// Plans are read through the constant address space: with a wave-uniform query
// index every field is a scalar load, as if the plan were a kernel argument.
typedef const __attribute__((address_space(4))) Plan *PlanPtr;

__device__ __forceinline__ PlanPtr plan_at(const SearchArgs &a, int32_t q) {
    return reinterpret_cast<PlanPtr>(reinterpret_cast<uintptr_t>(a.plans)) + q;
}

// Stored position of root r of a depth-1 share of n rows visited in the order
// r -> (r * mul) mod n (mul coprime to n); mul = 0 keeps the stored order.
__host__ __device__ __forceinline__ unsigned long long permuted(unsigned long long r, unsigned long long mul,
                                                                unsigned long long n) {
    return mul ? (r * mul) % n : r;
}

// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t popc_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Value of lane `src` (wave-uniform index) for every lane.
__device__ __forceinline__ uint32_t read_lane(uint32_t x, uint32_t src) {
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), static_cast<int>(src)));
}

__device__ __forceinline__ unsigned long long read_lane64(unsigned long long x, uint32_t src) {
    uint32_t lo = read_lane(static_cast<uint32_t>(x), src);
    uint32_t hi = read_lane(static_cast<uint32_t>(x >> 32), src);
    return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// Value held by lane `src` (per-lane index), through the LDS crossbar.
__device__ __forceinline__ uint32_t shfl(uint32_t x, uint32_t src) {
    return static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(static_cast<int>(src << 2), static_cast<int>(x)));
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
    for (int off = 32; off >= 1; off >>= 1) {
        uint32_t lo = static_cast<uint32_t>(x), hi = static_cast<uint32_t>(x >> 32);
        uint32_t src = lane_id() ^ off;
        lo = shfl(lo, src);
        hi = shfl(hi, src);
        x += (static_cast<uint64_t>(hi) << 32) | lo;
    }
    return x;
}

// Membership of v in the ascending list col[lo, lo + n) (Sec. 5.2 costs each
// test as one binary search).  A lower-bound bisection with no early exit keeps
// the invariant "the first entry >= v lies in [lo, lo + n]" and halves n until
// fewer than kTail entries remain; the step is a select, not a branch, so a
// wavefront pays one compare and two selects per probe and no per-lane control
// flow.  The tail is then read as one window of kTail consecutive entries that
// ends at min(lo + kTail - 1, last entry) (starting at index 0 if that is
// lower); only window entries inside [lo, last entry] count.  Every array
// searched here holds at least kTail entries, so the window stays inside it,
// and one base address with constant offsets lets all kTail loads be in flight
// together (a clamped index per load costs an address pair each, and under
// register pressure the loads were issued one round trip at a time).
// (Bisecting several lists in lockstep, one round trip for all of them, cost
// more instructions per candidate than it saved: same box, the 8-vertex
// workload ran at 34.7, 37.1 and 38.5 G embeddings/s with four, two and one
// lists, the 12-32-vertex sample at 14.6, 15.4 and 15.7.)  Adds the entries
// examined to probes and the bytes of the loads issued to bytes.
// Tail of 8 entries (one or two 64-byte sectors): against 4, +1 % on the
// 8-vertex workload and +3 % on the 12-32-vertex sample.
constexpr uint32_t kTail = static_cast<uint32_t>(kListWindow);

__device__ __forceinline__ bool in_list(const int32_t *__restrict__ col, uint32_t lo, uint32_t n, int32_t v,
                                        uint32_t &probes, uint32_t &bytes) {
    const uint32_t last = lo + n - 1u;  // callers pass n >= 1
    while (n >= kTail) {
        const uint32_t h = n >> 1;
        const int32_t x = col[lo + h];
        lo = x < v ? lo + h : lo;
        n -= h;
        ++probes;
        bytes += 4u;
    }
    const uint32_t hi = lo + (kTail - 1u) < last ? lo + (kTail - 1u) : last;
    const uint32_t p = hi >= kTail - 1u ? hi - (kTail - 1u) : 0u;
    const int32_t *w = col + p;
    int32_t x[kTail];
#pragma unroll
    for (uint32_t j = 0; j < kTail; ++j) x[j] = w[j];
    const uint32_t jlo = lo - p, span = hi - lo;  // counted entries: j in [jlo, jlo + span]
    uint32_t hit = 0;
#pragma unroll
    for (uint32_t j = 0; j < kTail; ++j) hit |= static_cast<uint32_t>(x[j] == v) << j;
    probes += span + 1u;
    bytes += 4u * kTail;  // the whole window is read
    return ((hit >> jlo) & ((2u << span) - 1u)) != 0u;
}

// Per-wavefront stack in LDS (Sec. 5.1: S is |V(Q)| x warp width) for exactly k
// levels (the launch sizes the dynamic LDS from the query).  Element (level i,
// lane q) of a plane is at [i * 64 + q].  Two layouts:
//   full (12 B per (level, lane)): the entry caches its vertex's id-sorted list
//     start and degree, so membership tests bisect N(w) with no extra load;
//   slim (4 B): the entry keeps only its vertex and parent lane, packed in one
//     word (graphs of at most 2^24 vertices); membership tests bisect the
//     label slice of N(w) in lcol (ids ascending within a label), whose bounds
//     cost one 8-byte load per list but which is shorter than N(w).
// The task group of each parent lane (its candidate slice: start in lcol and
// length << 8 | source level) is needed only while its level is the one being
// scattered, so the current level's sits in two registers per lane, and a
// descent parks it in the wavefront's area of device memory (Slice, 8 B per
// (level, lane), one coalesced 512-byte store) until the backtrack that loads
// it again.  That keeps 512 B per level out of LDS: a 32-vertex query's stack
// takes 8.6 KB instead of 27 KB, so 18 wavefronts fit per CU instead of 5.
struct WaveStack {
    uint32_t *e;      // slim: data vertex | lane of the parent entry at level - 1 << 24
    int32_t *v;       // full: data vertex of the task at (level, lane)
    uint32_t *st;     // full: start of N(v) in col[] (ids ascending)
    uint32_t *dp;     // full: |N(v)| << 8 | lane of the parent entry at level - 1
    uint32_t *cur_j;  // per level: scatter cursor, offset in the current parent's slice
    uint32_t *cur_i;  //   ... current parent lane (64 = level exhausted)
    uint32_t *end_j;  // per level: end of the task range, offset in parent end_i's slice
    uint32_t *end_i;  //   ... parent lane (64 = no bound: the whole pool)
    uint8_t *own;     // scatter scratch: parent starting at each slot
};

// Entry planes of a stack for queries of up to `levels` positions: the last
// position is counted (or written out) where it is tested and never pushed, so
// levels - 1 planes hold every entry (one for a one-vertex query, whose pool rows
// are its matches).  The scatter cursors are per position, the last included.
__host__ __device__ constexpr int stack_planes(int levels) { return levels > 1 ? levels - 1 : 1; }

__host__ __device__ constexpr size_t stack_bytes(int levels, bool slim) {
    return static_cast<size_t>(stack_planes(levels)) * kWave * (slim ? 4u : 12u) +
           static_cast<size_t>(levels) * 16u + kWave;
}

// Task group of one parent lane at one level: cs = start of its candidate slice
// in lcol, cl = slice length << 8 | the level of its source list (0xff: none).
struct Slice {
    uint32_t cs, cl;
};

template <bool SLIM>
__device__ __forceinline__ WaveStack carve_stack(uint8_t *base, int levels) {
    WaveStack S;
    const size_t plane = static_cast<size_t>(stack_planes(levels)) * kWave * 4u;
    uint8_t *p = base;
    if (SLIM) {
        S.e = reinterpret_cast<uint32_t *>(p);
        S.v = nullptr;
        S.st = nullptr;
        S.dp = nullptr;
        p += plane;
    } else {
        S.e = nullptr;
        S.v = reinterpret_cast<int32_t *>(p);
        S.st = reinterpret_cast<uint32_t *>(p + plane);
        S.dp = reinterpret_cast<uint32_t *>(p + 2 * plane);
        p += 3 * plane;
    }
    p = base + (static_cast<size_t>(p - base) + 3u) / 4u * 4u;
    uint32_t *lv = reinterpret_cast<uint32_t *>(p);
    S.cur_j = lv;
    S.cur_i = lv + levels;
    S.end_j = lv + 2 * levels;
    S.end_i = lv + 3 * levels;
    S.own = reinterpret_cast<uint8_t *>(lv + 4 * levels);
    return S;
}

__device__ __forceinline__ uint32_t ent_deg(const WaveStack &S, int i, uint32_t q) { return S.dp[i * kWave + q] >> 8; }

// The slim entry packs the vertex (ids below 2^24: the engine picks the full
// layout for larger graphs) and the parent lane into one word, so one LDS read
// gives both.
constexpr uint32_t kSlimVertexMask = 0xffffffu;

template <bool SLIM>
__device__ __forceinline__ int32_t ent_v(const WaveStack &S, int i, uint32_t q) {
    if (SLIM) return static_cast<int32_t>(S.e[i * kWave + q] & kSlimVertexMask);
    return S.v[i * kWave + q];
}

template <bool SLIM>
__device__ __forceinline__ uint32_t ent_pid(const WaveStack &S, int i, uint32_t q) {
    if (SLIM) return S.e[i * kWave + q] >> 24;
    return S.dp[i * kWave + q] & 0xffu;
}

template <bool SLIM>
__device__ __forceinline__ void push_entry(WaveStack &S, int i, uint32_t lane, int32_t v, VInfo vi, uint32_t pid) {
    if (SLIM) {
        // lanes without a task push -1: masked, never read as a match
        S.e[i * kWave + lane] = (static_cast<uint32_t>(v) & kSlimVertexMask) | (pid << 24);
    } else {
        S.v[i * kWave + lane] = v;
        S.st[i * kWave + lane] = vi.x;
        S.dp[i * kWave + lane] = (vi_deg(vi) << 8) | pid;
    }
}

// Candidate-graph list of the query edge from position i (a backward neighbour
// of l) to position l: the edges of position l are numbered from gslot[l] in
// the order of their backward positions.
__device__ __forceinline__ uint32_t cg_slot(PlanPtr P, int l, uint32_t bw, int i) {
    return P->gslot[l] + static_cast<uint32_t>(__builtin_popcount(bw & ((1u << i) - 1u)));
}

struct Gen {
    uint32_t tasks;    // |C^L| by the paper's rule: the smallest backward list
    uint32_t scanned;  // length of the label slice that is actually scanned
    uint32_t lookups;  // slice bounds read
    uint32_t bytes;    // device-memory bytes those reads requested
    Slice sl;          // this lane's task group at the new level
};

// GenerateTask (Alg. 2): for every parent lane in F at level l-1, walk its chain
// and choose the local candidates among its backward neighbours' lists.  The
// paper takes the whole list of the neighbour with the fewest neighbours
// (Sec. 4.1), and that length is what `tasks` counts.  With label-partitioned
// lists only the slice of candidates labelled L(phi[l]) can pass the label
// check, so the smallest such slice is scanned instead (earliest position on
// ties); it yields exactly the same valid extensions.
template <bool SLIM, bool CG = false>
__device__ __forceinline__ Gen generate_tasks(WaveStack &S, const SearchArgs &a, PlanPtr P, int l, uint64_t F,
                                              uint32_t lane) {
    Gen g{0u, 0u, 0u, 0u, {0u, 0xffu}};
    uint32_t cs = 0, cl = 0xffu;
    if ((F >> lane) & 1ull) {
        const uint32_t bw = P->bwd[l];
        const int lowest = __builtin_ctz(bw);
        const int stride = a.loff_stride;
        const bool sliced = stride > 1;
        const uint32_t lab = sliced ? static_cast<uint32_t>(P->lab[l]) : 0u;
        uint32_t q = lane;
        uint32_t best_full = 0xffffffffu, best_n = 0xffffffffu, best_a = 0, best_j = 0;
        for (int i = l - 1; i >= lowest; --i) {
            if ((bw >> i) & 1u) {
                uint32_t d, sa, sn;
                if (CG) {
                    // candidate graph: N(w) restricted to C(phi[l]), one list per query edge
                    const uint32_t *o =
                        a.gbounds + 2ull * (static_cast<unsigned long long>(cg_slot(P, l, bw, i)) * a.gn +
                                            static_cast<uint32_t>(ent_v<SLIM>(S, i, q)));
                    sa = o[0];
                    sn = o[1] - sa;
                    d = sn;
                    ++g.lookups;
                    g.bytes += 8u;
                } else if (SLIM) {
                    // list bounds and slice bounds: three independent loads (the slice's
                    // two bounds are adjacent), all issued before any is used
                    const uint32_t *o = a.loff + static_cast<unsigned long long>(ent_v<SLIM>(S, i, q)) * stride;
                    uint2 sb;
                    __builtin_memcpy(&sb, o + lab, sizeof(sb));
                    const uint32_t row0 = o[0];
                    const uint32_t rowe = o[stride - 1 + (sliced ? 0 : 1)];
                    d = rowe - row0;  // whole list: first to last bound
                    sa = sb.x;
                    sn = sb.y - sb.x;
                    ++g.lookups;
                    g.bytes += 16u;  // list bounds and slice bounds
                } else {
                    d = ent_deg(S, i, q);
                    if (sliced) {
                        const uint32_t *o = a.loff + static_cast<unsigned long long>(ent_v<SLIM>(S, i, q)) * stride + lab;
                        sa = o[0];
                        sn = o[1] - sa;
                        ++g.lookups;
                        g.bytes += 8u;
                    } else {
                        sa = S.st[i * kWave + q];
                        sn = d;
                    }
                }
                best_full = d < best_full ? d : best_full;
                if (sn <= best_n) {
                    best_n = sn;
                    best_a = sa;
                    best_j = static_cast<uint32_t>(i);
                }
            }
            q = ent_pid<SLIM>(S, i, q);
        }
        g.tasks = best_full;
        g.scanned = best_n;
        cs = best_a;
        cl = (best_n << 8) | best_j;
    }
    g.sl.cs = cs;
    g.sl.cl = cl;
    return g;
}

__device__ __forceinline__ void open_level(WaveStack &S, int l, uint32_t lane) {
    if (lane == 0) {
        S.cur_i[l] = 0;
        S.cur_j[l] = 0;
        S.end_i[l] = kWave;
        S.end_j[l] = 0;
    }
}

// Unscattered tasks of this lane's task group (slice sl), given its level's
// cursor (ci, cjo) and end (ei, ej).  Also returns the group's slice.
__device__ __forceinline__ uint32_t remaining(Slice sl, uint32_t lane, uint32_t ci, uint32_t cjo, uint32_t ei,
                                              uint32_t ej, uint32_t &cst, uint32_t &cln) {
    cst = sl.cs;
    cln = sl.cl >> 8;
    if (lane < ci || lane > ei) return 0u;
    const uint32_t lo = lane == ci ? cjo : 0u;
    const uint32_t hi = lane == ei ? (ej < cln ? ej : cln) : cln;
    return hi > lo ? hi - lo : 0u;
}

struct Round {
    uint32_t ntask;  // tasks this round (0: level exhausted)
    uint32_t owner;  // parent lane of this lane's task
    int32_t v;       // candidate of this lane's task (valid if lane < ntask)
    uint32_t run;    // lanes [run & 0xff, run >> 8) hold this parent's tasks of the round (ascending ids)
    uint32_t js;     // level of the backward neighbour whose list the candidate came from
};

// ScatterTask (Alg. 2) for the whole wavefront: hand the next <= 64 tasks of
// level l to lanes 0..ntask-1 and advance the level's cursor.
__device__ __forceinline__ Round scatter(WaveStack &S, const int32_t *__restrict__ lcol, int l, uint32_t lane,
                                        Slice sl) {
    Round r;
    const uint32_t ci = __builtin_amdgcn_readfirstlane(S.cur_i[l]);
    const uint32_t cjo = __builtin_amdgcn_readfirstlane(S.cur_j[l]);
    const uint32_t ei = __builtin_amdgcn_readfirstlane(S.end_i[l]);
    const uint32_t ej = __builtin_amdgcn_readfirstlane(S.end_j[l]);
    uint32_t cst, cln;
    const uint32_t rem = remaining(sl, lane, ci, cjo, ei, ej, cst, cln);
    const uint32_t rc = rem < 64u ? rem : 64u;
    // exclusive scan of rc (values <= 64: seven bit planes)
    uint32_t ex = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < 7; ++b) {
        uint64_t m = ballot((rc >> b) & 1u);
        ex += popc_below(m) << b;
        tot += static_cast<uint32_t>(__popcll(m)) << b;
    }
    if (tot == 0) {
        r.ntask = 0;
        r.owner = 0;
        r.v = -1;
        r.run = 0;
        r.js = 0xffu;
        return r;
    }
    r.ntask = tot < 64u ? tot : 64u;
    volatile uint8_t *own = S.own;
    own[lane] = 0xffu;
    __builtin_amdgcn_wave_barrier();
    if (rc != 0u && ex < 64u) own[ex] = static_cast<uint8_t>(lane);
    __builtin_amdgcn_wave_barrier();
    const uint32_t o = own[lane];
    const uint64_t starts = ballot(o != 0xffu);
    const uint64_t upto = lane == 63u ? ~0ull : ((2ull << lane) - 1ull);
    const uint32_t s = 63u - static_cast<uint32_t>(__clzll(starts & upto));
    const uint64_t later = starts & ~upto;  // runs starting after this lane
    const uint32_t e = later ? static_cast<uint32_t>(__builtin_ctzll(later)) : 64u;
    r.run = s | ((e < r.ntask ? e : r.ntask) << 8);
    const uint32_t owner = shfl(o, s);
    const uint32_t ocst = shfl(cst, owner);
    r.js = shfl(sl.cl, owner) & 0xffu;
    const uint32_t j = lane - s + (owner == ci ? cjo : 0u);
    r.owner = owner;
    r.v = lane < r.ntask ? lcol[ocst + j] : -1;
    // advance the cursor past slot 63; rc is clamped, so a lone parent with more
    // than 64 tasks left shows up only in rem
    if (tot > 64u || ballot(rem > rc) != 0ull) {
        const uint32_t p63 = read_lane(owner, 63);
        const uint32_t s63 = read_lane(s, 63);
        const uint32_t used = 64u - s63 + (p63 == ci ? cjo : 0u);
        const uint32_t len63 = read_lane(cln, p63);
        const uint32_t stop63 = p63 == ei ? (ej < len63 ? ej : len63) : len63;
        if (lane == 0) {
            if (used >= stop63) {
                S.cur_i[l] = p63 + 1;
                S.cur_j[l] = 0;
            } else {
                S.cur_i[l] = p63;
                S.cur_j[l] = used;
            }
        }
    } else if (lane == 0) {
        S.cur_i[l] = 64;
    }
    return r;
}

// Bits [lo, hi) of a 64-bit lane mask.
__device__ __forceinline__ uint64_t lane_range(uint32_t lo, uint32_t hi) {
    const uint64_t below_hi = hi >= 64u ? ~0ull : ((1ull << hi) - 1ull);
    return below_hi & ~((1ull << lo) - 1ull);
}

// LDS-staged intersection (Sec. 5.2 costs each membership test as one binary
// search; here a run of candidates shares one list).  The lanes calling this
// together belong to one or more runs; within a run every lane tests the same
// ascending list B = list[0 .. n) and the run's candidates, taken in lane order,
// form the ascending sequence A (distinct ids).  The run's lanes load B into
// their share of the staging area (slots entries per lane, so n <= slots * r
// fits), write A next to it, and intersect the two by merge path (Green,
// McColl and Bader, 2012): the merge of A and B (A first on ties) is cut into
// r segments of equal length, lane j finds where segment j starts by bisecting
// its diagonal, then walks the segment.  When the walk takes A[x] it has just
// passed every entry of B below A[x], so A[x] is in B iff the next entry of B
// equals it; lane j writes that into flag x, and each lane reads its own flag.
// A list longer than twice the run makes that walk long, so there each lane
// bisects the staged copy instead: merge path or binary search, picked by the
// ratio of list length to run.  One wavefront's LDS operations complete in
// issue order, so the writes of one step are seen by the reads of the next.
// Adds the entries this lane loaded to probes and their bytes to bytes.
__device__ __forceinline__ bool merge_member(const int32_t *__restrict__ list, uint32_t n, uint8_t *area,
                                             uint32_t slots, uint32_t run, int32_t v, uint32_t &probes,
                                             uint32_t &bytes) {
    const uint32_t rs = run & 0xffu, re = run >> 8;
    const uint64_t mine = ballot(true) & lane_range(rs, re);
    const uint32_t r = static_cast<uint32_t>(__popcll(mine));
    const uint32_t j = popc_below(mine);
    int32_t *B = reinterpret_cast<int32_t *>(area) + rs * slots;
    int32_t *A = reinterpret_cast<int32_t *>(area) + kWave * slots + rs;
    uint8_t *F = area + (kWave * slots + kWave) * 4u + rs;
    A[j] = v;
    for (uint32_t k = j; k < n; k += r) {
        B[k] = list[k];
        ++probes;
        bytes += 4u;
    }
    if (n > 2u * r) {
        // a list long against the run: each lane bisects the staged copy in LDS
        // (branch-free lower bound), which costs log2(n) LDS reads instead of the
        // merge walk's (n + r) / r steps after a diagonal search
        uint32_t lo = 0, len = n;
        while (len > 1u) {
            const uint32_t h = len >> 1;
            lo = B[lo + h - 1u] < v ? lo + h : lo;
            len -= h;
        }
        return B[lo] == v;
    }
    const uint32_t total = r + n;
    const uint32_t seg = (total + r - 1u) / r;
    const uint32_t k0 = j * seg < total ? j * seg : total;
    const uint32_t k1 = k0 + seg < total ? k0 + seg : total;
    // split of diagonal k0: the number x of A's entries among the first k0 of the merge
    uint32_t x = k0 > n ? k0 - n : 0u;
    uint32_t xh = k0 < r ? k0 : r;
    while (x < xh) {
        const uint32_t mid = (x + xh) >> 1;
        if (B[k0 - mid - 1u] >= A[mid]) x = mid + 1u;
        else xh = mid;
    }
    uint32_t y = k0 - x;
    for (uint32_t k = k0; k < k1; ++k) {
        if (x < r && (y >= n || A[x] <= B[y])) {
            F[x] = static_cast<uint8_t>(y < n && B[y] == A[x]);
            ++x;
        } else {
            ++y;
        }
    }
    return F[j] != 0;
}

// Membership of v in the list of backward neighbour w at position l (slim
// layout): w's label slice for l's label, or on the candidate graph the list of
// query edge `edge` for w.  One round reads the list bounds and w's hub id; an
// empty list rejects v; a hub's list is answered by one bit of its adjacency
// bitmap; a list short against its run (n <= slots x the run's lanes still
// testing) is staged in LDS and intersected by merge path; any other list is
// bisected in device memory lane by lane (in_list).  Every lane of a run has
// the same w, so the lanes of one run take the same branch.
template <bool CG>
__device__ __forceinline__ bool slim_member(const SearchArgs &a, uint8_t *marea, uint32_t run, uint32_t lab,
                                            uint32_t w, uint32_t edge, int32_t v, uint32_t &probes,
                                            uint32_t &lookups, uint32_t &bytes) {
    const uint32_t *o = CG ? a.gbounds + 2ull * (static_cast<unsigned long long>(edge) * a.gn + w)
                           : a.loff + static_cast<unsigned long long>(w) * a.loff_stride + lab;
    const uint32_t b0 = o[0], b1 = o[1];
    const int32_t hub = a.hub_id ? a.hub_id[w] : -1;  // read in the same round as the bounds
    ++lookups;
    bytes += a.hub_id ? 12u : 8u;
    const uint32_t n = b1 - b0;
    bool in = false;
    if (n != 0u) {
        if (hub >= 0) {
            const uint32_t word =
                a.hub_bits[static_cast<unsigned long long>(hub) * a.hub_words + (static_cast<uint32_t>(v) >> 5)];
            ++probes;
            bytes += 4u;
            in = ((word >> (static_cast<uint32_t>(v) & 31u)) & 1u) != 0u;
        } else {
            // lanes of this run still testing here: all of them reached this point with the same list
            const uint32_t live =
                a.merge_slots > 0 ? static_cast<uint32_t>(__popcll(ballot(true) & lane_range(run & 0xffu, run >> 8)))
                                  : 0u;
            if (n <= static_cast<uint32_t>(a.merge_slots) * live)
                in = merge_member(a.lcol + b0, n, marea, static_cast<uint32_t>(a.merge_slots), run, v, probes, bytes);
            else
                in = in_list(a.lcol, b0, n, v, probes, bytes);
        }
    }
    return in;
}

// Process (Alg. 2): label and degree filters, then one walk down the parent
// chain checking injectivity and membership in every backward neighbour's list
// other than the one the candidate came from, one list at a time.  The walk is
// wave-uniform: every lane steps down its chain (its chain index is always a
// lane of the stack, so a lane that already failed reads inside the stack and
// ignores what it reads), only the membership tests run under the lanes still
// alive, and the wavefront leaves the walk once no lane is.  Keeping the loop
// and the per-level branches scalar removes the per-lane exit masks a
// data-dependent break costs at every level of the chain.
template <bool SLIM, bool SB, bool CG = false>
__device__ __forceinline__ bool process(WaveStack &S, const SearchArgs &a, PlanPtr P, int l, const Round &r,
                                        uint32_t lane, VInfo &vi, uint32_t &probes, uint32_t &lookups,
                                        uint32_t &bytes, uint8_t *marea) {
    bool ok = lane < r.ntask;
    // The vertex record serves the filters only (the slim stack keeps no copy of
    // it), and often they hold already: a label slice holds that label alone,
    // every candidate neighbours a matched vertex (degree >= 1), and a
    // candidate-graph list holds only vertices that passed both filters.
    const bool need = !SLIM || (!CG && (a.loff_stride <= 1 || P->qdeg[l] > 1));
    vi = make_uint2(0u, 0u);
    if (ok && need) {
        vi = a.vinfo[r.v];
        bytes += 8u;
    }
    if (need)
        ok = ok && vi_lab(vi) == static_cast<uint32_t>(P->lab[l]) && vi_deg(vi) >= static_cast<uint32_t>(P->qdeg[l]);
    if (ballot(ok) == 0ull) return false;
    const uint32_t bw = P->bwd[l];
    // symmetry-breaking conditions: only in launches that hold a query with them
    const uint32_t sblt = SB ? P->sb_lt[l] : 0u, sbgt = SB ? P->sb_gt[l] : 0u;
    // the backward neighbour whose list the candidate came from needs no test;
    // it is the same for every lane of a run
    const uint32_t js = r.js;
    const uint32_t lab = a.loff_stride > 1 ? static_cast<uint32_t>(P->lab[l]) : 0u;
    // the verdict is kept as data (0 or 1) rather than as
    // a branch condition, so it is a plain register across the levels
    uint32_t okv = ok ? 1u : 0u;
    uint32_t q = r.owner;
    for (int i = l - 1; i >= 0; --i) {
        const int32_t w = ent_v<SLIM>(S, i, q);
        const uint32_t below = ent_pid<SLIM>(S, i, q);
        okv = w != r.v ? okv : 0u;
        if (SB) {
            const bool lt = ((sblt >> i) & 1u) != 0u, gt = ((sbgt >> i) & 1u) != 0u;
            okv = (!lt || w < r.v) && (!gt || r.v < w) ? okv : 0u;
        }
        if ((bw >> i) & 1u) {
            if (okv != 0u && static_cast<uint32_t>(i) != js) {
                bool in;
                if (SLIM) {
                    in = slim_member<CG>(a, marea, r.run, lab, static_cast<uint32_t>(w),
                                         CG ? cg_slot(P, l, bw, i) : 0u, r.v, probes, lookups, bytes);
                } else {
                    const uint32_t d = ent_deg(S, i, q);
                    in = d != 0u && in_list(a.col, S.st[i * kWave + q], d, r.v, probes, bytes);
                }
                okv = in ? okv : 0u;
            }
            if (ballot(okv != 0u) == 0ull) break;
        }
        q = below;
    }
    ok = okv != 0u;
    return ok;
}

__device__ __forceinline__ unsigned long long lane0_atomic_add(unsigned long long *p, unsigned long long x) {
    unsigned long long old = 0;
    if (lane_id() == 0) old = atomicAdd(p, x);
    return read_lane64(old, 0);
}

__device__ __forceinline__ void lane0_add(int *p, int x) {
    if (lane_id() == 0) atomicAdd(p, x);
}

__device__ __forceinline__ unsigned int load_abort(Control *ctl) {
    unsigned int v = 0;
    if (lane_id() == 0) v = __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return read_lane(v, 0);
}

__device__ __forceinline__ void set_abort(Control *ctl, unsigned int why) {
    if (lane_id() == 0) atomicCAS(&ctl->abort, kAbortNone, why);
}

template <class T>
__device__ __forceinline__ T load_agent(T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ void store_agent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Dynamic balancing (Sec. 4.3): an idle wavefront sets its bit in the idle
// bitmap and polls its own mailbox; a busy wavefront claims a set bit and
// writes the donated work into that wavefront's mailbox.  Only the donor and
// the one idle wavefront touch a mailbox, and the bitmap spreads the idle
// wavefronts over many words, so neither waiting nor claiming funnels through
// one hot word (a queue with one tail counter serialises thousands of
// wavefronts that run dry at the same moment).
//
// Every access to the bitmap and the mailboxes is an agent-scope atomic, which
// on gfx950 reads and writes at the device coherence point without cache-wide
// maintenance; an agent-scope release/acquire fence would instead write back
// and invalidate the whole L2 of the XCD, evicting the graph for every
// wavefront there.  Order is kept by waiting for all of the wavefront's memory
// operations (s_waitcnt 0) before the store that hands data over; a reader
// issues its payload loads only after it has seen that store.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wait_memory() { __builtin_amdgcn_s_waitcnt(0); }

// Claim one waiting wavefront; returns its id or -1.
__device__ int32_t claim_idle(const SearchArgs &a, uint32_t start) {
    const uint32_t lane = lane_id();
    const uint32_t nwords = (static_cast<uint32_t>(a.steal_slots) + 63u) / 64u;
    for (uint32_t base = 0; base < nwords; base += kWave) {
        const uint32_t w = (start + base + lane) % nwords;
        unsigned long long bits = 0;
        if (base + lane < nwords) bits = load_agent(&a.idle_bits[w]);
        uint64_t any = ballot(bits != 0ull);
        while (any) {
            const uint32_t src = static_cast<uint32_t>(__builtin_ctzll(any));
            any &= any - 1;
            const uint32_t word = read_lane(w, src);
            const unsigned long long seen = read_lane64(bits, src);
            int32_t id = -1;
            if (lane == 0) {
                const uint32_t b = static_cast<uint32_t>(__builtin_ctzll(seen));
                const unsigned long long mask = 1ull << b;
                const unsigned long long old = __hip_atomic_fetch_and(&a.idle_bits[word], ~mask, __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_AGENT);
                if (old & mask) id = static_cast<int32_t>(word * 64u + b);
            }
            id = static_cast<int32_t>(read_lane(static_cast<uint32_t>(id), 0));
            if (id >= 0) return id;
        }
    }
    return -1;
}

// Inclusive prefix sum over the wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (uint32_t off = 1; off < kWave; off <<= 1) {
        const uint32_t y = shfl(x, lane >= off ? lane - off : lane);
        if (lane >= off) x += y;
    }
    return x;
}

// Dynamic balancing (Sec. 4.3): when wavefronts wait for work, give one of
// them the upper half of the unscattered tasks of this wavefront's
// shallowest non-leaf level holding at least `threshold` of them ("split the
// stack in half").  The donor keeps the lower half by moving that level's end.
// The thief takes over one work unit of query cq.  Returns the bytes this lane
// wrote into the thief's mailbox (0 everywhere when nothing was handed over).
template <bool SLIM>
__device__ uint32_t donate(WaveStack &S, const SearchArgs &a, PlanPtr P, int32_t cq, int base, int l, uint32_t lane,
                           Slice cur, const Slice *parked) {
    const int k = P->k;
    const int top = l < k - 2 ? l : k - 2;
    for (int L = base; L <= top; ++L) {
        const uint32_t ci = __builtin_amdgcn_readfirstlane(S.cur_i[L]);
        if (ci >= kWave) continue;
        const uint32_t cjo = __builtin_amdgcn_readfirstlane(S.cur_j[L]);
        const uint32_t ei = __builtin_amdgcn_readfirstlane(S.end_i[L]);
        const uint32_t ej = __builtin_amdgcn_readfirstlane(S.end_j[L]);
        // the level being scattered holds its task groups in registers; the others are parked
        const Slice sl = L == l ? cur : parked[L * kWave + lane];
        uint32_t cst, cln;
        const uint32_t rem = remaining(sl, lane, ci, cjo, ei, ej, cst, cln);
        const uint32_t incl = wave_incl_scan(rem);
        const uint32_t total = read_lane(incl, 63);
        if (total < static_cast<uint32_t>(a.steal_threshold)) continue;
        Control *ctl = a.ctl;
        const int32_t thief = claim_idle(a, (blockIdx.x * 37u) & 0xffffu);
        if (thief < 0) return 0u;
        if (lane == 0) atomicAdd(&ctl->idle_count, -1);
        // split at h: the donor keeps tasks [0, h), the thief takes [h, total)
        const uint32_t h = total / 2;
        const uint32_t excl = incl - rem;
        const uint64_t hit = ballot(rem > 0 && excl <= h && h < incl);
        const uint32_t p = static_cast<uint32_t>(__builtin_ctzll(hit));
        const uint32_t excl_p = read_lane(excl, p);
        const uint32_t pj = (p == ci ? cjo : 0u) + (h - excl_p);
        Mailbox &mb = a.mail[thief];
        const bool mine = lane >= p && lane <= ei && (sl.cl & 0xffu) != 0xffu;
        const uint64_t lanes = ballot(mine);
        if (mine) {
            uint32_t q = lane;
            for (int i = L - 1; i >= 0; --i) {
                store_agent(&mb.rows[lane * kMaxK + i], ent_v<SLIM>(S, i, q));
                q = ent_pid<SLIM>(S, i, q);
            }
        }
        if (lane == 0) {
            store_agent(&mb.lanes, static_cast<unsigned long long>(lanes));
            store_agent(&mb.depth, L);
            store_agent(&mb.pi, static_cast<int32_t>(p));
            store_agent(&mb.pj, static_cast<int32_t>(pj));
            store_agent(&mb.ei, static_cast<int32_t>(ei));
            store_agent(&mb.ej, static_cast<int32_t>(ej));
            store_agent(&mb.qid, cq);
            atomicAdd(&ctl->busy, 1);  // the thief is busy from the hand-over on
            atomicAdd(&a.qctl[cq].live, 1);
            S.end_i[L] = p;
            S.end_j[L] = pj;
        }
        wait_memory();
        if (lane == 0) store_agent(&mb.status, static_cast<unsigned int>(kMailFull));
        return mine ? 4u * static_cast<uint32_t>(L) : 0u;  // this lane's rows written to the mailbox
    }
    return 0u;
}

enum Mode { kCount = 0, kEnumerate = 1, kExpand = 2 };

// Persistent search.  Every wavefront loops: take work (64 pool rows, or a
// donation once the pool is empty), load it as the bottom of its stack, and run
// Alg. 2's Search iteratively until the stack is empty.  kExpand stops at the
// pool level and appends the valid extensions to the next pool instead (one
// breadth-first step of the initialisation); donations then split the long
// lists of hub rows at that level.
// Size bound of the level after an expansion, for one new row (positions 0..d,
// position d being the row's candidate): its smallest label slice for position
// d + 1 among that position's backward neighbours.
template <bool SLIM>
__device__ __forceinline__ uint32_t next_level_bound(const WaveStack &S, const SearchArgs &a, PlanPtr P, int d,
                                                     const Round &r) {
    const uint32_t bw = P->bwd[d + 1];
    const uint32_t lab = a.loff_stride > 1 ? static_cast<uint32_t>(P->lab[d + 1]) : 0u;
    uint32_t best = 0xffffffffu;
    for (int i = 0; i <= d; ++i) {
        if (!((bw >> i) & 1u)) continue;
        const int32_t w = i == d ? r.v : ent_v<SLIM>(S, i, r.owner);
        const uint32_t *o = a.loff + static_cast<unsigned long long>(w) * a.loff_stride + lab;
        const uint32_t n = o[1] - o[0];
        best = n < best ? n : best;
    }
    return best;
}

// Expansion output is staged in LDS and written out kStageRows rows at a time:
// one atomic and coalesced stores per flush instead of per scatter round.
constexpr int kStageRows = 128;
constexpr int kStageWidth = 8;  // pool rows up to this many positions are staged

__device__ __forceinline__ void flush_stage(int32_t *stage, uint32_t &staged, int width, const SearchArgs &a) {
    if (staged == 0) return;
    const unsigned long long b0 = lane0_atomic_add(&a.ctl->out_rows, staged);
    const unsigned long long n_ok = b0 >= a.out_cap ? 0ull
                                    : (a.out_cap - b0 < staged ? a.out_cap - b0 : static_cast<unsigned long long>(staged));
    const uint32_t ints = static_cast<uint32_t>(n_ok) * static_cast<uint32_t>(width);
    __builtin_amdgcn_wave_barrier();
    for (uint32_t t = lane_id(); t < ints; t += kWave) a.out[b0 * width + t] = stage[t];
    __builtin_amdgcn_wave_barrier();
    staged = 0;
}

// LDS of one wavefront for a query of `levels` positions (stack, plus the output
// staging buffer of an expansion).
// Staging area of the LDS-staged intersection: slots list entries per lane, the
// candidates (one per lane) and their flags.
__host__ __device__ constexpr size_t merge_area_bytes(int slots) {
    return slots > 0 ? static_cast<size_t>(slots) * kWave * 4u + kWave * 4u + kWave : 0u;
}

__host__ __device__ constexpr size_t wave_lds_bytes(int levels, bool expand, bool slim, int slots) {
    return stack_bytes(levels, slim) + (expand ? static_cast<size_t>(kStageRows) * kStageWidth * 4u : 0u) +
           (slim ? (merge_area_bytes(slots) + 15u) / 16u * 16u : 0u);
}

// First phase of a two-phase pool: a root's position-1 task group keeps only
// its first hub_cut tasks (the second phase holds the rest).
__device__ __forceinline__ void first_phase_cut(Slice &sl, PlanPtr P) {
    if ((sl.cl >> 8) > P->hub_cut) sl.cl = (P->hub_cut << 8) | (sl.cl & 0xffu);
}

// Query that item t of a stream (queries p0 .. p1 - 1) belongs to: the current
// one when t is in its range, else a bisection of the plans' first items.
__device__ __forceinline__ int32_t find_query(const SearchArgs &a, PlanPtr P, int32_t cq, int32_t p0, int32_t p1,
                                              unsigned long long t) {
    if (cq >= p0 && cq < p1 && t >= P->item0 && t < P->item_end) return cq;
    int32_t lo = p0, hi = p1 - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (plan_at(a, mid)->item0 <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Indices of a wavefront's 64-bit counter totals.
enum { kTotTasks, kTotScanned, kTotLookups, kTotProbes, kTotGroups, kTotActive, kTotIssued, kTotSteals,
       kTotBytes, kTotBytesLate, kTotals };

// Work counters of the query a wavefront is on.  The per-lane and per-window
// counters are 32-bit and cover at most 32 rounds (a task group's |C^L| is below
// 2^24, so 32 of them fit); every 32 rounds, and when a work item is claimed or
// the wavefront moves to another query, they are summed over the wavefront and
// added to its 64-bit totals.  The totals and the match count are wave-uniform,
// so they sit in scalar registers and cost no vector registers per lane.
struct Tally {
    uint32_t tasks_run, scanned_run;           // per lane since the last fold
    uint32_t probes_run, lookups_run;          // per lane since the last fold
    uint32_t bytes_run;                        // per lane: device-memory bytes requested since the last fold
    uint32_t groups_run, active_run, issued_run;  // wave-uniform, since the last fold
    uint64_t count;                            // wave-uniform: matches not yet added to the query's count
    uint64_t tot[kTotals];                     // wave-uniform totals
};

// Sum over the wavefront as a wave-uniform (scalar) value.
__device__ __forceinline__ uint64_t wave_total64(uint64_t x) {
    x = wave_sum64(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t x) {
    for (int off = 32; off >= 1; off >>= 1) x += shfl(x, lane_id() ^ static_cast<uint32_t>(off));
    return __builtin_amdgcn_readfirstlane(x);
}

// Adds the window's counters to the wavefront's totals; late: this window saw
// the abort word set.
__device__ __forceinline__ void fold_run(Tally &t, bool late = false) {
    const uint64_t tasks = wave_total64(t.tasks_run), scanned = wave_total64(t.scanned_run);
    const uint32_t probes = wave_sum32(t.probes_run), lookups = wave_sum32(t.lookups_run);
    const uint32_t b = wave_sum32(t.bytes_run);
    {
        uint64_t *x = t.tot;
        x[kTotTasks] += tasks;
        x[kTotScanned] += scanned;
        x[kTotProbes] += probes;
        x[kTotLookups] += lookups;
        x[kTotGroups] += t.groups_run;
        x[kTotActive] += t.active_run;
        x[kTotIssued] += t.issued_run;
        x[late ? kTotBytesLate : kTotBytes] += b;
    }
    t.tasks_run = t.scanned_run = t.probes_run = t.lookups_run = t.bytes_run = 0;
    t.groups_run = t.active_run = t.issued_run = 0;
}

// Adds the wavefront's matches to query q's count; returns true once the count
// has reached the query's cap (the caller can drop its remaining work at once).
__device__ __forceinline__ bool count_flush(const SearchArgs &a, PlanPtr P, int32_t q, Tally &t) {
    if (!t.count) return false;
    const unsigned long long before = lane0_atomic_add(&a.qctl[q].count, t.count);
    const bool capped = P->cap && before + t.count >= P->cap;
    if (capped && lane_id() == 0) {
        atomicCAS(&a.qctl[q].abort, kAbortNone, kAbortCap);
        // a launch of one query is over: every wavefront, idle ones included, exits
        if (a.nq == 1) atomicCAS(&a.ctl->abort, kAbortNone, kAbortCap);
    }
    t.count = 0;
    return capped;
}

// Adds the wavefront's counters to query q's slots and zeroes them.  Bytes
// since the last poll count as late if the query or the launch has been
// aborted by now.
__device__ __forceinline__ void tally_flush(const SearchArgs &a, PlanPtr P, int32_t q, Tally &t) {
    (void)count_flush(a, P, q, t);
    unsigned int ab = 0;
    if (lane_id() == 0)
        ab = __hip_atomic_load(&a.qctl[q].abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) |
             __hip_atomic_load(&a.ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    fold_run(t, read_lane(ab, 0) != kAbortNone);
    if (lane_id() == 0) {
        QCtl &c = a.qctl[q];
        const uint64_t *x = t.tot;
        if (x[kTotGroups]) atomicAdd(&c.groups, x[kTotGroups]);
        if (x[kTotTasks]) atomicAdd(&c.tasks, x[kTotTasks]);
        if (x[kTotScanned]) atomicAdd(&c.scanned, x[kTotScanned]);
        if (x[kTotLookups]) atomicAdd(&c.lookups, x[kTotLookups]);
        if (x[kTotProbes]) atomicAdd(&c.probes, x[kTotProbes]);
        if (x[kTotActive]) atomicAdd(&c.lanes_active, x[kTotActive]);
        if (x[kTotIssued]) atomicAdd(&c.lanes_issued, x[kTotIssued]);
        if (x[kTotSteals]) atomicAdd(&c.steals, x[kTotSteals]);
        if (a.nq > 1) atomicMax(&c.t_last, static_cast<unsigned long long>(wall_clock64()));
        if (x[kTotBytes]) atomicAdd(&c.bytes, x[kTotBytes]);
        if (x[kTotBytesLate]) atomicAdd(&c.bytes_late, x[kTotBytesLate]);
    }
    for (int i = 0; i < kTotals; ++i) t.tot[i] = 0ull;
}

__device__ __forceinline__ unsigned int load_word(unsigned int *p) {
    unsigned int v = 0;
    if (lane_id() == 0) v = load_agent(p);
    return read_lane(v, 0);
}

// OCC is the number of wavefronts per SIMD the registers are budgeted for:
// 4 (up to 128 VGPRs, no spills) or 5 (96 VGPRs, a few spilled to scratch).
template <int MODE, bool SLIM, bool SB, bool CG, int OCC>
__global__ __launch_bounds__(kBlock, OCC) void search_kernel(SearchArgs a) {
    static_assert(!CG || (SLIM && MODE != kExpand), "the candidate graph runs the slim depth-first search");
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const int levels = a.levels;
    uint8_t *mine = lds + (threadIdx.x / kWave) * wave_lds_bytes(levels, MODE == kExpand, SLIM, a.merge_slots);
    WaveStack S = carve_stack<SLIM>(mine, levels);
    int32_t *stage = reinterpret_cast<int32_t *>(mine + stack_bytes(levels, SLIM));
    uint8_t *marea = mine + stack_bytes(levels, SLIM) +
                     (MODE == kExpand ? static_cast<size_t>(kStageRows) * kStageWidth * 4u : 0u);
    uint32_t staged = 0;
    const uint32_t lane = lane_id();
    Control *ctl = a.ctl;
    const bool stealing = a.mail != nullptr;
    const uint32_t wave_id = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    // this wavefront's parked task groups, one level per 64 entries
    Slice *parked = reinterpret_cast<Slice *>(a.parked) + static_cast<size_t>(wave_id) * levels * kWave;
    Slice cur{0u, 0xffu};  // task group of this lane at the level being scattered

    int32_t cq = 0;  // query of the wavefront's current work (wave-uniform)
    PlanPtr P = plan_at(a, 0);
    int32_t sid = static_cast<int32_t>(wave_id % static_cast<uint32_t>(a.nstreams));  // home stream first
    int32_t dry = 0;  // streams found exhausted
    unsigned long long qstart = 0;  // start of that query's time budget
    Tally t{};
    uint64_t my_bound = 0;
    uint32_t rounds = 0;
    bool stop = false;
    bool items_left = true;
    const unsigned long long deadline = a.budget ? a.ctl->t0 + a.budget : 0ull;
    if (stealing) lane0_add(&ctl->busy, 1);

    while (!stop) {
        int base = 0;
        bool have = false;
        // a work item: 64 pool rows of one query, skipped once that query reached its cap
        while (items_left) {
            StreamCtl &sc = a.streams[sid];
            const unsigned long long it = lane0_atomic_add(&sc.next, 1ull);
            // the stream's fields are fixed during the launch: read them as wave-uniform
            if (it >= read_lane64(sc.items, 0)) {  // this stream ran dry: help the next one
                if (++dry >= a.nstreams) items_left = false;
                sid = sid + 1 == a.nstreams ? 0 : sid + 1;
                continue;
            }
            const int32_t q = find_query(a, P, cq, __builtin_amdgcn_readfirstlane(sc.plan0),
                                         __builtin_amdgcn_readfirstlane(sc.plan1), it);
            if (q != cq) {
                tally_flush(a, P, cq, t);
                cq = q;
                P = plan_at(a, q);
            }
            if (load_word(&a.qctl[cq].abort) != kAbortNone) {
                // capped or out of time: nobody needs the query's other items
                if (lane == 0) atomicMax(&sc.next, static_cast<unsigned long long>(P->item_end));
                continue;
            }
            if (P->budget || a.nq > 1) {  // the query's clock starts with its first claimed item
                unsigned long long old = 0;
                if (lane == 0) {
                    const unsigned long long now = wall_clock64();
                    old = atomicCAS(&a.qctl[cq].t_start, 0ull, now);
                    if (old == 0ull) old = now;
                }
                qstart = read_lane64(old, 0);
            }
            if (P->vmode && it >= P->item_split) {
                // second phase of the pool: 64 consecutive tasks of position 1.  Each lane
                // finds its task's root (the last root whose first task index is <= the
                // task), puts the root at level 0 and processes the candidate as a scatter
                // round at level 1 would.
                const unsigned long long tb = (it - P->item_split) * kWave;
                const unsigned long long left = P->tasks1 - tb;
                const uint32_t ntask = left < kWave ? static_cast<uint32_t>(left) : kWave;
                const int32_t *roots = a.pool + P->row0;
                const uint32_t *off = a.voff + P->vrow0;
                int32_t root = 0, v = -1;
                VInfo rvi = make_uint2(0u, 0u);
                if (lane < ntask) {
                    const uint32_t task = static_cast<uint32_t>(tb) + lane;
                    uint32_t lo = 0, hi = static_cast<uint32_t>(P->rows) - 1u;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi + 1u) >> 1;
                        if (off[mid] <= task) lo = mid;
                        else hi = mid - 1u;
                        t.bytes_run += 4u;
                    }
                    root = roots[permuted(lo, P->perm_mul, P->rows)];
                    if (!SLIM) rvi = a.vinfo[root];
                    v = a.lcol[a.vstart[P->vrow0 + lo] + (task - off[lo])];
                    t.bytes_run += SLIM ? 16u : 24u;  // root, its first task, slice start, candidate (+ record)
                }
                push_entry<SLIM>(S, 0, lane, root, rvi, lane);
                Round r1;
                r1.ntask = ntask;
                r1.owner = lane;
                r1.v = v;
                r1.run = lane | ((lane + 1u) << 8);  // every lane is its own root
                r1.js = 0u;                          // the candidate came from position 0's list
                VInfo vi;
                const bool ok = process<SLIM, SB, CG>(S, a, P, 1, r1, lane, vi, t.probes_run, t.lookups_run,
                                                      t.bytes_run, marea);
                const uint64_t m = ballot(ok);
                t.active_run += ntask;
                t.issued_run += kWave;
                if (P->k == 2) {
                    if (MODE == kEnumerate && m) {
                        const unsigned long long b0 = lane0_atomic_add(&ctl->out_rows, __popcll(m));
                        const unsigned long long slot = b0 + popc_below(m);
                        if (ok && slot < a.out_cap) {
                            int32_t *row = a.out + slot * 2ull;
                            row[P->phi[0]] = root;
                            row[P->phi[1]] = v;
                            t.bytes_run += 8u;
                        }
                    }
                    t.count += __popcll(m);
                    (void)count_flush(a, P, cq, t);
                    continue;
                }
                if (!m) continue;
                lane0_add(&a.qctl[cq].live, 1);
                push_entry<SLIM>(S, 1, lane, v, vi, lane);
                const Gen g = generate_tasks<SLIM, CG>(S, a, P, 2, m, lane);
                cur = g.sl;
                t.tasks_run += g.tasks;
                t.scanned_run += g.scanned;
                t.lookups_run += g.lookups;
                t.bytes_run += g.bytes;
                t.groups_run += __popcll(m);
                fold_run(t);  // a claimed item's group can be as large as 2^24: fold at once
                open_level(S, 2, lane);
                base = 2;
                have = true;
                break;
            }
            const int d = P->depth;
            const uint32_t rpi = P->rpi ? P->rpi : static_cast<uint32_t>(kWave);
            const unsigned long long r0 = (it - P->item0) * rpi;
            const unsigned long long left = P->rows - r0;
            const uint32_t nrows = left < rpi ? static_cast<uint32_t>(left) : rpi;
            const bool mine = lane < nrows;
            const int32_t *src = a.pool + P->row0 + permuted(r0 + lane, P->perm_mul, P->rows) *
                                                        static_cast<unsigned long long>(d);
            for (int i = 0; i < d; ++i) {
                int32_t v = 0;
                VInfo vi = make_uint2(0u, 0u);
                if (mine) {
                    v = src[i];
                    vi = a.vinfo[v];
                }
                push_entry<SLIM>(S, i, lane, v, vi, lane);
            }
            t.bytes_run += mine ? 12u * static_cast<uint32_t>(d) : 0u;  // id and record per position
            const uint64_t F0 = ballot(mine);
            if (d >= P->k) {  // the rows are whole matches (a one-vertex query)
                t.count += __popcll(F0);
                (void)count_flush(a, P, cq, t);
                continue;
            }
            lane0_add(&a.qctl[cq].live, 1);
            Gen g = generate_tasks<SLIM, CG>(S, a, P, d, F0, lane);
            cur = g.sl;
            t.bytes_run += g.bytes;
            if (P->vmode) {  // first phase: each root's first hub_cut tasks only
                first_phase_cut(cur, P);
                g.scanned = g.scanned < P->hub_cut ? g.scanned : P->hub_cut;
            }
            t.tasks_run += g.tasks;
            t.scanned_run += g.scanned;
            t.lookups_run += g.lookups;
            t.groups_run += __popcll(F0);
            fold_run(t);  // a claimed item's group can be as large as 2^24: fold at once
            open_level(S, d, lane);
            base = d;
            have = true;
            break;
        }
        if (!have) {
            if (!stealing) break;
            // idle: wait for a donation until nobody holds work or the search aborts
            Mailbox &mb = a.mail[wave_id];
            if (lane == 0) store_agent(&mb.status, static_cast<unsigned int>(kMailWaiting));
            wait_memory();
            if (lane == 0) {
                atomicAdd(&ctl->busy, -1);
                atomicAdd(&ctl->idle_count, 1);
                __hip_atomic_fetch_or(&a.idle_bits[wave_id / 64u], 1ull << (wave_id % 64u), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
            }
            bool got = false;
            uint32_t nap = 1;  // exponential back-off on the wavefront's own mailbox
            for (uint32_t iter = 0;; ++iter) {
                for (uint32_t z = 0; z < nap; ++z) __builtin_amdgcn_s_sleep(16);
                nap = nap < 32u ? nap * 2u : 32u;
                if (load_word(&mb.status) == kMailFull) {
                    got = true;
                    break;
                }
                if ((iter & 7u) == 7u) {
                    if (deadline && wall_clock64() > deadline) set_abort(ctl, kAbortTime);
                    unsigned int ab = 0;
                    int busy = 0;
                    if (lane == 0) {
                        ab = load_agent(&ctl->abort);
                        busy = load_agent(&ctl->busy);
                    }
                    if (read_lane(ab, 0) != kAbortNone) break;
                    if (read_lane(static_cast<uint32_t>(busy), 0) == 0) break;
                }
            }
            if (!got) break;
            // the donated work: parent rows at level L-1 and a task range at level L of query qid
            int32_t q = 0;
            if (lane == 0) q = load_agent(&mb.qid);
            q = static_cast<int32_t>(read_lane(static_cast<uint32_t>(q), 0));
            if (q != cq) {
                tally_flush(a, P, cq, t);
                cq = q;
                P = plan_at(a, q);
            }
            if (P->budget) {
                unsigned long long ts = 0;
                if (lane == 0) ts = load_agent(&a.qctl[cq].t_start);
                qstart = read_lane64(ts, 0);
            }
            const int L = __builtin_amdgcn_readfirstlane(load_agent(&mb.depth));
            const uint64_t lanes = load_agent(&mb.lanes);
            const bool mine = (lanes >> lane) & 1ull;
            for (int i = 0; i < L; ++i) {
                int32_t v = 0;
                VInfo vi = make_uint2(0u, 0u);
                if (mine) {
                    v = load_agent(&mb.rows[lane * kMaxK + i]);
                    vi = a.vinfo[v];
                }
                push_entry<SLIM>(S, i, lane, v, vi, lane);
            }
            t.bytes_run += mine ? 12u * static_cast<uint32_t>(L) : 0u;
            // the tasks and groups were counted by the donor; the reads are this wavefront's
            const Gen gd = generate_tasks<SLIM, CG>(S, a, P, L, lanes, lane);
            cur = gd.sl;
            t.bytes_run += gd.bytes;
            // position 1 is donated only by first-phase items of a two-phase pool: keep their cut
            if (P->vmode && L == 1) first_phase_cut(cur, P);
            if (lane == 0) {
                S.cur_i[L] = static_cast<uint32_t>(load_agent(&mb.pi));
                S.cur_j[L] = static_cast<uint32_t>(load_agent(&mb.pj));
                S.end_i[L] = static_cast<uint32_t>(load_agent(&mb.ei));
                S.end_j[L] = static_cast<uint32_t>(load_agent(&mb.ej));
            }
            wait_memory();
            if (lane == 0) store_agent(&mb.status, static_cast<unsigned int>(kMailEmpty));
            base = L;
            t.tot[kTotSteals] += 1ull;
        }
        // the unit's query, made provably wave-uniform so that every plan field
        // in the loop below is a scalar load
        cq = __builtin_amdgcn_readfirstlane(cq);
        P = plan_at(a, cq);
        const int k = P->k;
        const int d = P->depth;
        bool dropped = false;  // the query reached its cap or time limit: drop the rest of this unit
        int l = base;
        while (l >= base) {
            const Round r = scatter(S, a.lcol, l, lane, cur);
            if (r.ntask == 0) {
                if (--l >= base) {  // back to the parked task groups of the level below
                    cur = parked[l * kWave + lane];
                    t.bytes_run += 8u;
                }
                continue;
            }
            t.active_run += r.ntask;
            t.issued_run += kWave;
            t.bytes_run += lane < r.ntask ? 4u : 0u;  // the candidate's id
            VInfo vi;
            const bool ok = process<SLIM, SB, CG>(S, a, P, l, r, lane, vi, t.probes_run, t.lookups_run, t.bytes_run,
                                                  marea);
            const uint64_t m = ballot(ok);
            if (MODE == kExpand) {
                if (m) {
                    const uint32_t nv = static_cast<uint32_t>(__popcll(m));
                    if (d + 1 <= kStageWidth) {
                        if (staged + nv > static_cast<uint32_t>(kStageRows)) flush_stage(stage, staged, d + 1, a);
                        if (ok) {
                            int32_t *row = stage + (staged + popc_below(m)) * static_cast<uint32_t>(d + 1);
                            for (int i = 0; i < d; ++i) row[i] = ent_v<SLIM>(S, i, r.owner);
                            row[d] = r.v;
                            if (a.measure_next) my_bound += next_level_bound<SLIM>(S, a, P, d, r);
                            t.bytes_run += 4u * static_cast<uint32_t>(d + 1);  // the row, written at the flush
                        }
                        staged += nv;
                    } else {
                        const unsigned long long b0 = lane0_atomic_add(&ctl->out_rows, nv);
                        const unsigned long long slot = b0 + popc_below(m);
                        if (ok && slot < a.out_cap) {
                            int32_t *row = a.out + slot * static_cast<unsigned long long>(d + 1);
                            for (int i = 0; i < d; ++i) row[i] = ent_v<SLIM>(S, i, r.owner);
                            row[d] = r.v;
                            t.bytes_run += 4u * static_cast<uint32_t>(d + 1);
                        }
                        if (ok && a.measure_next) my_bound += next_level_bound<SLIM>(S, a, P, d, r);
                    }
                }
            } else if (l == k - 1) {
                if (MODE == kEnumerate && m) {
                    const unsigned long long b0 = lane0_atomic_add(&ctl->out_rows, __popcll(m));
                    const unsigned long long slot = b0 + popc_below(m);
                    if (ok && slot < a.out_cap) {
                        int32_t *row = a.out + slot * static_cast<unsigned long long>(k);
                        row[P->phi[l]] = r.v;
                        uint32_t q = r.owner;
                        for (int i = l - 1; i >= 0; --i) {
                            row[P->phi[i]] = ent_v<SLIM>(S, i, q);
                            q = ent_pid<SLIM>(S, i, q);
                        }
                        t.bytes_run += 4u * static_cast<uint32_t>(k);
                    }
                }
                t.count += __popcll(m);
            } else if (m) {
                push_entry<SLIM>(S, l, lane, r.v, vi, r.owner);
                parked[l * kWave + lane] = cur;  // this level's task groups wait for the backtrack
                const Gen g = generate_tasks<SLIM, CG>(S, a, P, l + 1, m, lane);
                cur = g.sl;
                t.bytes_run += 8u;
                t.tasks_run += g.tasks;
                t.scanned_run += g.scanned;
                t.lookups_run += g.lookups;
                t.bytes_run += g.bytes;
                t.groups_run += __popcll(m);
                open_level(S, l + 1, lane);
                ++l;
            }
            ++rounds;
            if (t.count >= P->flush || (rounds & 31u) == 0) {
                (void)count_flush(a, P, cq, t);
                if ((rounds & 31u) == 0) {
                    if (deadline | P->budget) {
                        const unsigned long long now = wall_clock64();
                        if (deadline && now > deadline) set_abort(ctl, kAbortTime);
                        if (P->budget && now > qstart + P->budget && lane == 0) {
                            atomicCAS(&a.qctl[cq].abort, kAbortNone, kAbortTime);
                            if (a.nq == 1) atomicCAS(&ctl->abort, kAbortNone, kAbortTime);
                        }
                    }
                    if (load_abort(ctl) != kAbortNone) stop = true;
                    else if (a.nq > 1 && !dropped && load_word(&a.qctl[cq].abort) != kAbortNone) dropped = true;
                    if (stealing && !stop && !dropped) {
                        int waiting = 0;
                        if (lane == 0) waiting = load_agent(&ctl->idle_count);
                        if (static_cast<int>(read_lane(static_cast<uint32_t>(waiting), 0)) > 0)
                            t.bytes_run += donate<SLIM>(S, a, P, cq, base, l, lane, cur, parked);
                    }
                    fold_run(t, stop || dropped);
                }
                if (stop || dropped) break;
            }
        }
        // a unit that ran to its end is finished; one cut short by the time limit is not
        if (!stop) lane0_add(&a.qctl[cq].live, -1);
    }
    if (MODE == kExpand) {
        flush_stage(stage, staged, P->depth + 1, a);
        if (a.measure_next) {
            const uint64_t b = wave_sum64(my_bound);
            if (lane == 0 && b) atomicAdd(&ctl->measure, static_cast<unsigned long long>(b));
        }
    }
    tally_flush(a, P, cq, t);
}

// Second phase of a two-phase pool, first pass: each root's position-1 slice
// beyond its first hub_cut tasks (position 0 is position 1's only backward
// neighbour, so C^L is the root's list, and its slice with position 1's label is
// scanned).  The roots' groups and tasks are counted by the first phase.
__global__ __launch_bounds__(256) void level1_kernel(const int32_t *__restrict__ roots, int32_t R,
                                                     unsigned long long perm_mul, uint32_t hub_cut,
                                                     const uint32_t *__restrict__ loff, int32_t stride, int32_t lab1,
                                                     uint32_t *__restrict__ lens, uint32_t *__restrict__ vstart,
                                                     QCtl *qc) {
    uint64_t scanned = 0;
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < R;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int32_t v = roots[permuted(static_cast<unsigned long long>(i), perm_mul, static_cast<unsigned long long>(R))];
        const uint32_t *o = loff + static_cast<unsigned long long>(v) * stride + (stride > 1 ? lab1 : 0);
        const uint32_t st = o[0], len = o[1] - o[0];
        const uint32_t rest = len > hub_cut ? len - hub_cut : 0u;
        lens[i] = rest;
        vstart[i] = st + (len > hub_cut ? hub_cut : len);
        scanned += rest;
    }
    scanned = wave_sum64(scanned);
    if (lane_id() == 0 && scanned) atomicAdd(&qc->scanned, static_cast<unsigned long long>(scanned));
}

// Exclusive prefix sum of up to 2^31 uint32 values in three passes: per-block
// scans of kScanChunk values, a scan of the block totals, and the block offsets
// added back.  (Totals stay below 2^32: they are sums of degrees of one graph.)
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanChunk = kScanThreads * kScanPer;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *sh, uint32_t &total) {
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    const uint32_t incl = wave_incl_scan(x);
    if (lane == kWave - 1) sh[w] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (uint32_t j = 0; j < blockDim.x / kWave; ++j) {
        base += j < w ? sh[j] : 0u;
        tot += sh[j];
    }
    __syncthreads();
    total = tot;
    return base + incl - x;
}

__global__ __launch_bounds__(kScanThreads) void scan_chunks_kernel(const uint32_t *__restrict__ in, int32_t n,
                                                                   uint32_t *__restrict__ out,
                                                                   uint32_t *__restrict__ sums) {
    __shared__ uint32_t sh[kScanThreads / kWave];
    const long long b0 = static_cast<long long>(blockIdx.x) * kScanChunk + threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t local = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = b0 + j < n ? in[b0 + j] : 0u;
        local += v[j];
    }
    uint32_t total = 0;
    uint32_t run = block_excl_scan(local, sh, total);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        if (b0 + j < n) out[b0 + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block: exclusive scan of the nb chunk totals in place; the grand total
// sizes the query's virtual pool (tasks1, its work items, the stream's items).
__global__ __launch_bounds__(1024) void scan_sums_kernel(uint32_t *sums, int32_t nb, Plan *plan, StreamCtl *sc) {
    __shared__ uint32_t sh[1024 / kWave];
    const int32_t per = (nb + blockDim.x - 1) / blockDim.x;
    const int32_t b = threadIdx.x * per;
    uint32_t local = 0;
    for (int32_t j = 0; j < per; ++j)
        if (b + j < nb) local += sums[b + j];
    uint32_t total = 0;
    uint32_t run = block_excl_scan(local, sh, total);
    for (int32_t j = 0; j < per; ++j) {
        if (b + j < nb) {
            const uint32_t x = sums[b + j];
            sums[b + j] = run;
            run += x;
        }
    }
    if (threadIdx.x == 0) {
        const unsigned long long items = (static_cast<unsigned long long>(total) + kWave - 1) / kWave;
        plan->tasks1 = total;
        plan->item_end = plan->item_split + items;
        sc->items = plan->item_end;
    }
}

__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(uint32_t *__restrict__ out, int32_t n,
                                                                const uint32_t *__restrict__ sums) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * blockDim.x)
        out[i] += sums[i / kScanChunk];
}

__global__ void start_clock_kernel(Control *ctl) {
    if (threadIdx.x == 0) ctl->t0 = wall_clock64();
}

__global__ void steal_init_kernel(Mailbox *mail, unsigned long long *idle_bits, int32_t n) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mail[i].status = kMailEmpty;
    if (i < (n + 63) / 64) idle_bits[i] = 0ull;
}

// Candidates of the first query vertex: label and degree filter over all of V(G).
// With measure_lab >= 0 it also adds up each candidate's label slice for the
// second position (its only backward neighbour is the first), the size bound of
// the next pool level.
__global__ __launch_bounds__(256) void root_scan_kernel(const VInfo *__restrict__ vinfo, int32_t n, int32_t lab0,
                                                        int32_t qdeg0, int32_t *__restrict__ pool,
                                                        const uint32_t *__restrict__ loff, int32_t loff_stride,
                                                        int32_t measure_lab, Control *ctl) {
    const uint32_t lane = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->t0 = wall_clock64();
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    uint64_t bound = 0;
    for (long long base = static_cast<long long>(blockIdx.x) * blockDim.x + (threadIdx.x & ~(kWave - 1)); base < n;
         base += stride) {
        const long long v = base + lane;
        bool ok = false;
        if (v < n) {
            const VInfo vi = vinfo[v];
            ok = vi_lab(vi) == static_cast<uint32_t>(lab0) && vi_deg(vi) >= static_cast<uint32_t>(qdeg0);
        }
        const uint64_t m = ballot(ok);
        if (m) {
            const unsigned long long b = lane0_atomic_add(&ctl->out_rows, __popcll(m));
            if (ok) {
                pool[b + popc_below(m)] = static_cast<int32_t>(v);
                if (measure_lab >= 0) {
                    const uint32_t *o = loff + static_cast<unsigned long long>(v) * loff_stride + measure_lab;
                    bound += o[1] - o[0];
                }
            }
        }
    }
    if (measure_lab >= 0) {
        bound = wave_sum64(bound);
        if (lane == 0 && bound) atomicAdd(&ctl->measure, static_cast<unsigned long long>(bound));
    }
}

template <int MODE, bool SLIM, bool SB, bool CG, int OCC>
int blocks_per_cu(int levels, int waves_per_cu, int slots) {
    const size_t lds_bytes = wave_lds_bytes(levels, MODE == kExpand, SLIM, slots) * kWavesPerBlock;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, search_kernel<MODE, SLIM, SB, CG, OCC>, kBlock,
                                                     lds_bytes) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (waves_per_cu > 0) {
        const int want = (waves_per_cu + kWavesPerBlock - 1) / kWavesPerBlock;
        if (want < per_cu) per_cu = want;
    }
    return per_cu;
}

template <int MODE, bool SLIM, bool SB, bool CG, int OCC>
hipError_t launch_persistent(const SearchArgs &a, int num_cu, int waves_per_cu, hipStream_t s, int *grid_waves) {
    if (a.levels < 1 || a.levels > kMaxK || a.nq < 1 || !a.plans || !a.qctl || a.nstreams < 1 || !a.streams)
        return hipErrorInvalidValue;
    if (CG && (!a.gbounds || a.gn < 1)) return hipErrorInvalidValue;
    if (a.merge_slots < 0 || a.merge_slots > kMaxMergeSlots) return hipErrorInvalidValue;
    if (!a.parked || a.park_waves < 1) return hipErrorInvalidValue;
    SearchArgs b = a;
    if (!SLIM) b.merge_slots = 0;  // the full layout bisects whole lists
    const size_t lds_bytes = wave_lds_bytes(b.levels, MODE == kExpand, SLIM, b.merge_slots) * kWavesPerBlock;
    int blocks = num_cu * blocks_per_cu<MODE, SLIM, SB, CG, OCC>(b.levels, waves_per_cu, b.merge_slots);
    if (a.mail && blocks * kWavesPerBlock > a.steal_slots) blocks = a.steal_slots / kWavesPerBlock;  // one mailbox each
    if (blocks * kWavesPerBlock > a.park_waves) blocks = a.park_waves / kWavesPerBlock;  // one parking area each
    if (blocks < 1) blocks = 1;
    if (grid_waves) *grid_waves = blocks * kWavesPerBlock;
    hipLaunchKernelGGL((search_kernel<MODE, SLIM, SB, CG, OCC>), dim3(blocks), dim3(kBlock), lds_bytes, s, b);
    return hipGetLastError();
}

// The slim plain-graph kernels also exist with the register budget of five
// wavefronts per SIMD.  Their spills cost more than one extra wavefront per CU
// brings, so they run only where the occupancy calculator says they fit at
// least an eighth more wavefronts than the four-wavefront build (LDS, not
// registers, bounds residency for the deepest queries).
template <int MODE, bool SB>
bool five_waves_fit(int levels, int waves_per_cu, int slots) {
    return blocks_per_cu<MODE, true, SB, false, 5>(levels, waves_per_cu, slots) * 8 >
           blocks_per_cu<MODE, true, SB, false, 4>(levels, waves_per_cu, slots) * 9;
}

// One of the instantiations: mode x stack layout x symmetry conditions x
// candidate graph (slim layout, count and enumerate only) x register budget.
template <int MODE>
hipError_t launch_mode(const SearchArgs &a, int num_cu, int waves_per_cu, hipStream_t s, int *grid_waves) {
    if constexpr (MODE != kExpand) {
        if (a.cg) {
            if (a.sb) return launch_persistent<MODE, true, true, true, 4>(a, num_cu, waves_per_cu, s, grid_waves);
            return launch_persistent<MODE, true, false, true, 4>(a, num_cu, waves_per_cu, s, grid_waves);
        }
        if (a.slim) {
            if (a.sb) {
                if (five_waves_fit<MODE, true>(a.levels, waves_per_cu, a.merge_slots))
                    return launch_persistent<MODE, true, true, false, 5>(a, num_cu, waves_per_cu, s, grid_waves);
                return launch_persistent<MODE, true, true, false, 4>(a, num_cu, waves_per_cu, s, grid_waves);
            }
            if (five_waves_fit<MODE, false>(a.levels, waves_per_cu, a.merge_slots))
                return launch_persistent<MODE, true, false, false, 5>(a, num_cu, waves_per_cu, s, grid_waves);
            return launch_persistent<MODE, true, false, false, 4>(a, num_cu, waves_per_cu, s, grid_waves);
        }
    } else {
        if (a.cg) return hipErrorInvalidValue;
        if (a.slim) {
            if (a.sb) return launch_persistent<MODE, true, true, false, 4>(a, num_cu, waves_per_cu, s, grid_waves);
            return launch_persistent<MODE, true, false, false, 4>(a, num_cu, waves_per_cu, s, grid_waves);
        }
    }
    if (a.sb) return launch_persistent<MODE, false, true, false, 4>(a, num_cu, waves_per_cu, s, grid_waves);
    return launch_persistent<MODE, false, false, false, 4>(a, num_cu, waves_per_cu, s, grid_waves);
}

}  // namespace

hipError_t launch_root_scan(const VInfo *vinfo, int32_t n, int32_t lab0, int32_t qdeg0, int32_t *pool,
                            const uint32_t *loff, int32_t loff_stride, int32_t measure_lab, Control *ctl, int num_cu,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long blocks = (static_cast<long long>(n) + 255) / 256;
    if (blocks > num_cu * 8LL) blocks = num_cu * 8LL;
    hipLaunchKernelGGL(root_scan_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, vinfo, n, lab0,
                       qdeg0, pool, loff, loff_stride, measure_lab, ctl);
    return hipGetLastError();
}

hipError_t launch_expand(const SearchArgs &a, int num_cu, hipStream_t s) {
    return launch_mode<kExpand>(a, num_cu, 0, s, nullptr);
}

// Wavefronts per CU a slim plain-graph count launch keeps resident with
// `slots` staging entries per lane, in the build the launch would take.
int slim_residency(int levels, int waves_per_cu, int slots) {
    if (five_waves_fit<kCount, false>(levels, waves_per_cu, slots))
        return blocks_per_cu<kCount, true, false, false, 5>(levels, waves_per_cu, slots);
    return blocks_per_cu<kCount, true, false, false, 4>(levels, waves_per_cu, slots);
}

// The default staging: the staging area is kept unless it lowers the
// wavefronts a CU keeps resident, which happens only for the deepest queries,
// where LDS and not registers bounds residency.  Latency hiding is worth more
// there than staging, which the search then does without.
int auto_merge_slots(int levels, int waves_per_cu, int slots) {
    if (slots <= 0) return 0;
    return slim_residency(levels, waves_per_cu, slots) < slim_residency(levels, waves_per_cu, 0) ? 0 : slots;
}

int search_waves(int levels, int num_cu, int waves_per_cu, bool slim, int merge_slots, bool merge_auto) {
    if (slim && merge_auto) merge_slots = auto_merge_slots(levels, waves_per_cu, merge_slots);
    int per_cu = slim ? blocks_per_cu<kCount, true, false, false, 4>(levels, waves_per_cu, merge_slots)
                      : blocks_per_cu<kCount, false, false, false, 4>(levels, waves_per_cu, 0);
    if (slim && five_waves_fit<kCount, false>(levels, waves_per_cu, merge_slots))
        per_cu = blocks_per_cu<kCount, true, false, false, 5>(levels, waves_per_cu, merge_slots);
    return num_cu * per_cu * kWavesPerBlock;
}

hipError_t launch_search(const SearchArgs &a, bool enumerate, int num_cu, int waves_per_cu, hipStream_t s,
                         int *grid_waves_out) {
    SearchArgs b = a;
    if (b.slim && b.merge_auto) b.merge_slots = auto_merge_slots(b.levels, waves_per_cu, b.merge_slots);
    if (enumerate) return launch_mode<kEnumerate>(b, num_cu, waves_per_cu, s, grid_waves_out);
    return launch_mode<kCount>(b, num_cu, waves_per_cu, s, grid_waves_out);
}

hipError_t launch_level1(const int32_t *roots, int32_t R, unsigned long long perm_mul, uint32_t hub_cut,
                         const uint32_t *loff, int32_t stride, int32_t lab1, uint32_t *lens, uint32_t *vstart,
                         uint32_t *voff, uint32_t *tmp, QCtl *qc, Plan *plan, StreamCtl *sc, int num_cu,
                         hipStream_t s) {
    if (R < 1) return hipErrorInvalidValue;
    long long blocks = (static_cast<long long>(R) + 255) / 256;
    if (blocks > num_cu * 8LL) blocks = num_cu * 8LL;
    hipLaunchKernelGGL(level1_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, roots, R, perm_mul,
                       hub_cut, loff, stride, lab1, lens, vstart, qc);
    const int32_t nb = static_cast<int32_t>((static_cast<long long>(R) + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(scan_chunks_kernel, dim3(nb), dim3(kScanThreads), 0, s, lens, R, voff, tmp);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, tmp, nb, plan, sc);
    long long ablocks = (static_cast<long long>(R) + 255) / 256;
    if (ablocks > num_cu * 8LL) ablocks = num_cu * 8LL;
    hipLaunchKernelGGL(scan_add_kernel, dim3(static_cast<unsigned>(ablocks)), dim3(kScanThreads), 0, s, voff, R, tmp);
    return hipGetLastError();
}

hipError_t launch_start_clock(Control *ctl, hipStream_t s) {
    hipLaunchKernelGGL(start_clock_kernel, dim3(1), dim3(kWave), 0, s, ctl);
    return hipGetLastError();
}

hipError_t launch_steal_init(Mailbox *mail, unsigned long long *idle_bits, int32_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(steal_init_kernel, dim3((n + 255) / 256), dim3(256), 0, s, mail, idle_bits, n);
    return hipGetLastError();
}

}  // namespace gm
