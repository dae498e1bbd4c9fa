// gfx950 kernels that build the candidate graph G' of one query.
//
// When the paper compares with EGSM it runs its search on EGSM's candidate
// graph (experimental setup, Sec. 6.1); App. C describes G' as the output of a
// light filter over labels and query structure, the search then reading G'
// instead of G.  The filter here keeps, for every position l of the matching
// order, the largest set C(l) of vertices with l's label and at least l's
// query degree in which every vertex has, for every query neighbour l2 of l,
// a neighbour in C(l2).  G' holds, for each query edge (i, l) with i before l,
// the list N(v) restricted to C(l) for every v in C(i); the search takes its
// candidates and its membership tests from those lists.
//
// Layout (HBM):
//   bits:    one bitmap per position, row l at bits[l * wp], wp = 2 * ceil(n / 64)
//            words (a wavefront writes the two words of its 64 vertices);
//   clist:   the candidates of every position, ids ascending, one list after
//            the other (bounds[l] .. bounds[l + 1]); those of position 0 are the
//            search's roots;
//   gcol:    the lists, ids ascending (taken in order from G's label slices),
//            laid out by an exclusive prefix sum over (edge, candidate);
//   gbounds: per query edge e and candidate v of its earlier end, the start and
//            end of v's list at gbounds[2 * (e * n + v)] (entries of other
//            vertices are never written nor read: the search only looks up
//            vertices of C(i) for edge (i, l)).
//
// Every kernel streams vertices or candidates with coalesced loads; the sweeps
// and counts are bound by HBM and by random reads of the bitmaps (|Q| * n / 8
// bytes, which stay in L2 and the Infinity Cache for graphs up to tens of
// millions of vertices).
#include <hip/hip_runtime.h>

#include "gm_internal.h"

namespace gm {

namespace {

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ bool has_bit(const uint32_t *__restrict__ row, uint32_t v) {
    return (row[v >> 5] >> (v & 31u)) & 1u;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
    for (int off = 32; off >= 1; off >>= 1) {
        const int src = static_cast<int>((lane_id() ^ static_cast<uint32_t>(off)) << 2);
        const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(src, static_cast<int>(x)));
        const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(src, static_cast<int>(x >> 32)));
        x += (static_cast<uint64_t>(hi) << 32) | lo;
    }
    return x;
}

// Bounds of the slice of N(v) that can hold label c (the whole list when
// lists are not partitioned by label).
__device__ __forceinline__ uint2 slice(const uint32_t *__restrict__ loff, int32_t stride, uint32_t v, int32_t c) {
    const uint32_t *o = loff + static_cast<unsigned long long>(v) * stride + (stride > 1 ? c : 0);
    return make_uint2(o[0], o[1]);
}

// C0: bit v of row l set iff L(v) = lab[l] and d(v) >= qdeg[l].  A wavefront
// covers 64 consecutive vertices and writes their two words of every row.
__global__ __launch_bounds__(256) void cand_init_kernel(const VInfo *__restrict__ vinfo, int32_t n, CandQuery q,
                                                        uint32_t *__restrict__ bits, unsigned long long wp) {
    const uint32_t lane = lane_id();
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long base = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x - lane; base < n;
         base += step) {
        const long long v = base + lane;
        const VInfo vi = v < n ? vinfo[v] : make_uint2(0u, 0u);
        const uint32_t lab = vi_lab(vi), deg = vi_deg(vi);
        for (int l = 0; l < q.k; ++l) {
            const bool in = v < n && lab == static_cast<uint32_t>(q.lab[l]) && deg >= static_cast<uint32_t>(q.qdeg[l]);
            const unsigned long long m = __ballot(in);
            uint32_t *row = bits + static_cast<unsigned long long>(l) * wp + static_cast<unsigned long long>(base >> 5);
            if (lane == 0) row[0] = static_cast<uint32_t>(m);
            if (lane == 32) row[1] = static_cast<uint32_t>(m >> 32);
        }
    }
}

// One sweep of the support filter: v leaves C(l) when some query neighbour l2
// of l finds none of v's neighbours in C(l2).  Bits only go from 1 to 0, so a
// stale read during the sweep can only keep a vertex one more sweep; a sweep
// that clears nothing read the final sets everywhere, which is the fixed point.
__global__ __launch_bounds__(256) void cand_refine_kernel(const int32_t *__restrict__ lcol,
                                                          const uint32_t *__restrict__ loff, int32_t stride, int32_t n,
                                                          CandQuery q, uint32_t *bits, unsigned long long wp,
                                                          uint32_t *changed) {
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long vi = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; vi < n; vi += step) {
        const uint32_t v = static_cast<uint32_t>(vi);
        uint32_t mine = 0;
        for (int l = 0; l < q.k; ++l)
            if (has_bit(bits + static_cast<unsigned long long>(l) * wp, v)) mine |= 1u << l;
        uint32_t drop = 0;
        for (uint32_t todo = mine; todo; todo &= todo - 1u) {
            const int l = __builtin_ctz(todo);
            for (uint32_t nb = q.adj[l]; nb; nb &= nb - 1u) {
                const int l2 = __builtin_ctz(nb);
                const uint32_t *row2 = bits + static_cast<unsigned long long>(l2) * wp;
                const uint2 b = slice(loff, stride, v, q.lab[l2]);
                bool found = false;
                for (uint32_t p = b.x; p < b.y && !found; ++p) found = has_bit(row2, static_cast<uint32_t>(lcol[p]));
                if (!found) {
                    drop |= 1u << l;
                    break;
                }
            }
        }
        for (uint32_t todo = drop; todo; todo &= todo - 1u) {
            const int l = __builtin_ctz(todo);
            atomicAnd(bits + static_cast<unsigned long long>(l) * wp + (v >> 5), ~(1u << (v & 31u)));
        }
        if (drop) *changed = 1u;
    }
}

// Candidate lists of every position: the bitmap words were replaced by their
// popcounts and scanned (rank), so word i puts its set bits at clist[rank[i] ...].
__global__ __launch_bounds__(256) void cand_popc_kernel(const uint32_t *__restrict__ bits, unsigned long long words,
                                                        uint32_t *__restrict__ cnt) {
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
         i < static_cast<long long>(words); i += step)
        cnt[i] = static_cast<uint32_t>(__popc(bits[i]));
}

__global__ __launch_bounds__(256) void cand_list_kernel(const uint32_t *__restrict__ bits, unsigned long long wp,
                                                        int32_t k, const uint32_t *__restrict__ rank,
                                                        int32_t *__restrict__ clist, uint32_t *__restrict__ bounds) {
    const unsigned long long words = wp * static_cast<unsigned long long>(k);
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
         i < static_cast<long long>(words); i += step) {
        const unsigned long long w = static_cast<unsigned long long>(i) % wp;
        uint32_t word = bits[i];
        uint32_t at = rank[i];
        if (w == 0) bounds[static_cast<unsigned long long>(i) / wp] = at;  // first candidate of that position
        if (static_cast<unsigned long long>(i) == words - 1) bounds[k] = at + static_cast<uint32_t>(__popc(word));
        while (word) {
            const uint32_t b = static_cast<uint32_t>(__builtin_ctz(word));
            clist[at++] = static_cast<int32_t>(w * 32ull + b);
            word &= word - 1u;
        }
    }
}

// Length of every list of G': for query edge e = (src, dst) and the i-th
// candidate v of src, |N(v) restricted to C(dst)| at cnt[first + i], and the
// grand total.  blockIdx.y = e.
__global__ __launch_bounds__(256) void cand_count_kernel(const int32_t *__restrict__ lcol,
                                                         const uint32_t *__restrict__ loff, int32_t stride,
                                                         CandQuery q, const uint32_t *__restrict__ bits,
                                                         unsigned long long wp, const CandEdge *__restrict__ edges,
                                                         const int32_t *__restrict__ clist, uint32_t *__restrict__ cnt,
                                                         unsigned long long *total) {
    const CandEdge ed = edges[blockIdx.y];
    const uint32_t *rd = bits + static_cast<unsigned long long>(ed.dst) * wp;
    uint64_t sum = 0;
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < ed.len; i += step) {
        const uint32_t v = static_cast<uint32_t>(clist[ed.start + i]);
        const uint2 b = slice(loff, stride, v, q.lab[ed.dst]);
        uint32_t c = 0;
        for (uint32_t p = b.x; p < b.y; ++p) c += has_bit(rd, static_cast<uint32_t>(lcol[p])) ? 1u : 0u;
        cnt[ed.first + i] = c;
        sum += c;
    }
    sum = wave_sum64(sum);
    if (lane_id() == 0 && sum) atomicAdd(total, static_cast<unsigned long long>(sum));
}

// The lists at the offsets of the prefix sum, and their bounds.
__global__ __launch_bounds__(256) void cand_fill_kernel(const int32_t *__restrict__ lcol,
                                                        const uint32_t *__restrict__ loff, int32_t stride, int32_t n,
                                                        CandQuery q, const uint32_t *__restrict__ bits,
                                                        unsigned long long wp, const CandEdge *__restrict__ edges,
                                                        const int32_t *__restrict__ clist,
                                                        const uint32_t *__restrict__ offs, int32_t *__restrict__ gcol,
                                                        uint32_t *__restrict__ gbounds) {
    const int e = blockIdx.y;
    const CandEdge ed = edges[e];
    const uint32_t *rd = bits + static_cast<unsigned long long>(ed.dst) * wp;
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < ed.len; i += step) {
        const uint32_t v = static_cast<uint32_t>(clist[ed.start + i]);
        const uint32_t p0 = offs[ed.first + i];
        uint32_t at = p0;
        const uint2 b = slice(loff, stride, v, q.lab[ed.dst]);
        for (uint32_t p = b.x; p < b.y; ++p) {
            const int32_t w = lcol[p];
            if (has_bit(rd, static_cast<uint32_t>(w))) gcol[at++] = w;
        }
        *reinterpret_cast<uint2 *>(gbounds + 2ull * (static_cast<unsigned long long>(e) * n + v)) = make_uint2(p0, at);
    }
}

// Exclusive prefix sum in place, in three passes: per-block sums of chunks of
// kChunk values, one block scanning those sums, and each chunk rescanned with
// its offset.  The caller guarantees that the total fits 32 bits.
constexpr int kScanBlock = 256;
constexpr int kPer = 16;
constexpr unsigned long long kChunk = kScanBlock * kPer;

__device__ __forceinline__ uint32_t wave_incl(uint32_t x) {
    const uint32_t lane = lane_id();
    for (int off = 1; off < kWave; off <<= 1) {
        const int src = static_cast<int>((lane >= static_cast<uint32_t>(off) ? lane - off : lane) << 2);
        const uint32_t y = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(src, static_cast<int>(x)));
        if (lane >= static_cast<uint32_t>(off)) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread of the block; *total gets the block sum.
__device__ __forceinline__ uint32_t block_excl(uint32_t x, uint32_t *sh, uint32_t *total) {
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const uint32_t incl = wave_incl(x);
    if (lane == kWave - 1) sh[w] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (uint32_t j = 0; j < nw; ++j) {
        base += j < w ? sh[j] : 0u;
        tot += sh[j];
    }
    __syncthreads();
    *total = tot;
    return base + incl - x;
}

__global__ __launch_bounds__(kScanBlock) void chunk_sums_kernel(const uint32_t *__restrict__ x, unsigned long long m,
                                                                uint32_t *__restrict__ sums) {
    __shared__ uint32_t sh[kScanBlock / kWave];
    const unsigned long long b0 = blockIdx.x * kChunk + static_cast<unsigned long long>(threadIdx.x) * kPer;
    uint32_t local = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) local += b0 + j < m ? x[b0 + j] : 0u;
    uint32_t total = 0;
    block_excl(local, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void chunk_offsets_kernel(uint32_t *sums, unsigned long long nb) {
    __shared__ uint32_t sh[1024 / kWave];
    const unsigned long long per = (nb + blockDim.x - 1) / blockDim.x;
    const unsigned long long b = threadIdx.x * per;
    uint32_t local = 0;
    for (unsigned long long j = 0; j < per; ++j)
        if (b + j < nb) local += sums[b + j];
    uint32_t total = 0;
    uint32_t run = block_excl(local, sh, &total);
    for (unsigned long long j = 0; j < per; ++j) {
        if (b + j < nb) {
            const uint32_t t = sums[b + j];
            sums[b + j] = run;
            run += t;
        }
    }
}

__global__ __launch_bounds__(kScanBlock) void chunk_scan_kernel(uint32_t *__restrict__ x, unsigned long long m,
                                                                const uint32_t *__restrict__ sums) {
    __shared__ uint32_t sh[kScanBlock / kWave];
    const unsigned long long b0 = blockIdx.x * kChunk + static_cast<unsigned long long>(threadIdx.x) * kPer;
    uint32_t v[kPer];
    uint32_t local = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        v[j] = b0 + j < m ? x[b0 + j] : 0u;
        local += v[j];
    }
    uint32_t total = 0;
    uint32_t run = sums[blockIdx.x] + block_excl(local, sh, &total);
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        if (b0 + j < m) x[b0 + j] = run;
        run += v[j];
    }
}

unsigned grid_for(unsigned long long items, int num_cu) {
    unsigned long long blocks = (items + 255) / 256;
    const unsigned long long most = static_cast<unsigned long long>(num_cu) * 16ull;
    if (blocks > most) blocks = most;
    return static_cast<unsigned>(blocks < 1 ? 1 : blocks);
}

}  // namespace

unsigned long long cand_bitmap_words(int32_t n) { return 2ull * ((static_cast<unsigned long long>(n) + 63ull) / 64ull); }

unsigned long long cand_scan_temp_words(unsigned long long m) { return (m + kChunk - 1) / kChunk + 1; }

hipError_t launch_cand_init(const VInfo *vinfo, int32_t n, const CandQuery &q, uint32_t *bits, int num_cu,
                            hipStream_t s) {
    if (n <= 0 || q.k < 1 || q.k > kMaxK) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cand_init_kernel, dim3(grid_for(static_cast<unsigned long long>(n), num_cu)), dim3(256), 0, s,
                       vinfo, n, q, bits, cand_bitmap_words(n));
    return hipGetLastError();
}

hipError_t launch_cand_refine(const int32_t *lcol, const uint32_t *loff, int32_t stride, int32_t n,
                              const CandQuery &q, uint32_t *bits, uint32_t *changed, int num_cu, hipStream_t s) {
    if (n <= 0 || q.k < 1 || q.k > kMaxK) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cand_refine_kernel, dim3(grid_for(static_cast<unsigned long long>(n), num_cu)), dim3(256), 0,
                       s, lcol, loff, stride, n, q, bits, cand_bitmap_words(n), changed);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(uint32_t *x, unsigned long long m, uint32_t *tmp, hipStream_t s) {
    if (m == 0) return hipSuccess;
    const unsigned long long nb = (m + kChunk - 1) / kChunk;
    if (nb > 0xffffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chunk_sums_kernel, dim3(static_cast<unsigned>(nb)), dim3(kScanBlock), 0, s, x, m, tmp);
    hipLaunchKernelGGL(chunk_offsets_kernel, dim3(1), dim3(1024), 0, s, tmp, nb);
    hipLaunchKernelGGL(chunk_scan_kernel, dim3(static_cast<unsigned>(nb)), dim3(kScanBlock), 0, s, x, m, tmp);
    return hipGetLastError();
}

hipError_t launch_cand_lists(const uint32_t *bits, int32_t n, int32_t k, uint32_t *rank, uint32_t *tmp,
                             int32_t *clist, uint32_t *bounds, int num_cu, hipStream_t s) {
    if (n <= 0 || k < 1 || k > kMaxK) return hipErrorInvalidValue;
    const unsigned long long wp = cand_bitmap_words(n), words = wp * static_cast<unsigned long long>(k);
    hipLaunchKernelGGL(cand_popc_kernel, dim3(grid_for(words, num_cu)), dim3(256), 0, s, bits, words, rank);
    hipError_t h = hipGetLastError();
    if (h == hipSuccess) h = launch_exclusive_scan(rank, words, tmp, s);
    if (h != hipSuccess) return h;
    hipLaunchKernelGGL(cand_list_kernel, dim3(grid_for(words, num_cu)), dim3(256), 0, s, bits, wp, k, rank, clist,
                       bounds);
    return hipGetLastError();
}

hipError_t launch_cand_count(const int32_t *lcol, const uint32_t *loff, int32_t stride, int32_t n,
                             const CandQuery &q, const uint32_t *bits, const CandEdge *edges, int32_t m,
                             unsigned long long most, const int32_t *clist, uint32_t *cnt, unsigned long long *total,
                             int num_cu, hipStream_t s) {
    if (n <= 0 || m < 1 || m > kMaxCandEdges) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cand_count_kernel, dim3(grid_for(most, num_cu), static_cast<unsigned>(m)), dim3(256), 0, s,
                       lcol, loff, stride, q, bits, cand_bitmap_words(n), edges, clist, cnt, total);
    return hipGetLastError();
}

hipError_t launch_cand_fill(const int32_t *lcol, const uint32_t *loff, int32_t stride, int32_t n,
                            const CandQuery &q, const uint32_t *bits, const CandEdge *edges, int32_t m,
                            unsigned long long most, const int32_t *clist, const uint32_t *offs, int32_t *gcol,
                            uint32_t *gbounds, int num_cu, hipStream_t s) {
    if (n <= 0 || m < 1 || m > kMaxCandEdges) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cand_fill_kernel, dim3(grid_for(most, num_cu), static_cast<unsigned>(m)), dim3(256), 0, s,
                       lcol, loff, stride, n, q, bits, cand_bitmap_words(n), edges, clist, offs, gcol, gbounds);
    return hipGetLastError();
}

}  // namespace gm
