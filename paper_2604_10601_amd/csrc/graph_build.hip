// gfx950 kernels that check an input graph and build the engine's derived
// structures from it on the device (the load step of the C ABI, before any
// query; Def. 1 fixes what a data graph is: simple, undirected, labelled).
//
//   * row_ptr check: non-decreasing offsets that start at 0.
//   * entry check, one wavefront per vertex: every neighbour id in [0, n), rows
//     strictly ascending (so no duplicate edges), no self-loops, degree below
//     2^24 (the vertex record's field), and, unless the caller trusts its input,
//     symmetry (each stored edge found in the other endpoint's row by bisection).
//   * vertex records: (first adjacency slot, degree << 8 | compact label).
//   * label slices, one wavefront per vertex: N(v) reordered by (label, id) into
//     lcol, with the slice bounds of every label in loff.  Each 64-entry chunk
//     is split by label with ballots (one round per distinct label in the chunk)
//     and the chunks are taken in order, so each slice keeps the ascending id
//     order the membership tests bisect.
//   * hub adjacency bitmaps: one bit per vertex of G for each chosen hub.
//
// Row offsets come as 4- or 8-byte integers (both are common in caller-owned
// device buffers); every other array has one fixed type.
#include <hip/hip_runtime.h>

#include "gm_internal.h"

namespace gm {

namespace {

constexpr int kGbBlock = 256;
constexpr int kGbWaves = kGbBlock / kWave;

__device__ __forceinline__ uint32_t gb_lane() { return threadIdx.x & (kWave - 1); }

template <typename RP>
__device__ __forceinline__ long long rp_at(const void *row_ptr, long long i) {
    return static_cast<long long>(static_cast<const RP *>(row_ptr)[i]);
}

template <typename RP>
__global__ __launch_bounds__(kGbBlock) void gb_rowptr_kernel(const void *row_ptr, int32_t n, unsigned int *err) {
    for (long long v = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += static_cast<long long>(gridDim.x) * blockDim.x) {
        const long long a = rp_at<RP>(row_ptr, v), b = rp_at<RP>(row_ptr, v + 1);
        unsigned int bad = 0;
        if (b < a) bad |= kGraphBadRowPtr;
        if (v == 0 && a != 0) bad |= kGraphBadRowPtr;
        if (b - a >= (1ll << 24)) bad |= kGraphBadDegree;
        if (bad) atomicOr(err, bad);
    }
}

// Requires offsets that passed gb_rowptr_kernel (so every row lies inside col).
template <typename RP>
__global__ __launch_bounds__(kGbBlock) void gb_entries_kernel(const void *row_ptr, const int32_t *__restrict__ col,
                                                              int32_t n, int32_t symmetric, unsigned int *err) {
    const uint32_t lane = gb_lane();
    const long long waves = static_cast<long long>(gridDim.x) * kGbWaves;
    unsigned int bad = 0;
    for (long long v = static_cast<long long>(blockIdx.x) * kGbWaves + threadIdx.x / kWave; v < n; v += waves) {
        const long long lo = rp_at<RP>(row_ptr, v), hi = rp_at<RP>(row_ptr, v + 1);
        for (long long p = lo + lane; p < hi; p += kWave) {
            const int32_t w = col[p];
            if (w < 0 || w >= n || w == v || (p > lo && col[p - 1] >= w)) {
                bad |= kGraphBadEntry;
                continue;
            }
            if (symmetric) {
                long long a = rp_at<RP>(row_ptr, w), b = rp_at<RP>(row_ptr, w + 1);
                while (a < b) {
                    const long long mid = a + ((b - a) >> 1);
                    if (col[mid] < v) a = mid + 1;
                    else b = mid;
                }
                if (a >= rp_at<RP>(row_ptr, w + 1) || col[a] != v) bad |= kGraphAsymmetric;
            }
        }
    }
    if (bad) atomicOr(err, bad);
}

__global__ __launch_bounds__(kGbBlock) void gb_label_hist_kernel(const uint8_t *__restrict__ labels, int32_t n,
                                                                 unsigned int *hist) {
    __shared__ unsigned int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (long long v = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += static_cast<long long>(gridDim.x) * blockDim.x)
        atomicAdd(&h[labels[v]], 1u);
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

struct LabelMap {
    uint8_t id[256];
};

__global__ __launch_bounds__(kGbBlock) void gb_label_map_kernel(const uint8_t *__restrict__ labels, int32_t n,
                                                                LabelMap map, uint8_t *__restrict__ clab) {
    for (long long v = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += static_cast<long long>(gridDim.x) * blockDim.x)
        clab[v] = map.id[labels[v]];
}

// Vertex records; loff32, if given, receives the offsets as 32-bit values.
template <typename RP>
__global__ __launch_bounds__(kGbBlock) void gb_vinfo_kernel(const void *row_ptr, const uint8_t *__restrict__ clab,
                                                            int32_t n, VInfo *__restrict__ vinfo,
                                                            uint32_t *__restrict__ loff32) {
    for (long long v = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += static_cast<long long>(gridDim.x) * blockDim.x) {
        const long long a = rp_at<RP>(row_ptr, v), b = rp_at<RP>(row_ptr, v + 1);
        vinfo[v] = make_uint2(static_cast<uint32_t>(a), (static_cast<uint32_t>(b - a) << 8) | clab[v]);
        if (loff32) {
            loff32[v] = static_cast<uint32_t>(a);
            if (v == n - 1) loff32[n] = static_cast<uint32_t>(b);
        }
    }
}

// Label slices of N(v): loff[v * stride + c] is the first slot of label c's
// slice in lcol, loff[v * stride + stride - 1] the end of N(v) (stride = labels + 1).
__global__ __launch_bounds__(kGbBlock) void gb_slices_kernel(const VInfo *__restrict__ vinfo,
                                                             const int32_t *__restrict__ col, int32_t n,
                                                             int32_t stride, uint32_t *__restrict__ loff,
                                                             int32_t *__restrict__ lcol) {
    __shared__ uint32_t cnt_all[kGbWaves][256];
    const uint32_t lane = gb_lane();
    uint32_t *cnt = cnt_all[threadIdx.x / kWave];
    const long long waves = static_cast<long long>(gridDim.x) * kGbWaves;
    const int32_t labels = stride - 1;
    for (long long v = static_cast<long long>(blockIdx.x) * kGbWaves + threadIdx.x / kWave; v < n; v += waves) {
        const VInfo vi = vinfo[v];
        const uint32_t start = vi.x, deg = vi.y >> 8;
        for (int32_t c = lane; c < stride; c += kWave) cnt[c] = 0;
        __builtin_amdgcn_wave_barrier();
        // per-label sizes
        for (uint32_t b = 0; b < deg; b += kWave) {
            const bool have = b + lane < deg;
            const uint32_t lab = have ? (vinfo[col[start + b + lane]].y & 0xffu) : 0u;
            uint64_t left = __ballot(have);
            while (left) {
                const uint32_t leader = static_cast<uint32_t>(__builtin_ctzll(left));
                const uint32_t c = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(lab), static_cast<int>(leader)));
                const uint64_t m = __ballot(have && lab == c) & left;
                if (lane == leader) cnt[c] += static_cast<uint32_t>(__popcll(m));
                left &= ~m;
            }
            __builtin_amdgcn_wave_barrier();
        }
        // slice bounds: exclusive prefix over labels (a lane per label, <= 255 labels)
        uint32_t run = start;
        for (int32_t c0 = 0; c0 < labels; c0 += kWave) {
            const int32_t c = c0 + static_cast<int32_t>(lane);
            uint32_t x = c < labels ? cnt[c] : 0u;
            uint32_t incl = x;
            for (uint32_t off = 1; off < kWave; off <<= 1) {
                const uint32_t y = static_cast<uint32_t>(
                    __builtin_amdgcn_ds_bpermute(static_cast<int>((lane >= off ? lane - off : lane) << 2), static_cast<int>(incl)));
                if (lane >= off) incl += y;
            }
            const uint32_t first = run + incl - x;
            __builtin_amdgcn_wave_barrier();
            if (c < labels) {
                loff[static_cast<unsigned long long>(v) * stride + c] = first;
                cnt[c] = first;  // fill cursor
            }
            run += static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(incl), kWave - 1));
        }
        if (lane == 0) loff[static_cast<unsigned long long>(v) * stride + labels] = start + deg;
        __builtin_amdgcn_wave_barrier();
        // stable fill: chunks in order, lanes in order within a label
        for (uint32_t b = 0; b < deg; b += kWave) {
            const bool have = b + lane < deg;
            const int32_t w = have ? col[start + b + lane] : 0;
            const uint32_t lab = have ? (vinfo[w].y & 0xffu) : 0u;
            uint64_t left = __ballot(have);
            while (left) {
                const uint32_t leader = static_cast<uint32_t>(__builtin_ctzll(left));
                const uint32_t c = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(lab), static_cast<int>(leader)));
                const uint64_t m = __ballot(have && lab == c) & left;
                const uint32_t base = cnt[c];
                if ((m >> lane) & 1ull) {
                    const uint32_t below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
                    lcol[base + below] = w;
                }
                __builtin_amdgcn_wave_barrier();
                if (lane == leader) cnt[c] = base + static_cast<uint32_t>(__popcll(m));
                __builtin_amdgcn_wave_barrier();
                left &= ~m;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ __launch_bounds__(kGbBlock) void gb_hub_bits_kernel(const VInfo *__restrict__ vinfo,
                                                               const int32_t *__restrict__ col,
                                                               const int32_t *__restrict__ hubs, int32_t nh,
                                                               uint32_t *__restrict__ bits, unsigned long long words) {
    for (int32_t h = blockIdx.x; h < nh; h += gridDim.x) {
        const VInfo vi = vinfo[hubs[h]];
        const uint32_t start = vi.x, deg = vi.y >> 8;
        uint32_t *row = bits + static_cast<unsigned long long>(h) * words;
        for (uint32_t p = threadIdx.x; p < deg; p += blockDim.x) {
            const uint32_t w = static_cast<uint32_t>(col[start + p]);
            atomicOr(&row[w >> 5], 1u << (w & 31u));
        }
    }
}

__global__ __launch_bounds__(kGbBlock) void gb_hub_id_kernel(const int32_t *__restrict__ hubs, int32_t nh,
                                                             int32_t *__restrict__ hub_id) {
    const int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h < nh) hub_id[hubs[h]] = h;
}

unsigned int grid_for(long long items, int per_block, int num_cu) {
    long long b = (items + per_block - 1) / per_block;
    const long long cap = static_cast<long long>(num_cu > 0 ? num_cu : 1) * 16;
    if (b > cap) b = cap;
    return static_cast<unsigned int>(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_graph_check(const void *row_ptr, int row_ptr_bytes, const int32_t *col, int32_t n, bool symmetric,
                              unsigned int *err, bool entries, int num_cu, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (row_ptr_bytes != 4 && row_ptr_bytes != 8) return hipErrorInvalidValue;
    if (!entries) {
        const unsigned int g = grid_for(n, kGbBlock, num_cu);
        if (row_ptr_bytes == 8) hipLaunchKernelGGL(gb_rowptr_kernel<long long>, dim3(g), dim3(kGbBlock), 0, s, row_ptr, n, err);
        else hipLaunchKernelGGL(gb_rowptr_kernel<int32_t>, dim3(g), dim3(kGbBlock), 0, s, row_ptr, n, err);
    } else {
        const unsigned int g = grid_for(n, kGbWaves, num_cu);
        if (row_ptr_bytes == 8)
            hipLaunchKernelGGL(gb_entries_kernel<long long>, dim3(g), dim3(kGbBlock), 0, s, row_ptr, col, n,
                               symmetric ? 1 : 0, err);
        else
            hipLaunchKernelGGL(gb_entries_kernel<int32_t>, dim3(g), dim3(kGbBlock), 0, s, row_ptr, col, n,
                               symmetric ? 1 : 0, err);
    }
    return hipGetLastError();
}

hipError_t launch_label_hist(const uint8_t *labels, int32_t n, unsigned int *hist256, int num_cu, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gb_label_hist_kernel, dim3(grid_for(n, kGbBlock, num_cu)), dim3(kGbBlock), 0, s, labels, n,
                       hist256);
    return hipGetLastError();
}

hipError_t launch_label_map(const uint8_t *labels, int32_t n, const uint8_t *map256, uint8_t *clab, int num_cu,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    LabelMap m;
    for (int i = 0; i < 256; ++i) m.id[i] = map256[i];
    hipLaunchKernelGGL(gb_label_map_kernel, dim3(grid_for(n, kGbBlock, num_cu)), dim3(kGbBlock), 0, s, labels, n, m,
                       clab);
    return hipGetLastError();
}

hipError_t launch_graph_build(const void *row_ptr, int row_ptr_bytes, const int32_t *col, const uint8_t *clab,
                              int32_t n, int32_t stride, VInfo *vinfo, uint32_t *loff, int32_t *lcol, int num_cu,
                              hipStream_t s) {
    if (n <= 0) {
        if (stride <= 1) return hipMemsetAsync(loff, 0, sizeof(uint32_t), s);  // loff[0] = 0
        return hipSuccess;
    }
    if (row_ptr_bytes != 4 && row_ptr_bytes != 8) return hipErrorInvalidValue;
    const unsigned int g = grid_for(n, kGbBlock, num_cu);
    uint32_t *loff32 = stride > 1 ? nullptr : loff;
    if (row_ptr_bytes == 8)
        hipLaunchKernelGGL(gb_vinfo_kernel<long long>, dim3(g), dim3(kGbBlock), 0, s, row_ptr, clab, n, vinfo, loff32);
    else
        hipLaunchKernelGGL(gb_vinfo_kernel<int32_t>, dim3(g), dim3(kGbBlock), 0, s, row_ptr, clab, n, vinfo, loff32);
    if (stride > 1)
        hipLaunchKernelGGL(gb_slices_kernel, dim3(grid_for(n, kGbWaves, num_cu)), dim3(kGbBlock), 0, s, vinfo, col, n,
                           stride, loff, lcol);
    return hipGetLastError();
}

hipError_t launch_hub_bitmaps(const VInfo *vinfo, const int32_t *col, const int32_t *hubs, int32_t nh, uint32_t *bits,
                              unsigned long long words, int32_t *hub_id, int num_cu, hipStream_t s) {
    if (nh <= 0) return hipSuccess;
    hipLaunchKernelGGL(gb_hub_bits_kernel, dim3(grid_for(nh, 1, num_cu)), dim3(kGbBlock), 0, s, vinfo, col, hubs, nh,
                       bits, words);
    hipLaunchKernelGGL(gb_hub_id_kernel, dim3((nh + kGbBlock - 1) / kGbBlock), dim3(kGbBlock), 0, s, hubs, nh, hub_id);
    return hipGetLastError();
}

}  // namespace gm
