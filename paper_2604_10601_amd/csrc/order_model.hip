// Order cost model: a 3-layer perceptron that predicts the log2 search time of
// a (query, matching order) pair from the features gm_order_features builds.
// The matching order is the paper's main lever on the search space (Sec. 2.2,
// Sec. 3 uses RI's heuristic); the model ranks candidate orders so the engine
// can run the one predicted cheapest, with the heuristic order as fallback.
//
//   h1 = relu(x W1 + b1)    W1: in_dim x hidden
//   h2 = relu(h1 W2 + b2)   W2: hidden x hidden
//   y  = h2 w3 + b3         w3: hidden (kept as column 0 of a hidden x 32 matrix)
//
// Weights live as fp32 master copies (Adam state beside them) and as bf16
// copies that the products read; activations entering a product are rounded
// to bf16 (round to nearest even); every product accumulates in fp32 on the
// MFMA units (v_mfma_f32_16x16x32_bf16: one 16 x 16 output tile per wavefront,
// 32 products deep per instruction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "gmatch.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int kTile = 16;   // output tile edge
constexpr int kDepth = 32;  // products per MFMA
constexpr int kOutCols = 32;  // the last layer's weight matrix is hidden x 32, column 0 used

__host__ __device__ inline uint16_t bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<uint16_t>((u >> 16) | 0x40u);  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return static_cast<uint16_t>(u >> 16);
}

// C[M x N] = A[M x K] B[K x N] with A(i, k) = A[i * sar + k * sac] and
// B(k, j) = B[k * sbr + j * sbc], bf16 inputs, fp32 output (row stride ldc).
// M and N are multiples of 16 and K of 32 (the host pads); one wavefront per
// 16 x 16 tile, four wavefronts per block.
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const uint16_t *__restrict__ A, long long sar, long long sac,
                                                        const uint16_t *__restrict__ B, long long sbr, long long sbc,
                                                        float *__restrict__ C, long long ldc, int M, int N, int K) {
    const int lane = threadIdx.x & 63;
    const long long tile = static_cast<long long>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int tiles_n = N / kTile;
    if (tile >= static_cast<long long>(M / kTile) * tiles_n) return;
    const int i0 = static_cast<int>(tile / tiles_n) * kTile, j0 = static_cast<int>(tile % tiles_n) * kTile;
    const int row = i0 + (lane & 15), col = j0 + (lane & 15), kq = 8 * (lane >> 4);
    float4v acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += kDepth) {
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const long long k = k0 + kq + j;
            a[j] = __builtin_bit_cast(__bf16, A[row * sar + k * sac]);
            b[j] = __builtin_bit_cast(__bf16, B[k * sbr + col * sbc]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) C[static_cast<long long>(i0 + 4 * (lane >> 4) + j) * ldc + col] = acc[j];
}

__global__ void to_bf16_kernel(const float *__restrict__ x, uint16_t *__restrict__ y, long long n) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * blockDim.x)
        y[i] = bf16_bits(x[i]);
}

// Rows idx[0 .. rows) of X (row length d, bf16) into Xb; rows beyond `valid` are zero.
__global__ void gather_rows_kernel(const uint16_t *__restrict__ X, const int32_t *__restrict__ idx, int rows, int valid,
                                   int d, uint16_t *__restrict__ Xb) {
    const long long n = static_cast<long long>(rows) * d;
    for (long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int r = static_cast<int>(t / d), c = static_cast<int>(t % d);
        Xb[t] = r < valid ? X[static_cast<long long>(idx[r]) * d + c] : uint16_t(0);
    }
}

// Z[M x N] += b (per column), then relu if asked; also writes Z rounded to bf16.
__global__ void bias_act_kernel(float *__restrict__ Z, const float *__restrict__ b, int M, int N, int relu,
                                uint16_t *__restrict__ Zb) {
    const long long n = static_cast<long long>(M) * N;
    for (long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += static_cast<long long>(gridDim.x) * blockDim.x) {
        float z = Z[t] + b[t % N];
        if (relu) z = z > 0.f ? z : 0.f;
        Z[t] = z;
        if (Zb) Zb[t] = bf16_bits(z);
    }
}

// Output layer: y_i = Y[i * ldy] + b3.  For training, dY[i][0] = 2 (y_i - t_i) / valid
// for the first `valid` rows (mean squared error), zero elsewhere, and the squared
// errors are summed into *loss.
__global__ void out_grad_kernel(const float *__restrict__ Y, long long ldy, const float *__restrict__ b3,
                                const float *__restrict__ t, int M, int valid, float *__restrict__ dY,
                                uint16_t *__restrict__ dYb, float *__restrict__ loss) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) {
        float g = 0.f;
        if (i < valid) {
            const float e = Y[static_cast<long long>(i) * ldy] + b3[0] - t[i];
            g = 2.f * e / static_cast<float>(valid);
            atomicAdd(loss, e * e);
        }
        for (int c = 0; c < kOutCols; ++c) {
            const float v = c == 0 ? g : 0.f;
            dY[static_cast<long long>(i) * kOutCols + c] = v;
            dYb[static_cast<long long>(i) * kOutCols + c] = bf16_bits(v);
        }
    }
}

// dZ *= [Z > 0] (relu'), also rounded to bf16.
__global__ void relu_grad_kernel(float *__restrict__ dZ, const float *__restrict__ Z, long long n,
                                 uint16_t *__restrict__ dZb) {
    for (long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += static_cast<long long>(gridDim.x) * blockDim.x) {
        const float g = Z[t] > 0.f ? dZ[t] : 0.f;
        dZ[t] = g;
        dZb[t] = bf16_bits(g);
    }
}

// db[j] = sum over the M rows of dZ[i * ld + j], j < ncols (one thread per column).
__global__ void colsum_kernel(const float *__restrict__ dZ, int M, int ld, int ncols, float *__restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ncols) return;
    float s = 0.f;
    for (int i = 0; i < M; ++i) s += dZ[static_cast<long long>(i) * ld + j];
    db[j] = s;
}

// t[idx[r]] for the first `valid` of `rows` rows, zero beyond.
__global__ void gather_f32_kernel(const float *__restrict__ t, const int32_t *__restrict__ idx, int rows, int valid,
                                  float *__restrict__ tb) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x)
        tb[r] = r < valid ? t[idx[r]] : 0.f;
}

// Adam (Kingma and Ba, 2015) on fp32 master weights; refreshes the bf16 copy.
// mask (optional) zeroes entries that must stay zero (the unused output columns).
__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                            float c2, uint16_t *__restrict__ wb, int cols, int keep_cols) {
    for (long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += static_cast<long long>(gridDim.x) * blockDim.x) {
        if (cols && static_cast<int>(t % cols) >= keep_cols) continue;
        const float gt = g[t];
        const float mt = b1 * m[t] + (1.f - b1) * gt;
        const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
        m[t] = mt;
        v[t] = vt;
        const float wt = w[t] - lr * (mt / c1) / (std::sqrt(vt / c2) + eps);
        w[t] = wt;
        if (wb) wb[t] = bf16_bits(wt);
    }
}

unsigned grid_for(long long n, int block = 256) {
    long long g = (n + block - 1) / block;
    return static_cast<unsigned>(std::max<long long>(1, std::min<long long>(g, 4096)));
}

}  // namespace

struct gm_model {
    int device = 0;
    int in_dim = 0;  // padded to a multiple of 32
    int hidden = 0;
    std::string err;
    hipStream_t stream = nullptr;
    // parameters: fp32 master, bf16 copies, Adam moments
    struct Param {
        long long n = 0;
        int cols = 0, keep = 0;  // keep: leading columns that may be nonzero (0 = all)
        float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
        uint16_t *wb = nullptr;
    } W1, B1, W2, B2, W3, B3;
    long long step = 0;
    // activations for up to cap rows
    int cap = 0;
    uint16_t *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *dYb = nullptr, *dH2b = nullptr, *dH1b = nullptr;
    float *H1 = nullptr, *H2 = nullptr, *Y = nullptr, *dY = nullptr, *dH2 = nullptr, *dH1 = nullptr;
    float *Xf = nullptr;  // fp32 inputs before rounding
    float *tb = nullptr, *loss = nullptr;
    int32_t *idx = nullptr;

    gm_status fail(gm_status s, const std::string &m) {
        err = m;
        return s;
    }
};

namespace {

#define MTRY(M, call)                                                                                \
    do {                                                                                             \
        hipError_t h_ = (call);                                                                      \
        if (h_ != hipSuccess) return (M)->fail(GM_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(h_)); \
    } while (0)

template <class T>
hipError_t dalloc(T **p, long long n) {
    return hipMalloc(reinterpret_cast<void **>(p), static_cast<size_t>(std::max<long long>(n, 1)) * sizeof(T));
}

void free_param(gm_model::Param &p) {
    for (void *b : {static_cast<void *>(p.w), static_cast<void *>(p.g), static_cast<void *>(p.m),
                    static_cast<void *>(p.v), static_cast<void *>(p.wb)})
        if (b) (void)hipFree(b);
    p = gm_model::Param{};
}

gm_status alloc_param(gm_model *M, gm_model::Param &p, long long n, int cols, int keep) {
    p.n = n;
    p.cols = cols;
    p.keep = keep;
    MTRY(M, dalloc(&p.w, n));
    MTRY(M, dalloc(&p.g, n));
    MTRY(M, dalloc(&p.m, n));
    MTRY(M, dalloc(&p.v, n));
    MTRY(M, dalloc(&p.wb, n));
    MTRY(M, hipMemsetAsync(p.m, 0, n * sizeof(float), M->stream));
    MTRY(M, hipMemsetAsync(p.v, 0, n * sizeof(float), M->stream));
    MTRY(M, hipMemsetAsync(p.g, 0, n * sizeof(float), M->stream));
    return GM_OK;
}

gm_status upload_param(gm_model *M, gm_model::Param &p, const std::vector<float> &host) {
    MTRY(M, hipMemcpyAsync(p.w, host.data(), p.n * sizeof(float), hipMemcpyHostToDevice, M->stream));
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(p.n)), dim3(256), 0, M->stream, p.w, p.wb, p.n);
    MTRY(M, hipGetLastError());
    MTRY(M, hipStreamSynchronize(M->stream));
    return GM_OK;
}

gm_status ensure_rows(gm_model *M, int rows) {
    if (rows <= M->cap) return GM_OK;
    for (void *b : {static_cast<void *>(M->Xb), static_cast<void *>(M->H1b), static_cast<void *>(M->H2b),
                    static_cast<void *>(M->dYb), static_cast<void *>(M->dH2b), static_cast<void *>(M->dH1b),
                    static_cast<void *>(M->H1), static_cast<void *>(M->H2), static_cast<void *>(M->Y),
                    static_cast<void *>(M->dY), static_cast<void *>(M->dH2), static_cast<void *>(M->dH1),
                    static_cast<void *>(M->tb), static_cast<void *>(M->idx), static_cast<void *>(M->Xf)})
        if (b) (void)hipFree(b);
    M->cap = 0;
    const long long r = rows, D = M->in_dim, H = M->hidden;
    MTRY(M, dalloc(&M->Xb, r * D));
    MTRY(M, dalloc(&M->H1b, r * H));
    MTRY(M, dalloc(&M->H2b, r * H));
    MTRY(M, dalloc(&M->dYb, r * kOutCols));
    MTRY(M, dalloc(&M->dH2b, r * H));
    MTRY(M, dalloc(&M->dH1b, r * H));
    MTRY(M, dalloc(&M->H1, r * H));
    MTRY(M, dalloc(&M->H2, r * H));
    MTRY(M, dalloc(&M->Y, r * kOutCols));
    MTRY(M, dalloc(&M->dY, r * kOutCols));
    MTRY(M, dalloc(&M->dH2, r * H));
    MTRY(M, dalloc(&M->dH1, r * H));
    MTRY(M, dalloc(&M->tb, r));
    MTRY(M, dalloc(&M->idx, r));
    MTRY(M, dalloc(&M->Xf, r * D));
    M->cap = rows;
    return GM_OK;
}

// C = A B on the model's stream; strides as in gemm_bf16_kernel.
void gemm(gm_model *M, const uint16_t *A, long long sar, long long sac, const uint16_t *B, long long sbr,
          long long sbc, float *C, long long ldc, int m, int n, int k) {
    const long long tiles = static_cast<long long>(m / kTile) * (n / kTile);
    hipLaunchKernelGGL(gemm_bf16_kernel, dim3(static_cast<unsigned>((tiles + 3) / 4)), dim3(256), 0, M->stream, A, sar,
                       sac, B, sbr, sbc, C, ldc, m, n, k);
}

// Forward pass over the `rows` rows in M->Xb (rows: a multiple of 32).
void forward(gm_model *M, int rows) {
    const int D = M->in_dim, H = M->hidden;
    gemm(M, M->Xb, D, 1, M->W1.wb, H, 1, M->H1, H, rows, H, D);
    hipLaunchKernelGGL(bias_act_kernel, dim3(grid_for(static_cast<long long>(rows) * H)), dim3(256), 0, M->stream,
                       M->H1, M->B1.w, rows, H, 1, M->H1b);
    gemm(M, M->H1b, H, 1, M->W2.wb, H, 1, M->H2, H, rows, H, H);
    hipLaunchKernelGGL(bias_act_kernel, dim3(grid_for(static_cast<long long>(rows) * H)), dim3(256), 0, M->stream,
                       M->H2, M->B2.w, rows, H, 1, M->H2b);
    gemm(M, M->H2b, H, 1, M->W3.wb, kOutCols, 1, M->Y, kOutCols, rows, kOutCols, H);
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace

extern "C" {

gm_status gm_model_create(int32_t device, int32_t in_dim, int32_t hidden, uint64_t seed, gm_model **out) {
    if (!out || in_dim < 1 || in_dim > 4096 || hidden < 32 || hidden > 1024 || hidden % 32) return GM_ERR_ARG;
    *out = nullptr;
    gm_model *M = new (std::nothrow) gm_model();
    if (!M) return GM_ERR_NOMEM;
    M->device = device;
    M->in_dim = round_up(in_dim, kDepth);
    M->hidden = hidden;
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&M->stream, hipStreamNonBlocking) != hipSuccess) {
        delete M;
        return GM_ERR_DEVICE;
    }
    const long long D = M->in_dim, H = hidden;
    gm_status st = alloc_param(M, M->W1, D * H, 0, 0);
    if (!st) st = alloc_param(M, M->B1, H, 0, 0);
    if (!st) st = alloc_param(M, M->W2, H * H, 0, 0);
    if (!st) st = alloc_param(M, M->B2, H, 0, 0);
    if (!st) st = alloc_param(M, M->W3, H * kOutCols, kOutCols, 1);
    if (!st) st = alloc_param(M, M->B3, 1, 0, 0);
    if (st) {
        gm_model_destroy(M);
        return st;
    }
    // He initialisation for the relu layers, small output layer; padded inputs have zero weights
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.f, 1.f);
    std::vector<float> w1(D * H, 0.f), w2(H * H), w3(H * kOutCols, 0.f), b1(H, 0.f), b2(H, 0.f), b3(1, 0.f);
    const float s1 = std::sqrt(2.f / static_cast<float>(in_dim)), s2 = std::sqrt(2.f / static_cast<float>(H));
    for (long long i = 0; i < static_cast<long long>(in_dim) * H; ++i) w1[i] = s1 * nd(rng);
    for (auto &x : w2) x = s2 * nd(rng);
    for (long long i = 0; i < H; ++i) w3[i * kOutCols] = std::sqrt(1.f / static_cast<float>(H)) * nd(rng);
    st = upload_param(M, M->W1, w1);
    if (!st) st = upload_param(M, M->B1, b1);
    if (!st) st = upload_param(M, M->W2, w2);
    if (!st) st = upload_param(M, M->B2, b2);
    if (!st) st = upload_param(M, M->W3, w3);
    if (!st) st = upload_param(M, M->B3, b3);
    if (st) {
        gm_model_destroy(M);
        return st;
    }
    *out = M;
    return GM_OK;
}

void gm_model_destroy(gm_model *M) {
    if (!M) return;
    (void)hipSetDevice(M->device);
    if (M->stream) (void)hipStreamSynchronize(M->stream);
    for (gm_model::Param *p : {&M->W1, &M->B1, &M->W2, &M->B2, &M->W3, &M->B3}) free_param(*p);
    for (void *b : {static_cast<void *>(M->Xb), static_cast<void *>(M->H1b), static_cast<void *>(M->H2b),
                    static_cast<void *>(M->dYb), static_cast<void *>(M->dH2b), static_cast<void *>(M->dH1b),
                    static_cast<void *>(M->H1), static_cast<void *>(M->H2), static_cast<void *>(M->Y),
                    static_cast<void *>(M->dY), static_cast<void *>(M->dH2), static_cast<void *>(M->dH1),
                    static_cast<void *>(M->tb), static_cast<void *>(M->idx), static_cast<void *>(M->loss),
                    static_cast<void *>(M->Xf)})
        if (b) (void)hipFree(b);
    if (M->stream) (void)hipStreamDestroy(M->stream);
    delete M;
}

gm_status gm_model_get_params(const gm_model *M, float *w1, float *b1, float *w2, float *b2, float *w3, float *b3) {
    if (!M || !w1 || !b1 || !w2 || !b2 || !w3 || !b3) return GM_ERR_ARG;
    gm_model *m = const_cast<gm_model *>(M);
    MTRY(m, hipSetDevice(M->device));
    const long long D = M->in_dim, H = M->hidden;
    MTRY(m, hipMemcpy(w1, M->W1.w, D * H * sizeof(float), hipMemcpyDeviceToHost));
    MTRY(m, hipMemcpy(b1, M->B1.w, H * sizeof(float), hipMemcpyDeviceToHost));
    MTRY(m, hipMemcpy(w2, M->W2.w, H * H * sizeof(float), hipMemcpyDeviceToHost));
    MTRY(m, hipMemcpy(b2, M->B2.w, H * sizeof(float), hipMemcpyDeviceToHost));
    std::vector<float> w3p(static_cast<size_t>(H * kOutCols));
    MTRY(m, hipMemcpy(w3p.data(), M->W3.w, w3p.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (long long i = 0; i < H; ++i) w3[i] = w3p[i * kOutCols];
    MTRY(m, hipMemcpy(b3, M->B3.w, sizeof(float), hipMemcpyDeviceToHost));
    return GM_OK;
}

gm_status gm_model_set_params(gm_model *M, const float *w1, const float *b1, const float *w2, const float *b2,
                              const float *w3, const float *b3) {
    if (!M || !w1 || !b1 || !w2 || !b2 || !w3 || !b3) return GM_ERR_ARG;
    MTRY(M, hipSetDevice(M->device));
    const long long D = M->in_dim, H = M->hidden;
    std::vector<float> w3p(static_cast<size_t>(H * kOutCols), 0.f);
    for (long long i = 0; i < H; ++i) w3p[i * kOutCols] = w3[i];
    gm_status st = upload_param(M, M->W1, std::vector<float>(w1, w1 + D * H));
    if (!st) st = upload_param(M, M->B1, std::vector<float>(b1, b1 + H));
    if (!st) st = upload_param(M, M->W2, std::vector<float>(w2, w2 + H * H));
    if (!st) st = upload_param(M, M->B2, std::vector<float>(b2, b2 + H));
    if (!st) st = upload_param(M, M->W3, w3p);
    if (!st) st = upload_param(M, M->B3, std::vector<float>(b3, b3 + 1));
    if (!st) {
        for (gm_model::Param *p : {&M->W1, &M->B1, &M->W2, &M->B2, &M->W3, &M->B3}) {
            MTRY(M, hipMemsetAsync(p->m, 0, p->n * sizeof(float), M->stream));
            MTRY(M, hipMemsetAsync(p->v, 0, p->n * sizeof(float), M->stream));
        }
        M->step = 0;
        MTRY(M, hipStreamSynchronize(M->stream));
    }
    return st;
}

gm_status gm_model_predict(gm_model *M, const float *x, int32_t n, int32_t dim, float *y) {
    if (!M || n < 0 || (n > 0 && (!x || !y)) || dim < 1 || dim > M->in_dim) return GM_ERR_ARG;
    if (n == 0) return GM_OK;
    MTRY(M, hipSetDevice(M->device));
    const int D = M->in_dim;
    constexpr int kChunk = 4096;
    std::vector<float> xp;
    std::vector<float> yp;
    for (int r0 = 0; r0 < n; r0 += kChunk) {
        const int rows = std::min(kChunk, n - r0), padded = round_up(rows, kDepth);
        gm_status st = ensure_rows(M, padded);
        if (st) return st;
        xp.assign(static_cast<size_t>(padded) * D, 0.f);
        for (int r = 0; r < rows; ++r)
            std::copy(x + static_cast<long long>(r0 + r) * dim, x + static_cast<long long>(r0 + r + 1) * dim,
                      xp.begin() + static_cast<long long>(r) * D);
        MTRY(M, hipMemcpyAsync(M->Xf, xp.data(), xp.size() * sizeof(float), hipMemcpyHostToDevice, M->stream));
        hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(static_cast<long long>(padded) * D)), dim3(256), 0, M->stream,
                           M->Xf, M->Xb, static_cast<long long>(padded) * D);
        forward(M, padded);
        yp.resize(static_cast<size_t>(padded) * kOutCols);
        MTRY(M, hipMemcpyAsync(yp.data(), M->Y, yp.size() * sizeof(float), hipMemcpyDeviceToHost, M->stream));
        float b3 = 0.f;
        MTRY(M, hipMemcpyAsync(&b3, M->B3.w, sizeof(float), hipMemcpyDeviceToHost, M->stream));
        MTRY(M, hipStreamSynchronize(M->stream));
        for (int r = 0; r < rows; ++r) y[r0 + r] = yp[static_cast<size_t>(r) * kOutCols] + b3;
    }
    return GM_OK;
}

gm_status gm_model_train(gm_model *M, const float *x, const float *t, int32_t n, int32_t dim, int32_t epochs,
                         int32_t batch, float lr, uint64_t seed, float *mean_loss) {
    if (!M || n < 1 || !x || !t || dim < 1 || dim > M->in_dim || epochs < 0 || batch < 1 || !(lr > 0.f))
        return GM_ERR_ARG;
    MTRY(M, hipSetDevice(M->device));
    const int D = M->in_dim, H = M->hidden;
    const int B = round_up(std::min(batch, n), kDepth);
    // whole training set on the device, in bf16, padded rows of D
    if (M->in_dim * static_cast<long long>(n) > (1ll << 31)) return M->fail(GM_ERR_ARG, "training set too large");
    gm_status st = ensure_rows(M, std::max(B, 32));
    if (st) return st;
    std::vector<float> xp(static_cast<size_t>(n) * D, 0.f);
    for (int r = 0; r < n; ++r)
        std::copy(x + static_cast<long long>(r) * dim, x + static_cast<long long>(r + 1) * dim,
                  xp.begin() + static_cast<long long>(r) * D);
    float *dx = nullptr, *dt = nullptr;
    uint16_t *dxb = nullptr;
    auto cleanup = [&]() {
        if (dx) (void)hipFree(dx);
        if (dt) (void)hipFree(dt);
        if (dxb) (void)hipFree(dxb);
    };
    if (dalloc(&dx, static_cast<long long>(n) * D) != hipSuccess || dalloc(&dt, n) != hipSuccess ||
        dalloc(&dxb, static_cast<long long>(n) * D) != hipSuccess || (!M->loss && dalloc(&M->loss, 1) != hipSuccess)) {
        cleanup();
        return M->fail(GM_ERR_NOMEM, "training set upload");
    }
    hipError_t h = hipMemcpyAsync(dx, xp.data(), xp.size() * sizeof(float), hipMemcpyHostToDevice, M->stream);
    if (h == hipSuccess) h = hipMemcpyAsync(dt, t, static_cast<size_t>(n) * sizeof(float), hipMemcpyHostToDevice, M->stream);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(static_cast<long long>(n) * D)), dim3(256), 0, M->stream, dx, dxb,
                       static_cast<long long>(n) * D);
    if (h == hipSuccess) h = hipMemsetAsync(M->loss, 0, sizeof(float), M->stream);
    std::vector<int32_t> order(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) order[i] = i;
    std::mt19937_64 rng(seed);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    long long seen = 0;
    for (int ep = 0; ep < epochs && h == hipSuccess; ++ep) {
        std::shuffle(order.begin(), order.end(), rng);
        h = hipMemsetAsync(M->loss, 0, sizeof(float), M->stream);  // the last epoch's loss is reported
        seen = 0;
        for (int r0 = 0; r0 < n && h == hipSuccess; r0 += B) {
            const int valid = std::min(B, n - r0);
            h = hipMemcpyAsync(M->idx, order.data() + r0, static_cast<size_t>(valid) * sizeof(int32_t),
                               hipMemcpyHostToDevice, M->stream);
            if (h != hipSuccess) break;
            // rows and targets of the batch (padding rows are zero and carry no gradient)
            hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for(static_cast<long long>(B) * D)), dim3(256), 0,
                               M->stream, dxb, M->idx, B, valid, D, M->Xb);
            hipLaunchKernelGGL(gather_f32_kernel, dim3(grid_for(B)), dim3(256), 0, M->stream, dt, M->idx, B, valid,
                               M->tb);
            forward(M, B);
            hipLaunchKernelGGL(out_grad_kernel, dim3(grid_for(B)), dim3(256), 0, M->stream, M->Y,
                               static_cast<long long>(kOutCols), M->B3.w, M->tb, B, valid, M->dY, M->dYb, M->loss);
            // output layer: dW3 = H2^T dY, db3 = sum dY[:, 0], dH2 = dY W3^T
            gemm(M, M->H2b, 1, H, M->dYb, kOutCols, 1, M->W3.g, kOutCols, H, kOutCols, B);
            hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(64), 0, M->stream, M->dY, B, kOutCols, 1, M->B3.g);
            gemm(M, M->dYb, kOutCols, 1, M->W3.wb, 1, kOutCols, M->dH2, H, B, H, kOutCols);
            hipLaunchKernelGGL(relu_grad_kernel, dim3(grid_for(static_cast<long long>(B) * H)), dim3(256), 0,
                               M->stream, M->dH2, M->H2, static_cast<long long>(B) * H, M->dH2b);
            // layer 2: dW2 = H1^T dH2, db2 = colsum, dH1 = dH2 W2^T
            gemm(M, M->H1b, 1, H, M->dH2b, H, 1, M->W2.g, H, H, H, B);
            hipLaunchKernelGGL(colsum_kernel, dim3((H + 63) / 64), dim3(64), 0, M->stream, M->dH2, B, H, H, M->B2.g);
            gemm(M, M->dH2b, H, 1, M->W2.wb, 1, H, M->dH1, H, B, H, H);
            hipLaunchKernelGGL(relu_grad_kernel, dim3(grid_for(static_cast<long long>(B) * H)), dim3(256), 0,
                               M->stream, M->dH1, M->H1, static_cast<long long>(B) * H, M->dH1b);
            // layer 1: dW1 = X^T dH1, db1 = colsum
            gemm(M, M->Xb, 1, D, M->dH1b, H, 1, M->W1.g, H, D, H, B);
            hipLaunchKernelGGL(colsum_kernel, dim3((H + 63) / 64), dim3(64), 0, M->stream, M->dH1, B, H, H, M->B1.g);
            ++M->step;
            const float c1 = 1.f - std::pow(b1, static_cast<float>(M->step));
            const float c2 = 1.f - std::pow(b2, static_cast<float>(M->step));
            for (gm_model::Param *p : {&M->W1, &M->B1, &M->W2, &M->B2, &M->W3, &M->B3})
                hipLaunchKernelGGL(adam_kernel, dim3(grid_for(p->n)), dim3(256), 0, M->stream, p->w, p->g, p->m,
                                   p->v, p->n, lr, b1, b2, eps, c1, c2, p->wb, p->cols, p->keep ? p->keep : p->cols);
            h = hipGetLastError();
            seen += valid;
        }
    }
    float loss_sum = 0.f;
    if (h == hipSuccess) h = hipMemcpyAsync(&loss_sum, M->loss, sizeof(float), hipMemcpyDeviceToHost, M->stream);
    if (h == hipSuccess) h = hipStreamSynchronize(M->stream);
    cleanup();
    if (h != hipSuccess) return M->fail(GM_ERR_DEVICE, std::string("training: ") + hipGetErrorString(h));
    if (mean_loss) *mean_loss = seen ? loss_sum / static_cast<float>(seen) : 0.f;
    return GM_OK;
}

const char *gm_model_last_error(const gm_model *M) { return M ? M->err.c_str() : "null model"; }

}  // extern "C"
