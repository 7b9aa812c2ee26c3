// Kernels of the learned plan chooser: exact column statistics (distinct
// count and largest value frequencies) that its features are made of, and a
// small FP32 multilayer perceptron with training (forward, backward, Adam)
// and inference, all on the GPU.
//
// The perceptron:
//
//   h1 = relu(X W1 + b1)    X: B x D,  W1: D x H
//   h2 = relu(h1 W2 + b2)   W2: H x H
//   y  = h2 W3 + b3         W3: H x 1
//   loss = mean over the batch of (y - t)^2
//
// Matrices are row-major.  Every reduction (over the batch for weight
// gradients, over the inner dimension for products) is computed by one
// thread in a fixed order, so gradients are deterministic run to run.  The
// network is tiny (66 K multiply-adds per row), so plain FMA tiles are used
// rather than matrix cores.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdint>

#include "fj_launch.h"

namespace fj {

constexpr int kTile = 16;

// C[M x N] = op(A) op(B) (+ bias) (relu), op = transpose when the flag is set.
// A is M x K (or K x M when ta), B is K x N (or N x K when tb).
__global__ void __launch_bounds__(kTile *kTile) k_gemm(const float *__restrict__ A, const float *__restrict__ B,
                                                      const float *__restrict__ bias, float *__restrict__ C, int M,
                                                      int N, int K, int ta, int tb, int relu, int accumulate) {
    __shared__ float As[kTile][kTile + 1];
    __shared__ float Bs[kTile][kTile + 1];
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
    const int row = blockIdx.y * kTile + ty, col = blockIdx.x * kTile + tx;
    float acc = 0.f;
    for (int k0 = 0; k0 < K; k0 += kTile) {
        // A tile: rows of C, k columns
        {
            const int r = blockIdx.y * kTile + ty, k = k0 + tx;
            float a = 0.f;
            if (r < M && k < K) a = ta ? A[(size_t)k * M + r] : A[(size_t)r * K + k];
            As[ty][tx] = a;
        }
        // B tile: k rows, columns of C
        {
            const int k = k0 + ty, c = blockIdx.x * kTile + tx;
            float b = 0.f;
            if (k < K && c < N) b = tb ? B[(size_t)c * K + k] : B[(size_t)k * N + c];
            Bs[ty][tx] = b;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kTile; k++) acc = fmaf(As[ty][k], Bs[k][tx], acc);
        __syncthreads();
    }
    if (row < M && col < N) {
        if (bias) acc += bias[col];
        if (relu) acc = fmaxf(acc, 0.f);
        const size_t o = (size_t)row * N + col;
        C[o] = accumulate ? C[o] + acc : acc;
    }
}

// Inference for a few rows in one launch: one workgroup per input row, one
// thread per hidden unit; the row and both hidden layers stay in LDS.  Each
// dot product runs in index order in one thread.  x and y may be pinned
// host memory.
__global__ void k_mlp_rows(const float *__restrict__ x, int D, int H, const float *__restrict__ w, int64_t oW1,
                           int64_t ob1, int64_t oW2, int64_t ob2, int64_t oW3, int64_t ob3, float *__restrict__ y) {
    extern __shared__ float sm[];
    float *xs = sm, *h1 = sm + D, *h2 = h1 + H;
    const int r = blockIdx.x, j = threadIdx.x;
    for (int i = j; i < D; i += blockDim.x) xs[i] = x[(size_t)r * D + i];
    __syncthreads();
    if (j < H) {
        const float *W1 = w + oW1;
        float a = 0.f;
        for (int i = 0; i < D; i++) a = fmaf(xs[i], W1[(size_t)i * H + j], a);
        h1[j] = fmaxf(a + w[ob1 + j], 0.f);
    }
    __syncthreads();
    if (j < H) {
        const float *W2 = w + oW2;
        float a = 0.f;
        for (int k = 0; k < H; k++) a = fmaf(h1[k], W2[(size_t)k * H + j], a);
        h2[j] = fmaxf(a + w[ob2 + j], 0.f);
    }
    __syncthreads();
    if (j == 0) {
        float a = 0.f;
        for (int k = 0; k < H; k++) a = fmaf(h2[k], w[oW3 + k], a);
        y[r] = a + w[ob3];
    }
}

// Inference for the chooser's candidates (D, H <= 128, at most 32 rows) in
// one workgroup of 1,024 threads, so that one launch costs one round of
// memory latency: every global load (W1 and W2 as 16-byte vectors, the rows
// from pinned host memory, the biases) is issued at the start, W1 and the
// rows are kept in LDS for layer 1, and W2 replaces W1 there for layer 2.
// Thread (g, j) computes hidden unit j of rows g, g + 8, ...; each dot
// product still runs in index order in one thread, so the scores equal
// k_mlp_rows' bit for bit.
constexpr int kScoreThreads = 1024;
constexpr int kScoreMaxD = 128, kScoreMaxH = 128, kScoreMaxB = 32;
constexpr int kScoreVec = kScoreMaxD * kScoreMaxH / 4 / kScoreThreads;   // float4 of a weight matrix per thread

__global__ void __launch_bounds__(kScoreThreads) k_mlp_score(const float *__restrict__ x, int B, int D, int H,
                                                             const float *__restrict__ w, int64_t oW1, int64_t ob1,
                                                             int64_t oW2, int64_t ob2, int64_t oW3, int64_t ob3,
                                                             float *__restrict__ y) {
    __shared__ float ws[kScoreMaxD * kScoreMaxH];
    __shared__ float xs[kScoreMaxB * kScoreMaxD];
    __shared__ float h1[kScoreMaxB * kScoreMaxH];
    __shared__ float h2[kScoreMaxB * kScoreMaxH];
    const int t = threadIdx.x;
    const int nw1 = D * H / 4, nw2 = H * H / 4, nx = B * D;
    const float4 *W1 = (const float4 *)(w + oW1), *W2 = (const float4 *)(w + oW2);
    float4 a1[kScoreVec], a2[kScoreVec];
#pragma unroll
    for (int v = 0; v < kScoreVec; v++) {
        const int i = v * kScoreThreads + t;
        a1[v] = i < nw1 ? W1[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        a2[v] = i < nw2 ? W2[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float xv[(kScoreMaxB * kScoreMaxD + kScoreThreads - 1) / kScoreThreads];
#pragma unroll
    for (int v = 0; v < (kScoreMaxB * kScoreMaxD + kScoreThreads - 1) / kScoreThreads; v++) {
        const int i = v * kScoreThreads + t;
        xv[v] = i < nx ? x[i] : 0.f;
    }
    const int j = t % kScoreMaxH, g = t / kScoreMaxH;
    constexpr int kGroups = kScoreThreads / kScoreMaxH;
    const bool unit = j < H;
    const float bj1 = unit ? w[ob1 + j] : 0.f, bj2 = unit ? w[ob2 + j] : 0.f;
#pragma unroll
    for (int v = 0; v < kScoreVec; v++) {
        const int i = v * kScoreThreads + t;
        if (i < nw1) ((float4 *)ws)[i] = a1[v];
    }
#pragma unroll
    for (int v = 0; v < (kScoreMaxB * kScoreMaxD + kScoreThreads - 1) / kScoreThreads; v++) {
        const int i = v * kScoreThreads + t;
        if (i < nx) xs[i] = xv[v];
    }
    __syncthreads();
    if (unit)
        for (int r = g; r < B; r += kGroups) {
            float a = 0.f;
            for (int i = 0; i < D; i++) a = fmaf(xs[r * D + i], ws[i * H + j], a);
            h1[r * H + j] = fmaxf(a + bj1, 0.f);
        }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < kScoreVec; v++) {
        const int i = v * kScoreThreads + t;
        if (i < nw2) ((float4 *)ws)[i] = a2[v];
    }
    __syncthreads();
    if (unit)
        for (int r = g; r < B; r += kGroups) {
            float a = 0.f;
            for (int k = 0; k < H; k++) a = fmaf(h1[r * H + k], ws[k * H + j], a);
            h2[r * H + j] = fmaxf(a + bj2, 0.f);
        }
    __syncthreads();
    if (t < B) {
        float a = 0.f;
        for (int k = 0; k < H; k++) a = fmaf(h2[t * H + k], w[oW3 + k], a);
        y[t] = a + w[ob3];
    }
}

// dY = 2 (y - t) / B, and the loss terms
__global__ void k_mse_grad(const float *y, const float *t, float *dy, float *sq, int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const float d = y[i] - t[i];
    dy[i] = 2.f * d / (float)B;
    sq[i] = d * d;
}

// dZ = dH * (H > 0)   (the ReLU's derivative through its output)
__global__ void k_relu_back(const float *h, float *dz, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(h[i] > 0.f)) dz[i] = 0.f;
}

// bias gradient: column sums of dZ (B x N), one thread per column, rows in order
__global__ void k_colsum(const float *dz, float *db, int B, int N) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int i = 0; i < B; i++) s += dz[(size_t)i * N + j];
    db[j] = s;
}

// sum of a vector in index order by one thread (small B)
__global__ void k_sum(const float *x, int n, float *out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < n; i++) s += x[i];
        *out = s;
    }
}

// Adam (Kingma and Ba) with bias correction folded into the step size.
__global__ void k_adam(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------ column sketch
//
// A hash table of (value, count) with linear probing counts every value of
// the column; the distinct count is the number of occupied slots and the
// top-k frequencies are the k largest counts.  The value 0xFFFFFFFF marks an
// empty slot; rows holding that bit pattern (int32 -1) are counted in a
// separate counter instead.

constexpr uint32_t kSkEmpty = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t sk_hash(uint32_t k) {
    // MurmurHash3 32-bit finalizer
    k ^= k >> 16;
    k *= 0x85ebca6bu;
    k ^= k >> 13;
    k *= 0xc2b2ae35u;
    k ^= k >> 16;
    return k;
}

__global__ void k_sk_init(uint32_t *keys, uint32_t *cnt, uint32_t cap, unsigned long long *res) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cap) {
        keys[i] = kSkEmpty;
        cnt[i] = 0;
    }
    if (i < kSketchRes) res[i] = 0;
}

// One row per thread.  Lanes of a wave holding the same value as the wave's
// first unfinished lane are counted together (a few rounds), which takes the
// pressure of heavy hitters off single slots; the rest insert one by one.
__global__ void k_sk_insert(const int32_t *__restrict__ col, const uint32_t *__restrict__ sel, uint32_t n,
                            uint32_t *keys, uint32_t *cnt, uint32_t mask, unsigned long long *res) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool live = i < n;
    uint32_t key = 0;
    if (live) key = (uint32_t)col[sel ? sel[i] : i];
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int round = 0; round < 4; round++) {
        const unsigned long long act = __ballot(live);
        if (act == 0) return;
        const int leader = __ffsll((long long)act) - 1;
        const uint32_t lk = __shfl(key, leader);
        const bool same = live && key == lk;
        const unsigned long long grp = __ballot(same);
        if (lane == leader) {
            const uint32_t c = (uint32_t)__popcll(grp);
            if (lk == kSkEmpty) {
                atomicAdd(&res[kSkOther], (unsigned long long)c);
            } else {
                uint32_t h = sk_hash(lk) & mask;
                for (uint32_t probe = 0; probe <= mask; probe++) {
                    const uint32_t prev = atomicCAS(&keys[h], kSkEmpty, lk);
                    if (prev == kSkEmpty || prev == lk) {
                        atomicAdd(&cnt[h], c);
                        break;
                    }
                    h = (h + 1) & mask;
                }
            }
        }
        if (same) live = false;
    }
    if (!live) return;
    if (key == kSkEmpty) {
        atomicAdd(&res[kSkOther], 1ull);
        return;
    }
    uint32_t h = sk_hash(key) & mask;
    for (uint32_t probe = 0; probe <= mask; probe++) {
        const uint32_t prev = atomicCAS(&keys[h], kSkEmpty, key);
        if (prev == kSkEmpty || prev == key) {
            atomicAdd(&cnt[h], 1u);
            return;
        }
        h = (h + 1) & mask;
    }
}

// keep t[0..7] descending; v enters if it beats the smallest
__device__ __forceinline__ void top_insert(uint32_t (&t)[kSketchTop], uint32_t v) {
#pragma unroll
    for (int j = 0; j < kSketchTop; j++) {
        const uint32_t hi = t[j] > v ? t[j] : v;
        const uint32_t lo = t[j] > v ? v : t[j];
        t[j] = hi;
        v = lo;
    }
}

// Block b reduces the slots of a grid-stride slice: occupied slots are
// added to the distinct counter and the block's top-k counts go to
// part[b * k ..].  Block size kSkBlock.
constexpr int kSkBlock = 256;

__global__ void __launch_bounds__(kSkBlock) k_sk_reduce(const uint32_t *keys, const uint32_t *cnt, uint32_t cap,
                                                        uint32_t *part, unsigned long long *res) {
    __shared__ uint32_t lds[kSkBlock * kSketchTop];
    __shared__ uint32_t occ[kSkBlock / 64];
    uint32_t t[kSketchTop];
#pragma unroll
    for (int j = 0; j < kSketchTop; j++) t[j] = 0;
    uint32_t o = 0;
    for (uint32_t i = blockIdx.x * kSkBlock + threadIdx.x; i < cap; i += gridDim.x * kSkBlock) {
        if (keys[i] != kSkEmpty) {
            o++;
            top_insert(t, cnt[i]);
        }
    }
    // distinct: wave sums, one atomic per block
    for (int d = 32; d > 0; d >>= 1) o += __shfl_down(o, d);
    if ((threadIdx.x & 63) == 0) occ[threadIdx.x >> 6] = o;
#pragma unroll
    for (int j = 0; j < kSketchTop; j++) lds[threadIdx.x * kSketchTop + j] = t[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int w = 0; w < kSkBlock / 64; w++) s += occ[w];
        atomicAdd(&res[kSkDistinct], s);
    }
    // tree merge of the per-thread lists
    for (int half = kSkBlock / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) {
#pragma unroll
            for (int j = 0; j < kSketchTop; j++) top_insert(t, lds[(threadIdx.x + half) * kSketchTop + j]);
        }
        __syncthreads();
        if ((int)threadIdx.x < half) {
#pragma unroll
            for (int j = 0; j < kSketchTop; j++) lds[threadIdx.x * kSketchTop + j] = t[j];
        }
        __syncthreads();
    }
    if (threadIdx.x < kSketchTop) part[blockIdx.x * kSketchTop + threadIdx.x] = lds[threadIdx.x];
}

// One thread merges the nb block lists and the separately counted value.
__global__ void k_sk_final(const uint32_t *part, int nb, unsigned long long *res) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t t[kSketchTop];
#pragma unroll
    for (int j = 0; j < kSketchTop; j++) t[j] = 0;
    for (int b = 0; b < nb; b++) {
#pragma unroll
        for (int j = 0; j < kSketchTop; j++) top_insert(t, part[b * kSketchTop + j]);
    }
    const unsigned long long other = res[kSkOther];
    if (other) {
        top_insert(t, (uint32_t)other);
        res[kSkDistinct] += 1;
    }
#pragma unroll
    for (int j = 0; j < kSketchTop; j++) res[kSkTop + j] = t[j];
}

hipError_t launch_sketch(const SketchLaunch &a, hipStream_t s) {
    const uint32_t cap = a.mask + 1;
    const uint32_t ib = (std::max<uint32_t>(cap, kSketchRes) + 255) / 256;
    hipLaunchKernelGGL(k_sk_init, dim3(ib), dim3(256), 0, s, a.keys, a.cnt, cap, a.res);
    if (a.n) hipLaunchKernelGGL(k_sk_insert, dim3((a.n + 255) / 256), dim3(256), 0, s, a.col, a.sel, a.n, a.keys,
                                a.cnt, a.mask, a.res);
    const int nb = (int)std::min<uint32_t>(a.max_blocks, (cap + kSkBlock - 1) / kSkBlock);
    hipLaunchKernelGGL(k_sk_reduce, dim3(nb), dim3(kSkBlock), 0, s, a.keys, a.cnt, cap, a.part, a.res);
    hipLaunchKernelGGL(k_sk_final, dim3(1), dim3(64), 0, s, a.part, nb, a.res);
    return hipGetLastError();
}

// --------------------------------------------------------------- launchers

static inline dim3 grid2(int M, int N) { return dim3((N + kTile - 1) / kTile, (M + kTile - 1) / kTile); }

hipError_t mlp_gemm(const float *A, const float *B, const float *bias, float *C, int M, int N, int K, bool ta,
                    bool tb, bool relu, bool accumulate, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm, grid2(M, N), dim3(kTile * kTile), 0, s, A, B, bias, C, M, N, K, (int)ta, (int)tb,
                       (int)relu, (int)accumulate);
    return hipGetLastError();
}

hipError_t mlp_rows(const float *x, int B, int D, int H, const float *w, const int64_t off[6], float *y,
                    hipStream_t s) {
    // the one-workgroup kernel: small shapes, 16-byte aligned weight matrices
    const bool one = B >= 1 && B <= kScoreMaxB && D >= 1 && D <= kScoreMaxD && H >= 1 && H <= kScoreMaxH &&
                     D % 4 == 0 && H % 4 == 0 && off[0] % 4 == 0 && off[2] % 4 == 0 &&
                     ((uintptr_t)w % 16) == 0;
    if (one) {
        hipLaunchKernelGGL(k_mlp_score, dim3(1), dim3(kScoreThreads), 0, s, x, B, D, H, w, off[0], off[1], off[2],
                           off[3], off[4], off[5], y);
        return hipGetLastError();
    }
    const int block = ((H + 63) / 64) * 64;
    const size_t lds = (size_t)(D + 2 * H) * sizeof(float);
    hipLaunchKernelGGL(k_mlp_rows, dim3(B), dim3(block), lds, s, x, D, H, w, off[0], off[1], off[2], off[3], off[4],
                       off[5], y);
    return hipGetLastError();
}

hipError_t mlp_mse_grad(const float *y, const float *t, float *dy, float *sq, int B, hipStream_t s) {
    hipLaunchKernelGGL(k_mse_grad, dim3((B + 255) / 256), dim3(256), 0, s, y, t, dy, sq, B);
    return hipGetLastError();
}

hipError_t mlp_relu_back(const float *h, float *dz, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_relu_back, dim3((n + 255) / 256), dim3(256), 0, s, h, dz, n);
    return hipGetLastError();
}

hipError_t mlp_colsum(const float *dz, float *db, int B, int N, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3((N + 127) / 128), dim3(128), 0, s, dz, db, B, N);
    return hipGetLastError();
}

hipError_t mlp_sum(const float *x, int n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, s, x, n, out);
    return hipGetLastError();
}

hipError_t mlp_adam(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace fj
