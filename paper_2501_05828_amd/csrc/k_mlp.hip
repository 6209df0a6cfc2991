// Learned emission proposal on gfx950: a 34-64-64-64-1024 MLP with a softmax
// over the 32x32 equal-area direction cells, one row per (transmit,
// element).  It supplies the direction pdf p_t of the emission estimator
// (Eq. 4); uniform emission stays the fallback and the defensive mixture
// component.  Matrix products run on BF16 MFMA (operands rounded to nearest
// even BF16, FP32 accumulation); master weights, Adam state, softmax and
// loss are FP32.
#include <algorithm>

#include "philox.h"
#include "ur_internal.h"

namespace {
using namespace ur;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even (finite inputs)
    return (short)(u >> 16);
}

// C[M][N] = A[M][K] B[K][N] (+ bias[N]), then ReLU or a ReLU-derivative mask.
// A(i, k) = A[i * sar + k * sac], B(k, j) = B[k * sbr + j * sbc] (strides
// express transposes); C row-major.  A 256-thread block computes a 64x64
// tile; each wavefront owns a 32x32 quarter as 2x2 MFMA 16x16x16 tiles.
// Per K step of 16 the block stages BF16 tiles of A (64x16) and B (16x64)
// in LDS.  MFMA 16x16x16 lane layout: A row = lane % 16 and K = 4 (lane / 16)
// + j; B column = lane % 16, same K; result row = 4 (lane / 16) + j,
// column = lane % 16.
struct Gemm {
    const float *A;
    int64_t sar, sac;
    const float *B;
    int64_t sbr, sbc;
    float *C;
    int M, N, K;
    const float *bias;   // [N] or null
    const float *mask;   // [M][N] or null: C = mask > 0 ? C : 0
    int relu;
};

__global__ __launch_bounds__(256) void k_gemm_bf16(Gemm g) {
    __shared__ short As[64][16 + 4];
    __shared__ short Bs[16][64 + 4];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        for (int e = tid; e < 64 * 16; e += 256) {
            const int i = e >> 4, k = e & 15, gi = m0 + i, gk = k0 + k;
            const float v = (gi < g.M && gk < g.K) ? g.A[(int64_t)gi * g.sar + (int64_t)gk * g.sac] : 0.f;
            As[i][k] = to_bf16(v);
        }
        for (int e = tid; e < 16 * 64; e += 256) {
            const int k = e >> 6, j = e & 63, gk = k0 + k, gj = n0 + j;
            const float v = (gk < g.K && gj < g.N) ? g.B[(int64_t)gk * g.sbr + (int64_t)gj * g.sbc] : 0.f;
            Bs[k][j] = to_bf16(v);
        }
        __syncthreads();
        const int kk = (lane >> 4) * 4;
        for (int a = 0; a < 2; ++a) {
            const int r = wm + a * 16 + (lane & 15);
            const bf16x4 av = {As[r][kk], As[r][kk + 1], As[r][kk + 2], As[r][kk + 3]};
            for (int b = 0; b < 2; ++b) {
                const int c = wn + b * 16 + (lane & 15);
                const bf16x4 bv = {Bs[kk][c], Bs[kk + 1][c], Bs[kk + 2][c], Bs[kk + 3][c]};
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[a][b], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int j = 0; j < 4; ++j) {
                const int i = m0 + wm + a * 16 + (lane >> 4) * 4 + j;
                const int c = n0 + wn + b * 16 + (lane & 15);
                if (i >= g.M || c >= g.N) continue;
                float v = acc[a][b][j];
                if (g.bias) v += g.bias[c];
                if (g.relu) v = fmaxf(v, 0.f);
                if (g.mask && !(g.mask[(int64_t)i * g.N + c] > 0.f)) v = 0.f;
                g.C[(int64_t)i * g.N + c] = v;
            }
}

// Input rows: normalised element position and steering angle and their
// random Fourier encoding, computed in FP64 and stored as FP32.
__global__ void k_features(const double *xe, const double *angles, int E, int T, double half_ap, double amax,
                           const float *rff, float *X) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= E * T) return;
    const int e = r % E, tx = r / E;
    const double xn = xe[e] / half_ap, tn = angles[tx] / amax;
    float *x = X + (int64_t)r * 34;
    x[0] = (float)xn;
    x[1] = (float)tn;
    for (int i = 0; i < 16; ++i) {
        const double p = 2.0 * M_PI * ((double)rff[2 * i] * xn + (double)rff[2 * i + 1] * tn);
        x[2 + i] = (float)sin(p);
        x[18 + i] = (float)cos(p);
    }
}

__device__ __forceinline__ float block_reduce(float v, float *red, bool is_max) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = is_max ? fmaxf(red[tid], red[tid + s]) : red[tid] + red[tid + s];
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

// Softmax over the 1024 cells of each row and the weighted cross-entropy
// -sum H log q / sum H; dZ = (q sum_c H - H) / sum H.  One block per row.
__global__ __launch_bounds__(256) void k_softmax_ce(const float *Z, const float *H, const float *tot, float *Q,
                                                    float *dZ, float *loss) {
    __shared__ float red[256];
    const int64_t r = blockIdx.x;
    const float *z = Z + r * 1024;
    float zv[4], mx = -INFINITY;
    for (int j = 0; j < 4; ++j) {
        zv[j] = z[threadIdx.x + 256 * j];
        mx = fmaxf(mx, zv[j]);
    }
    mx = block_reduce(mx, red, true);
    float s = 0.f, hs = 0.f;
    for (int j = 0; j < 4; ++j) {
        s += expf(zv[j] - mx);
        if (H) hs += H[r * 1024 + threadIdx.x + 256 * j];
    }
    s = block_reduce(s, red, false);
    if (H) hs = block_reduce(hs, red, false);
    const float lse = logf(s);
    const float inv_tot = H ? 1.0f / *tot : 0.f;
    float part = 0.f;
    for (int j = 0; j < 4; ++j) {
        const int c = threadIdx.x + 256 * j;
        const float lq = zv[j] - mx - lse, q = expf(lq);
        if (Q) Q[r * 1024 + c] = q;
        if (H) {
            const float h = H[r * 1024 + c];
            dZ[r * 1024 + c] = (q * hs - h) * inv_tot;
            part -= h * lq;
        }
    }
    if (H && loss) {
        part = block_reduce(part, red, false);
        if (threadIdx.x == 0) atomicAdd(loss, part * inv_tot);
    }
}

// out[j] = sum_i X[i][j] (bias gradients); one lane per column.
__global__ void k_colsum(const float *X, int R, int N, float *out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int i = 0; i < R; ++i) s += X[(int64_t)i * N + j];
    out[j] = s;
}

// Sum of n floats by one block in a fixed order (each thread a fixed stride,
// then a fixed tree), so the total is the same bits on every call: it
// normalises every gradient of the training step, and a float atomic across
// blocks would round in arrival order.
constexpr int kSumThreads = 1024;
__global__ __launch_bounds__(kSumThreads) void k_sum(const float *x, int64_t n, float *out) {
    __shared__ float red[kSumThreads];
    float s = 0.f;
#pragma unroll 8
    for (int64_t i = threadIdx.x; i < n; i += kSumThreads) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = kSumThreads / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_fill(float *p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Adam (Kingma & Ba) with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void k_adam(float *w, float *m, float *v, const float *g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Defensive mixture q' = (1 - eps) q + eps / 1024 and its inclusive prefix
// sum per row (sequential within a row, so the table is deterministic).
__global__ void k_tables(const float *Q, int R, float eps, float *pdf, float *cdf) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    float acc = 0.f;
    for (int c = 0; c < 1024; ++c) {
        const float p = (1.f - eps) * Q[(int64_t)r * 1024 + c] + eps / 1024.f;
        pdf[(int64_t)r * 1024 + c] = p;
        acc += p;
        cdf[(int64_t)r * 1024 + c] = acc;
    }
}

// Minibatch histogram: `batch` records drawn uniformly (with replacement,
// Philox-indexed) from the recorded contributions, each adding |c| to its
// (row, cell) bin.
__global__ void k_record_hist(const RecordEntry *rec, int64_t n_rec, int64_t batch, uint32_t k0, uint32_t k1,
                              uint32_t step, int64_t n_bins, float *hist) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < batch; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t x4[4];
        philox4x32_10((uint32_t)i, step, 0u, 0u, k0, k1, x4);
        const uint32_t x = x4[0];
        const int64_t j = (int64_t)(((uint64_t)x * (uint64_t)n_rec) >> 32);
        const RecordEntry e = rec[j];
        if ((int64_t)e.bin < n_bins) atomicAdd(hist + e.bin, e.value);
    }
}

// Second moment of the recorded contributions per bin.
__global__ void k_record_s2(const RecordEntry *rec, int64_t n_rec, int64_t n_bins, float *s2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_rec; i += (int64_t)gridDim.x * blockDim.x) {
        const RecordEntry e = rec[i];
        if ((int64_t)e.bin < n_bins) atomicAdd(s2 + e.bin, e.value * e.value);
    }
}

// value := c^2 / sqrt(S2 * mean cost): summed over a bin this gives
// sqrt(S2 / mean cost), the density that minimises variance x time.
__global__ void k_record_weight(RecordEntry *rec, int64_t n_rec, int64_t n_bins, const float *s2, const float *cost,
                                float inv_rays_per_cell) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_rec; i += (int64_t)gridDim.x * blockDim.x) {
        RecordEntry e = rec[i];
        if ((int64_t)e.bin >= n_bins) continue;
        const float mc = fmaxf(cost[e.bin] * inv_rays_per_cell, 1.0f);
        const float q = s2[e.bin];
        e.value = q > 0.f ? e.value * e.value / sqrtf(q * mc) : 0.f;
        rec[i] = e;
    }
}

dim3 blocks_for(int64_t n, int per = 256) { return dim3((unsigned)std::min<int64_t>((n + per - 1) / per, 4096)); }

}  // namespace

hipError_t ur_mlp_gemm(const float *A, int64_t sar, int64_t sac, const float *B, int64_t sbr, int64_t sbc, float *C,
                       int M, int N, int K, const float *bias, const float *mask, int relu, hipStream_t s) {
    Gemm g{A, sar, sac, B, sbr, sbc, C, M, N, K, bias, mask, relu};
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t ur_mlp_features(const double *xe, const double *angles, int E, int T, double half_ap, double amax,
                           const float *rff, float *X, hipStream_t s) {
    hipLaunchKernelGGL(k_features, dim3((unsigned)((E * T + 127) / 128)), dim3(128), 0, s, xe, angles, E, T, half_ap,
                       amax, rff, X);
    return hipGetLastError();
}

hipError_t ur_mlp_softmax_ce(const float *Z, const float *H, const float *tot, float *Q, float *dZ, float *loss,
                             int R, hipStream_t s) {
    hipLaunchKernelGGL(k_softmax_ce, dim3((unsigned)R), dim3(256), 0, s, Z, H, tot, Q, dZ, loss);
    return hipGetLastError();
}

hipError_t ur_mlp_colsum(const float *X, int R, int N, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, X, R, N, out);
    return hipGetLastError();
}

hipError_t ur_mlp_sum(const float *x, int64_t n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kSumThreads), 0, s, x, n, out);
    return hipGetLastError();
}

hipError_t ur_mlp_fill(float *p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, blocks_for(n), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t ur_mlp_adam(float *w, float *m, float *v, const float *g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, m, v, g, n, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

hipError_t ur_mlp_tables(const float *Q, int R, float eps, float *pdf, float *cdf, hipStream_t s) {
    hipLaunchKernelGGL(k_tables, dim3((unsigned)((R + 63) / 64)), dim3(64), 0, s, Q, R, eps, pdf, cdf);
    return hipGetLastError();
}

hipError_t ur_mlp_record_hist(const ur::RecordEntry *rec, int64_t n_rec, int64_t batch, uint64_t seed, uint32_t step,
                              int64_t n_bins, float *hist, hipStream_t s) {
    hipError_t e = ur_mlp_fill(hist, n_bins, 0.f, s);
    if (e != hipSuccess || n_rec <= 0 || batch <= 0) return e;
    hipLaunchKernelGGL(k_record_hist, blocks_for(batch), dim3(256), 0, s, rec, n_rec, batch, (uint32_t)seed,
                       (uint32_t)(seed >> 32), step, n_bins, hist);
    return hipGetLastError();
}

hipError_t ur_mlp_record_reweight(ur::RecordEntry *rec, int64_t n_rec, const float *cost, double rays_per_row,
                                  float *s2, int64_t n_bins, hipStream_t s) {
    hipError_t e = ur_mlp_fill(s2, n_bins, 0.f, s);
    if (e != hipSuccess || n_rec <= 0) return e;
    hipLaunchKernelGGL(k_record_s2, blocks_for(n_rec), dim3(256), 0, s, rec, n_rec, n_bins, s2);
    hipLaunchKernelGGL(k_record_weight, blocks_for(n_rec), dim3(256), 0, s, rec, n_rec, n_bins, s2, cost,
                       (float)((double)ur::kCells / rays_per_row));
    return hipGetLastError();
}
