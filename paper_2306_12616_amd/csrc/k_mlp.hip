// Learned chemical potential: the small network 64 -> 256 -> 256 -> 1 (ReLU,
// float32) that maps Chebyshev trace moments to mu~, trained on the GPU with
// these kernels.  Everything is a handful of small dense products plus
// element-wise passes, so one general tiled SIMT product kernel (64 x 64
// output tiles, 4 x 4 per thread, K staged through LDS, fixed summation
// order: deterministic) carries forward and backward, with fused epilogues
// for bias + ReLU, bias only, and the ReLU mask of the backward pass.
#include "internal.h"
#include "reduce.h"

namespace chebdm {

namespace {

constexpr int TM = 64, TN = 64, TK = 16;

// C[i][j] = epi( sum_k A(i,k) B(k,j) ),  A(i,k) = transA ? A[k*lda+i] : A[i*lda+k],
// B(k,j) = transB ? B[j*ldb+k] : B[k*ldb+j].
// epi: 0 none, 1 relu(x + bias[j]), 2 x + bias[j], 3 x * (mask[i*ldc+j] > 0)
__global__ void __launch_bounds__(256)
k_mlp_gemm(int M, int N, int K, const float* __restrict__ A, int lda, int transA, const float* __restrict__ B,
           int ldb, int transB, float* __restrict__ C, int ldc, int epi, const float* __restrict__ bias,
           const float* __restrict__ mask) {
    __shared__ float As[TK][TM + 4];
    __shared__ float Bs[TK][TN + 4];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += TK) {
        for (int e = threadIdx.x; e < TK * TM; e += 256) {
            const int kk = e / TM, ii = e % TM;
            const int gi = i0 + ii, gk = k0 + kk;
            float v = 0.0f;
            if (gi < M && gk < K) v = transA ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk];
            As[kk][ii] = v;
        }
        for (int e = threadIdx.x; e < TK * TN; e += 256) {
            const int kk = e / TN, jj = e % TN;
            const int gj = j0 + jj, gk = k0 + kk;
            float v = 0.0f;
            if (gj < N && gk < K) v = transB ? B[(size_t)gj * ldb + gk] : B[(size_t)gk * ldb + gj];
            Bs[kk][jj] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = i0 + ty + 16 * r, j = j0 + tx + 16 * c;
            if (i >= M || j >= N) continue;
            float v = acc[r][c];
            if (epi == 1) v = fmaxf(v + bias[j], 0.0f);
            else if (epi == 2) v = v + bias[j];
            else if (epi == 3) v = mask[(size_t)i * ldc + j] > 0.0f ? v : 0.0f;
            C[(size_t)i * ldc + j] = v;
        }
}

// out[j] = sum_i A[i][j] (fixed order)
__global__ void __launch_bounds__(256) k_mlp_colsum(int M, int N, const float* __restrict__ A, float* __restrict__ out) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    float s = 0.0f;
    for (int i = 0; i < M; ++i) s += A[(size_t)i * N + j];
    out[j] = s;
}

// dy = 2 (y - t) / B, loss = mean (y - t)^2 (one work-group)
__global__ void __launch_bounds__(256)
k_mlp_loss(int Bn, const float* __restrict__ y, const float* __restrict__ t, float* __restrict__ dy,
           float* __restrict__ loss) {
    __shared__ double smem[4];
    double acc = 0.0;
    for (int b = threadIdx.x; b < Bn; b += 256) {
        const float r = y[b] - t[b];
        dy[b] = 2.0f * r / (float)Bn;
        acc += (double)r * (double)r;
    }
    acc = block_sum<256>(acc, smem);
    if (threadIdx.x == 0) *loss = (float)(acc / Bn);
}

// dZ2[b][o] = dy[b] w3[o] (A2[b][o] > 0)
__global__ void __launch_bounds__(256)
k_mlp_outer_mask(int Bn, int H, const float* __restrict__ dy, const float* __restrict__ w3,
                 const float* __restrict__ A2, float* __restrict__ dZ) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= Bn * H) return;
    const int b = idx / H, o = idx % H;
    dZ[idx] = A2[idx] > 0.0f ? dy[b] * w3[o] : 0.0f;
}

__global__ void __launch_bounds__(256)
k_mlp_adam(int n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
           float lr, float b1, float b2, float eps, float bc1, float bc2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

hipError_t gemm(hipStream_t st, int M, int N, int K, const float* A, int lda, int tA, const float* B, int ldb, int tB,
                float* C, int ldc, int epi, const float* bias, const float* mask) {
    dim3 grid((unsigned)((N + TN - 1) / TN), (unsigned)((M + TM - 1) / TM));
    hipLaunchKernelGGL(k_mlp_gemm, grid, dim3(256), 0, st, M, N, K, A, lda, tA, B, ldb, tB, C, ldc, epi, bias, mask);
    return hipGetLastError();
}

}  // namespace

// parameter offsets (floats)
constexpr int MLP_IN = 64, MLP_H = 256;
constexpr int64_t OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_H * MLP_IN, OFF_W2 = OFF_B1 + MLP_H,
                  OFF_B2 = OFF_W2 + MLP_H * MLP_H, OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_H,
                  MLP_NPARAM = OFF_B3 + 1;

int64_t mlp_nparams() { return MLP_NPARAM; }

// work: A1 (B x 256), A2 (B x 256) and, for backward, dZ2 (B x 256), dZ1 (B x 256), dy (B), loss (1)
hipError_t launch_mlp_forward(const float* w, const float* X, int Bn, float* y, float* work, hipStream_t st) {
    float* A1 = work;
    float* A2 = A1 + (size_t)Bn * MLP_H;
    hipError_t e;
    if ((e = gemm(st, Bn, MLP_H, MLP_IN, X, MLP_IN, 0, w + OFF_W1, MLP_IN, 1, A1, MLP_H, 1, w + OFF_B1, nullptr)))
        return e;
    if ((e = gemm(st, Bn, MLP_H, MLP_H, A1, MLP_H, 0, w + OFF_W2, MLP_H, 1, A2, MLP_H, 1, w + OFF_B2, nullptr)))
        return e;
    return gemm(st, Bn, 1, MLP_H, A2, MLP_H, 0, w + OFF_W3, 1, 0, y, 1, 2, w + OFF_B3, nullptr);
}

hipError_t launch_mlp_backward(const float* w, const float* X, const float* t, int Bn, float* g, float* work,
                               float* loss, hipStream_t st) {
    float* A1 = work;
    float* A2 = A1 + (size_t)Bn * MLP_H;
    float* dZ2 = A2 + (size_t)Bn * MLP_H;
    float* dZ1 = dZ2 + (size_t)Bn * MLP_H;
    float* y = dZ1 + (size_t)Bn * MLP_H;
    float* dy = y + Bn;
    hipError_t e;
    if ((e = launch_mlp_forward(w, X, Bn, y, work, st))) return e;
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, Bn, (const float*)y, t, dy, loss);
    // output layer
    if ((e = gemm(st, MLP_H, 1, Bn, A2, MLP_H, 1, dy, 1, 0, g + OFF_W3, 1, 0, nullptr, nullptr))) return e;
    hipLaunchKernelGGL(k_mlp_colsum, dim3(1), dim3(256), 0, st, Bn, 1, (const float*)dy, g + OFF_B3);
    // second hidden layer
    hipLaunchKernelGGL(k_mlp_outer_mask, dim3((unsigned)((Bn * MLP_H + 255) / 256)), dim3(256), 0, st, Bn, MLP_H,
                       (const float*)dy, w + OFF_W3, (const float*)A2, dZ2);
    if ((e = gemm(st, MLP_H, MLP_H, Bn, dZ2, MLP_H, 1, A1, MLP_H, 0, g + OFF_W2, MLP_H, 0, nullptr, nullptr))) return e;
    hipLaunchKernelGGL(k_mlp_colsum, dim3(1), dim3(256), 0, st, Bn, MLP_H, (const float*)dZ2, g + OFF_B2);
    // first hidden layer: dZ1 = (dZ2 W2) * (A1 > 0)
    if ((e = gemm(st, Bn, MLP_H, MLP_H, dZ2, MLP_H, 0, w + OFF_W2, MLP_H, 0, dZ1, MLP_H, 3, nullptr, A1))) return e;
    if ((e = gemm(st, MLP_H, MLP_IN, Bn, dZ1, MLP_H, 1, X, MLP_IN, 0, g + OFF_W1, MLP_IN, 0, nullptr, nullptr)))
        return e;
    hipLaunchKernelGGL(k_mlp_colsum, dim3(1), dim3(256), 0, st, Bn, MLP_H, (const float*)dZ1, g + OFF_B1);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                           float eps, float bc1, float bc2, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (int)n, w, g, m, v, lr, b1,
                       b2, eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace chebdm
