// k_mlp.h -- the warm-start network: a fully connected 6 -> 128 -> 128 -> 32
// map with GELU (z Phi(z), Phi from erff) after the two hidden layers, FP32,
// trained with a mean-squared-error loss and Adam.  Hand-written kernels:
//   k_gemm      C = P Q^T (+ bias, GELU, or times GELU'(Z)) for the three
//               products of a layer (forward X W^T, backward dZ W and dZ^T X)
//               through strides; 64 x 64 output tiles, 16 x 16 threads, each
//               thread a 4 x 4 block, the reduction staged through LDS
//   k_colsum    bias gradients (column sums, fixed order)
//   k_mse       loss partial sums (FP64) and dY = (Y - T) / B
//   k_adam      the Adam update with bias correction
// Layer sizes are tiny (at most 4096 x 128 x 128): these are latency-bound
// launches, not a contraction worth matrix cores.
#pragma once
#include <hip/hip_runtime.h>

namespace lb {

constexpr int MLP_IN = 6, MLP_H = 128, MLP_OUT = 32;
// parameter layout: W1 [H][IN], b1 [H], W2 [H][H], b2 [H], W3 [OUT][H], b3 [OUT]
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// epilogue of k_gemm
enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3 };

// C[i][j] = sum_r P[i*sPi + r*sPr] * Q[j*sQj + r*sQr], i < M, j < N, r < R.
//   EPI_BIAS:       C += bias[j]
//   EPI_BIAS_GELU:  Z = C + bias[j] stored to Zout (unless null), C = GELU(Z)
//   EPI_GELU_GRAD:  C *= GELU'(Zin[i][j])
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ P, int sPi, int sPr,
                                              const float* __restrict__ Q, int sQj, int sQr, int M, int N,
                                              int R, const float* __restrict__ bias,
                                              const float* __restrict__ Zin, float* __restrict__ Zout,
                                              float* __restrict__ C) {
  __shared__ float sp[16][64 + 1];
  __shared__ float sq[16][64 + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  float acc[4][4] = {};
  for (int r0 = 0; r0 < R; r0 += 16) {
    // stage 64 rows x 16 reduction entries of P and of Q
    // (consecutive threads walk the operand's unit-stride index)
    for (int q = threadIdx.x; q < 64 * 16; q += 256) {
      const int a = sPr == 1 ? q / 16 : q % 64, r = sPr == 1 ? q % 16 : q / 64;
      const int i = i0 + a, rr = r0 + r;
      sp[r][a] = (i < M && rr < R) ? P[(long long)i * sPi + (long long)rr * sPr] : 0.0f;
    }
    for (int q = threadIdx.x; q < 64 * 16; q += 256) {
      const int a = sQr == 1 ? q / 16 : q % 64, r = sQr == 1 ? q % 16 : q / 64;
      const int j = j0 + a, rr = r0 + r;
      sq[r][a] = (j < N && rr < R) ? Q[(long long)j * sQj + (long long)rr * sQr] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; r++) {
      float pv[4], qv[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        pv[u] = sp[r][ty * 4 + u];
        qv[u] = sq[r][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int v = 0; v < 4; v++) acc[u][v] += pv[u] * qv[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; u++)
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
      if (i >= M || j >= N) continue;
      float c = acc[u][v];
      const long long o = (long long)i * N + j;
      if (EPI == EPI_BIAS) c += bias[j];
      if (EPI == EPI_BIAS_GELU) {
        const float z = c + bias[j];
        if (Zout) Zout[o] = z;  // kept for the backward pass; a forward-only call passes null
        c = gelu(z);
      }
      if (EPI == EPI_GELU_GRAD) c *= gelu_grad(Zin[o]);
      C[o] = c;
    }
}

// out[j] = sum_i A[i][j] (rows in a fixed order)
__global__ void k_colsum(const float* __restrict__ A, int M, int N, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.0f;
  for (int i = 0; i < M; i++) s += A[(long long)i * N + j];
  out[j] = s;
}

// dY = (Y - T) / B and per-block partial sums of (Y - T)^2 in FP64
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             long long n, float invB, float* __restrict__ dY,
                                             double* __restrict__ part) {
  __shared__ double sh[4];
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  double e2 = 0.0;
  if (k < n) {
    const float e = Y[k] - T[k];
    dY[k] = e * invB;
    e2 = (double)e * (double)e;
  }
  for (int o = 32; o > 0; o >>= 1) e2 += __shfl_down(e2, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Adam with bias correction: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

}  // namespace lb
