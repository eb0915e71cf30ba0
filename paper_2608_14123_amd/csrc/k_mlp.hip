// K6: the learned subdomain correction -- a 3-layer MLP with BF16 weights and FP32
// accumulation, trained on the GPU.  GEMMs run on the CDNA matrix cores
// (v_mfma_f32_16x16x16bf16_1k); element-wise work (bias, ReLU and its derivative,
// MSE gradient, column sums, Adam) runs in plain kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.hpp"

namespace dgfas {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// FP32 -> BF16 with round-to-nearest-even (NaN kept quiet)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t b = __float_as_uint(f);
  if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x7fffffu)) return (uint16_t)((b >> 16) | 0x40);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ void to_bf16_kernel(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

void cast_bf16(int64_t n, const float* x, uint16_t* y, hipStream_t st) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, y);
}

// C[m][n] = sum_k A(m,k) B(k,n) (+ bias[n]) (ReLU) with A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn] in BF16, C row-major FP32 (ldc = N) and optionally a BF16 copy.
// Workgroup: 4 wavefronts, 64x64 tile, each wavefront 32x32 = 2x2 MFMA 16x16 blocks;
// K advances 32 per LDS stage.  Out-of-range rows/columns/k are zero-filled.
constexpr int GT = 64, GK = 32, GKP = GK + 8;

__global__ void __launch_bounds__(256)
gemm_bf16_kernel(int M, int N, int K, const uint16_t* __restrict__ A, int64_t sam, int64_t sak,
                 const uint16_t* __restrict__ B, int64_t sbk, int64_t sbn, float* __restrict__ C,
                 uint16_t* __restrict__ Cb, const float* __restrict__ bias, int relu, int accumulate) {
  __shared__ uint16_t As[GT][GKP];   // [m][k]
  __shared__ uint16_t Bs[GT][GKP];   // [n][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  v4f acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += GK) {
    // stage: 64x32 of A and 32x64 of B, 8 values per thread each
    for (int t = tid; t < GT * GK; t += 256) {
      const int r = t / GK, kk = t % GK;
      const int m = m0 + r, n = n0 + r, k = k0 + kk;
      As[r][kk] = (m < M && k < K) ? A[(int64_t)m * sam + (int64_t)k * sak] : (uint16_t)0;
      Bs[r][kk] = (n < N && k < K) ? B[(int64_t)k * sbk + (int64_t)n * sbn] : (uint16_t)0;
    }
    __syncthreads();
    for (int kk = 0; kk < GK; kk += 16) {
      // operand layout of the 16x16x16 bf16 MFMA: lane l holds A[l%16][4(l/16)+i], B[4(l/16)+i][l%16]
      const int kl = kk + 4 * (lane >> 4), rl = lane & 15;
      v4s fa[2], fb[2];
      for (int a = 0; a < 2; ++a)
        for (int i = 0; i < 4; ++i) fa[a][i] = (short)As[wm + 16 * a + rl][kl + i];
      for (int b = 0; b < 2; ++b)
        for (int i = 0; i < 4; ++i) fb[b][i] = (short)Bs[wn + 16 * b + rl][kl + i];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // result layout: lane l, register j holds D[4(l/16)+j][l%16]
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + wm + 16 * a + 4 * (lane >> 4) + j;
        const int n = n0 + wn + 16 * b + (lane & 15);
        if (m >= M || n >= N) continue;
        float v = acc[a][b][j];
        const int64_t o = (int64_t)m * N + n;
        if (accumulate) v += C[o];
        if (bias) v += bias[n];
        if (relu) v = v > 0.f ? v : 0.f;
        if (C) C[o] = v;
        if (Cb) Cb[o] = to_bf16(v);
      }
}

void gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
               int64_t sbn, float* C, uint16_t* Cb, const float* bias, int relu, int accumulate, hipStream_t st) {
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, Cb, bias, relu,
                     accumulate);
}

// dY = 2 (Y - T) / (rows * cols), loss partials per block
__global__ void mse_kernel(int64_t n, const float* __restrict__ Y, const float* __restrict__ T, float scale,
                           float* __restrict__ dY, uint16_t* __restrict__ dYb, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float d = Y[i] - T[i];
    s += (double)d * d;
    const float g = 2.f * scale * d;
    dY[i] = g;
    dYb[i] = to_bf16(g);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

void mse_grad(int64_t n, const float* Y, const float* T, float scale, float* dY, uint16_t* dYb, double* part,
              int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(mse_kernel, dim3(nblocks), dim3(256), 0, st, n, Y, T, scale, dY, dYb, part);
}

// dH (bf16) = G * [H > 0]  (G FP32 from the next layer's transposed GEMM)
__global__ void relu_back_kernel(int64_t n, float* __restrict__ G, const float* __restrict__ H,
                                 uint16_t* __restrict__ Gb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = H[i] > 0.f ? G[i] : 0.f;
  G[i] = g;
  Gb[i] = to_bf16(g);
}

void relu_back(int64_t n, float* G, const float* H, uint16_t* Gb, hipStream_t st) {
  hipLaunchKernelGGL(relu_back_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, G, H, Gb);
}

// out[c] = sum_r G[r][c] (bias gradient), fixed order per column
__global__ void colsum_kernel(int rows, int cols, const float* __restrict__ G, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += G[(int64_t)r * cols + c];
  out[c] = s;
}

void colsum(int rows, int cols, const float* G, float* out, hipStream_t st) {
  hipLaunchKernelGGL(colsum_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, rows, cols, G, out);
}

// Adam with bias correction; refreshes the BF16 weight copy
__global__ void adam_kernel(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, uint16_t* __restrict__ wb, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = to_bf16(wi);
}

void adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* wb, float lr, float b1, float b2,
          float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, w, g, m, v, wb, lr, b1, b2,
                     eps, c1, c2);
}

}  // namespace dgfas
