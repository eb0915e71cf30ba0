// K6: the learned subdomain correction -- a 3-layer MLP with BF16 weights and FP32
// accumulation, trained on the GPU.  GEMMs run on the CDNA matrix cores
// (v_mfma_f32_16x16x16bf16_1k); element-wise work (bias, ReLU and its derivative,
// MSE gradient, column sums, Adam) runs in plain kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

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
// Split K: with P set, slice z = blockIdx.z takes k in [z kper, (z + 1) kper) and writes its
// raw sum to P[z][m][n]; splitk_reduce adds the slices in order and applies the epilogue, so
// the result does not depend on scheduling.
constexpr int GT = 64, GK = 32, GKP = GK + 8;

// Stage S[r][kk] = X(r0 + r, k0 + kk) with X(r, k) = X[r sr + k sk] for the 64 x 32 tile, zero
// outside R x K; with `ones`, row R is a row of ones (1.0 in BF16 is 0x3f80) for k < K.  When
// one dimension is contiguous and 8-byte aligned, every thread loads runs of four BF16 values
// with one 8-byte load: along k (one 8-byte LDS store) or along r (four transposed LDS
// stores); otherwise, and at the ragged edges, one value per load.
__device__ __forceinline__ void stage_tile(uint16_t (*S)[GKP], const uint16_t* __restrict__ X, int R, int K, int r0,
                                           int k0, int64_t sr, int64_t sk, int mode, int tid, int ones) {
  const int Rone = ones ? R : -1;
  if (mode == 1) {            // contiguous along k
    for (int g = tid; g < GT * GK / 4; g += 256) {
      const int r = g / (GK / 4), kq = (g % (GK / 4)) * 4;
      const int rr = r0 + r, k = k0 + kq;
      uint2 v = make_uint2(0u, 0u);
      if (rr < R && k + 4 <= K) {
        v = *reinterpret_cast<const uint2*>(X + (int64_t)rr * sr + k);
      } else if (rr < R) {
        uint16_t t[4];
        for (int i = 0; i < 4; ++i) t[i] = k + i < K ? X[(int64_t)rr * sr + k + i] : (uint16_t)0;
        v = make_uint2((uint32_t)t[0] | ((uint32_t)t[1] << 16), (uint32_t)t[2] | ((uint32_t)t[3] << 16));
      } else if (rr == Rone) {
        uint16_t t[4];
        for (int i = 0; i < 4; ++i) t[i] = k + i < K ? (uint16_t)0x3f80 : (uint16_t)0;
        v = make_uint2((uint32_t)t[0] | ((uint32_t)t[1] << 16), (uint32_t)t[2] | ((uint32_t)t[3] << 16));
      }
      *reinterpret_cast<uint2*>(&S[r][kq]) = v;
    }
  } else if (mode == 2) {     // contiguous along r
    for (int g = tid; g < GT * GK / 4; g += 256) {
      const int kk = g / (GT / 4), rq = (g % (GT / 4)) * 4;
      const int k = k0 + kk, rr = r0 + rq;
      uint16_t t[4] = {0, 0, 0, 0};
      if (k < K && rr + 4 <= R) {
        const uint2 v = *reinterpret_cast<const uint2*>(X + (int64_t)k * sk + rr);
        t[0] = (uint16_t)(v.x & 0xffffu); t[1] = (uint16_t)(v.x >> 16);
        t[2] = (uint16_t)(v.y & 0xffffu); t[3] = (uint16_t)(v.y >> 16);
      } else if (k < K) {
        for (int i = 0; i < 4; ++i)
          t[i] = rr + i < R ? X[(int64_t)k * sk + rr + i] : (rr + i == Rone ? (uint16_t)0x3f80 : (uint16_t)0);
      }
      for (int i = 0; i < 4; ++i) S[rq + i][kk] = t[i];
    }
  } else {
    for (int t = tid; t < GT * GK; t += 256) {
      const int r = t / GK, kk = t % GK;
      const int rr = r0 + r, k = k0 + kk;
      S[r][kk] = k >= K ? (uint16_t)0
                 : rr < R ? X[(int64_t)rr * sr + (int64_t)k * sk] : (rr == Rone ? (uint16_t)0x3f80 : (uint16_t)0);
    }
  }
}

// staging mode of an operand: 1 contiguous along k, 2 contiguous along r, 0 general
inline int stage_mode(const uint16_t* X, int64_t sr, int64_t sk) {
  const bool al = (reinterpret_cast<uintptr_t>(X) % 8) == 0;
  if (al && sk == 1 && sr % 4 == 0) return 1;
  if (al && sr == 1 && sk % 4 == 0) return 2;
  return 0;
}

__global__ void __launch_bounds__(256)
gemm_bf16_kernel(int M, int N, int K, const uint16_t* __restrict__ A, int64_t sam, int64_t sak,
                 const uint16_t* __restrict__ B, int64_t sbk, int64_t sbn, float* __restrict__ C,
                 uint16_t* __restrict__ Cb, const float* __restrict__ bias, int relu, int accumulate, int amode,
                 int bmode, int kper, float* __restrict__ P, int ones) {
  __shared__ __align__(16) uint16_t As[GT][GKP];   // [m][k]; rows of 80 bytes keep 8-byte stores aligned
  __shared__ __align__(16) uint16_t Bs[GT][GKP];   // [n][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  v4f acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  const int kb = P ? blockIdx.z * kper : 0;
  const int ke = P ? min(K, kb + kper) : K;
  for (int k0 = kb; k0 < ke; k0 += GK) {
    // stage: 64x32 of A and 32x64 of B (as [n][k]); a slice ends on a multiple of GK, so the
    // zero fill at K is the only ragged edge
    stage_tile(As, A, M - ones, K, m0, k0, sam, sak, amode, tid, ones);
    stage_tile(Bs, B, N, K, n0, k0, sbn, sbk, bmode, tid, 0);
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
        if (P) {
          P[(int64_t)blockIdx.z * M * N + o] = v;
          continue;
        }
        if (accumulate) v += C[o];
        if (bias) v += bias[n];
        if (relu) v = v > 0.f ? v : 0.f;
        if (C) C[o] = v;
        if (Cb) Cb[o] = to_bf16(v);
      }
}

__global__ void splitk_reduce_kernel(int64_t mn, int N, int splits, const float* __restrict__ P, float* __restrict__ C,
                                     uint16_t* __restrict__ Cb, const float* __restrict__ bias, int relu,
                                     int accumulate) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= mn) return;
  float v = 0.f;
  for (int z = 0; z < splits; ++z) v += P[(int64_t)z * mn + o];
  if (accumulate) v += C[o];
  if (bias) v += bias[o % N];
  if (relu) v = v > 0.f ? v : 0.f;
  if (C) C[o] = v;
  if (Cb) Cb[o] = to_bf16(v);
}

int gemm_splits(int M, int N, int K, int64_t ws_cap) {
  const int64_t tiles = (int64_t)((N + GT - 1) / GT) * ((M + GT - 1) / GT);
  // fewer tiles than about two per CU and a long K: cut K into slices of at least 256
  if (tiles >= 512 || K < 512) return 1;
  int64_t s = std::min<int64_t>((1024 + tiles - 1) / tiles, K / 256);
  s = std::min<int64_t>(s, ws_cap / ((int64_t)M * N));
  return (int)std::max<int64_t>(1, s);
}

void gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
               int64_t sbn, float* C, uint16_t* Cb, const float* bias, int relu, int accumulate, hipStream_t st,
               float* ws, int64_t ws_cap, int ones) {
  int splits = ws ? gemm_splits(M, N, K, ws_cap) : 1;
  int kper = K;
  if (splits > 1) {
    kper = ((K + splits - 1) / splits + GK - 1) / GK * GK;
    splits = (K + kper - 1) / kper;
  }
  const int am = stage_mode(A, sam, sak), bm = stage_mode(B, sbn, sbk);
  if (splits <= 1) {
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, Cb, bias,
                       relu, accumulate, am, bm, K, (float*)nullptr, ones);
    return;
  }
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, splits);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, Cb, bias, relu,
                     accumulate, am, bm, kper, ws, ones);
  const int64_t mn = (int64_t)M * N;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, st, mn, N, splits, ws, C,
                     Cb, bias, relu, accumulate);
}

// dY = 2 (Y - T) / (rows * cols) as BF16 rows of pitch ldb (the padding columns are left
// alone), loss partials per block
__global__ void mse_kernel(int64_t n, int cols, int ldb, const float* __restrict__ Y, const float* __restrict__ T,
                           float scale, uint16_t* __restrict__ dYb, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float d = Y[i] - T[i];
    s += (double)d * d;
    const int64_t r = i / cols;
    dYb[r * ldb + (i - r * cols)] = to_bf16(2.f * scale * d);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

void mse_grad(int64_t n, int cols, int ldb, const float* Y, const float* T, float scale, uint16_t* dYb, double* part,
              int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(mse_kernel, dim3(nblocks), dim3(256), 0, st, n, cols, ldb, Y, T, scale, dYb, part);
}

// dst[r][c] = src[r][c] for c < cols, 0 for cols <= c < ldd (a row-padded BF16 copy)
__global__ void pad_rows_kernel(int rows, int cols, int ldd, const uint16_t* __restrict__ src,
                                uint16_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * ldd) return;
  const int64_t r = i / ldd;
  const int c = (int)(i - r * ldd);
  dst[i] = c < cols ? src[r * cols + c] : (uint16_t)0;
}

void pad_rows(int rows, int cols, int ldd, const uint16_t* src, uint16_t* dst, hipStream_t st) {
  const int64_t n = (int64_t)rows * ldd;
  hipLaunchKernelGGL(pad_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rows, cols, ldd, src, dst);
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
