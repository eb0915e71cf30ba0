// K3: per-element tensor-product transfers between p-levels (Sec. 3.2):
//   out (=|+=) (T x T x T)(in - in2),  T: n_out x n_in,
// used for P (projection), R = I^T (restriction) and I (prolongation).
// K4: BLAS-1 pieces of SCG (Alg. 6) with fixed-shape two-stage reductions, so
// every dot product is bitwise reproducible.
#include "device.hpp"
#include "kernels.hpp"
#include "blas.hpp"

namespace dgfas {

// one thread per output of the wider of the first two contraction steps (the inputs and the
// last step's outputs are taken in loops), so that neither a restriction nor a prolongation
// idles most of a workgroup sized for its largest array
template <int NI, int NO>
struct TrShape {
  static constexpr int W1 = NI * NI * NO, W2 = NI * NO * NO, W3 = NO * NO * NO;
  static constexpr int M3 = W1 > W2 ? W1 : W2;
  static constexpr int EPB = (M3 >= 256) ? 1 : (256 / M3);
  static constexpr int THREADS = ((EPB * M3 + 63) / 64) * 64;
};

// Element e of the launch list, sub-block s = rhs * ncomp + comp:
//   in  + rhs * stride_in  + off_in[e]  * ncomp + comp * NI^3
//   out + rhs * stride_out + off_out[e] * ncomp + comp * NO^3
template <int NI, int NO, typename T>
__global__ void __launch_bounds__((TrShape<NI, NO>::THREADS))
tensor3_kernel(XferArgs<T> a) {
  using S = TrShape<NI, NO>;
  constexpr int M3 = S::M3, EPB = S::EPB, I3 = NI * NI * NI, O3 = NO * NO * NO;
  const int nsub = a.nrhs * a.ncomp;
  const int lbs = xcd_block(((a.nel + EPB - 1) / EPB) * nsub);
  if (lbs < 0) return;
  const int lb = lbs / nsub, sub = lbs - lb * nsub;
  const int rhs = sub / a.ncomp, comp = sub - rhs * a.ncomp;
  const int tid = threadIdx.x;
  const int le = tid / M3, q = tid - le * M3;
  const int li = lb * EPB + le;
  const bool act = le < EPB && li < a.nel;
  const int e = act ? (a.elist ? a.elist[li] : li) : 0;
  const int64_t ib = (int64_t)rhs * a.stride_in + (a.off_in ? a.off_in[e] : (int64_t)e * I3) * a.ncomp +
                     (int64_t)comp * I3;
  const int64_t ob = (int64_t)rhs * a.stride_out + (a.off_out ? a.off_out[e] : (int64_t)e * O3) * a.ncomp +
                     (int64_t)comp * O3;
  __shared__ T sT[NO * NI];
  __shared__ T s0[EPB][NI * NI * NI];
  __shared__ T s1[EPB][NI * NI * NO];
  __shared__ T s2[EPB][NI * NO * NO];
  for (int t = tid; t < NO * NI; t += S::THREADS) sT[t] = a.Tm[t];
  if (act) {
    for (int t = q; t < I3; t += M3) {
      T v = a.in[ib + t];
      if (a.in2) v -= a.in2[ib + t];
      s0[le][t] = v;
    }
  }
  __syncthreads();
  if (act && q < NI * NI * NO) {   // [k][j][a]
    const int x = q % NO, j = (q / NO) % NI, k = q / (NO * NI);
    T s = 0;
    for (int i = 0; i < NI; ++i) s += sT[x * NI + i] * s0[le][(k * NI + j) * NI + i];
    s1[le][q] = s;
  }
  __syncthreads();
  if (act && q < NI * NO * NO) {   // [k][b][a]
    const int x = q % NO, y = (q / NO) % NO, k = q / (NO * NO);
    T s = 0;
    for (int j = 0; j < NI; ++j) s += sT[y * NI + j] * s1[le][(k * NI + j) * NO + x];
    s2[le][q] = s;
  }
  __syncthreads();
  for (int qq = q; act && qq < O3; qq += M3) {   // [c][b][a]
    const int x = qq % NO, y = (qq / NO) % NO, c = qq / (NO * NO);
    T s = 0;
    for (int k = 0; k < NI; ++k) s += sT[c * NI + k] * s2[le][(k * NO + y) * NO + x];
    const int64_t o = ob + qq;
    a.out[o] = a.accumulate ? a.out[o] + s : s;
  }
}

template <int NI, int NO, typename T>
void launch_t3(const XferArgs<T>& a, hipStream_t st) {
  using S = TrShape<NI, NO>;
  const int nb = ((a.nel + S::EPB - 1) / S::EPB) * a.nrhs * a.ncomp;
  hipLaunchKernelGGL((tensor3_kernel<NI, NO, T>), dim3(xcd_grid(nb)), dim3(S::THREADS), 0, st, a);
}

template <typename T>
bool tensor3(int n_in, int n_out, const XferArgs<T>& a, hipStream_t st) {
  if (a.nel <= 0) return true;
#define T3C(x, y) \
  if (n_in == x && n_out == y) { launch_t3<x, y, T>(a, st); return true; }
  // p-coarsening pairs (p_c = max(1, p_f / 2)), identity-degree copies and the
  // interpolations between any two degrees 1..8 used on mixed-degree meshes
  T3C(2, 2) T3C(2, 3) T3C(2, 4) T3C(2, 5) T3C(2, 6) T3C(2, 7) T3C(2, 8) T3C(2, 9)
  T3C(3, 2) T3C(3, 3) T3C(3, 4) T3C(3, 5) T3C(3, 6) T3C(3, 7) T3C(3, 8) T3C(3, 9)
  T3C(4, 2) T3C(4, 3) T3C(4, 4) T3C(4, 5) T3C(4, 6) T3C(4, 7) T3C(4, 8) T3C(4, 9)
  T3C(5, 2) T3C(5, 3) T3C(5, 4) T3C(5, 5) T3C(5, 6) T3C(5, 7) T3C(5, 8) T3C(5, 9)
  T3C(6, 2) T3C(6, 3) T3C(6, 4) T3C(6, 5) T3C(6, 6) T3C(6, 7) T3C(6, 8) T3C(6, 9)
  T3C(7, 2) T3C(7, 3) T3C(7, 4) T3C(7, 5) T3C(7, 6) T3C(7, 7) T3C(7, 8) T3C(7, 9)
  T3C(8, 2) T3C(8, 3) T3C(8, 4) T3C(8, 5) T3C(8, 6) T3C(8, 7) T3C(8, 8) T3C(8, 9)
  T3C(9, 2) T3C(9, 3) T3C(9, 4) T3C(9, 5) T3C(9, 6) T3C(9, 7) T3C(9, 8) T3C(9, 9)
#undef T3C
  return false;
}

template bool tensor3<double>(int, int, const XferArgs<double>&, hipStream_t);
template bool tensor3<float>(int, int, const XferArgs<float>&, hipStream_t);

// One workgroup per (parent, component, right-hand side), one thread per node: kinds 0 and 1
// gather the eight children (each contracted with its bits' 1D matrices through LDS, summed in
// child order), kind 2 contracts the parent's block once per child and adds it there.
template <int N, typename T>
__global__ void __launch_bounds__((N * N * N + 63) / 64 * 64) htransfer_kernel(HXferArgs<T> a) {
  constexpr int N2 = N * N, N3 = N * N * N;
  const int nsub = a.nrhs * a.ncomp;
  const int pidx = blockIdx.x / nsub, sub = blockIdx.x - pidx * nsub;
  if (pidx >= a.ncoarse) return;
  const int parent = a.parents ? a.parents[pidx] : pidx;
  const int rhs = sub / a.ncomp, comp = sub - rhs * a.ncomp;
  const int q = threadIdx.x;
  const bool act = q < N3;
  const int x = q % N, y = (q / N) % N, z = q / N2;
  __shared__ T sM[6][N2];
  __shared__ T s0[N3], s1[N3], s2[N3];
  for (int t = q; t < 6 * N2; t += blockDim.x) sM[t / N2][t % N2] = a.M[t];
  const int64_t cb = (int64_t)rhs * a.stride_c + ((int64_t)parent * a.ncomp + comp) * N3;
  // out_node = sum_k Mz[z][k] sum_j My[y][j] sum_i Mx[x][i] s0[k][j][i]
  auto contract = [&](const T* Mx, const T* My, const T* Mz) -> T {
    __syncthreads();
    if (act) {
      T v = 0;
      for (int i = 0; i < N; ++i) v += Mx[x * N + i] * s0[(z * N + y) * N + i];
      s1[q] = v;
    }
    __syncthreads();
    if (act) {
      T v = 0;
      for (int j = 0; j < N; ++j) v += My[y * N + j] * s1[(z * N + j) * N + x];
      s2[q] = v;
    }
    __syncthreads();
    T v = 0;
    if (act)
      for (int k = 0; k < N; ++k) v += Mz[z * N + k] * s2[(k * N + y) * N + x];
    return v;
  };
  if (a.kind <= 1) {
    const int m0 = a.kind == 0 ? 0 : 2;
    T acc = 0;
    for (int c = 0; c < 8; ++c) {
      const int bx = c & 1, by = (c >> 1) & 1, bz = c >> 2;
      const int child = a.children[(int64_t)pidx * 8 + c];
      __syncthreads();   // the previous child's contraction has read s0
      if (act) s0[q] = a.in[(int64_t)rhs * a.stride_f + ((int64_t)child * a.ncomp + comp) * N3 + q];
      acc += contract(sM[m0 + bx], sM[m0 + by], sM[m0 + bz]);
    }
    if (act) a.out[cb + q] = a.accumulate ? a.out[cb + q] + acc : acc;
  } else {
    if (act) s0[q] = a.in[cb + q] - (a.in2 ? a.in2[cb + q] : T(0));
    for (int c = 0; c < 8; ++c) {
      const int bx = c & 1, by = (c >> 1) & 1, bz = c >> 2;
      const int child = a.children[(int64_t)pidx * 8 + c];
      const T v = contract(sM[4 + bx], sM[4 + by], sM[4 + bz]);
      if (act) {
        T& o = a.out[(int64_t)rhs * a.stride_f + ((int64_t)child * a.ncomp + comp) * N3 + q];
        o = a.accumulate ? o + v : v;   // every child node belongs to one parent: written once
      }
    }
  }
}

template <typename T>
bool htransfer(int p, const HXferArgs<T>& a, hipStream_t st) {
  if (a.ncoarse <= 0) return true;
  const dim3 g((unsigned)((int64_t)a.ncoarse * a.nrhs * a.ncomp));
  switch (p) {
#define HTC(P) \
  case P: hipLaunchKernelGGL((htransfer_kernel<P + 1, T>), g, dim3(((P + 1) * (P + 1) * (P + 1) + 63) / 64 * 64), 0, st, a); return true;
    HTC(1) HTC(2) HTC(3) HTC(4) HTC(5) HTC(6) HTC(7) HTC(8)
#undef HTC
    default: return false;
  }
}
template bool htransfer<double>(int, const HXferArgs<double>&, hipStream_t);

__global__ void __launch_bounds__(256) copy_rows_kernel(const int* __restrict__ list, int n, int n3,
                                                        const double* __restrict__ src, double* __restrict__ dst) {
  const int i = blockIdx.x;
  if (i >= n) return;
  const int64_t o = (int64_t)list[i] * n3;
  for (int q = threadIdx.x; q < n3; q += blockDim.x) dst[o + q] = src[o + q];
}

void copy_rows(const int* list, int n, int n3, const double* src, double* dst, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(copy_rows_kernel, dim3(n), dim3(256), 0, st, list, n, n3, src, dst);
}

__global__ void __launch_bounds__(256) rows_sumsq_kernel(const int* __restrict__ list, int n, int n3,
                                                         const double* __restrict__ v, double* __restrict__ out) {
  __shared__ double sh[256];
  const int i = blockIdx.x;
  if (i >= n) return;
  const int64_t o = (int64_t)list[i] * n3;
  double s = 0;
  for (int q = threadIdx.x; q < n3; q += blockDim.x) s += v[o + q] * v[o + q];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = sh[0];
}

void rows_sumsq(const int* list, int n, int n3, const double* v, double* out, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(rows_sumsq_kernel, dim3(n), dim3(256), 0, st, list, n, n3, v, out);
}

// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;

int reduction_blocks(int64_t n) {
  int64_t b = (n + kRedThreads * 8 - 1) / (kRedThreads * 8);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

// v -= mean(v), per right-hand side: block sums in a fixed order, then every thread adds the
// (at most 1024) block sums of its right-hand side in order and subtracts the mean
__global__ void __launch_bounds__(kRedThreads) sum_partial_kernel(int64_t n, const double* __restrict__ v,
                                                                 double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const double* x = v + (int64_t)blockIdx.y * n;
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
    s += x[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = kRedThreads / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * 1024 + blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kRedThreads) subtract_mean_kernel(int64_t n, int nb, double* __restrict__ v,
                                                                   const double* __restrict__ partial) {
  __shared__ double mean;
  if (threadIdx.x == 0) {
    double s = 0;
    for (int b = 0; b < nb; ++b) s += partial[(int64_t)blockIdx.y * 1024 + b];
    mean = s / (double)n;
  }
  __syncthreads();
  double* x = v + (int64_t)blockIdx.y * n;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
    x[i] -= mean;
}

void project_mean(int64_t n, int nrhs, double* v, double* partial, hipStream_t st) {
  const int nb = reduction_blocks(n);
  hipLaunchKernelGGL(sum_partial_kernel, dim3(nb, nrhs), dim3(kRedThreads), 0, st, n, v, partial);
  hipLaunchKernelGGL(subtract_mean_kernel, dim3(nb, nrhs), dim3(kRedThreads), 0, st, n, nb, v, partial);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  return sh[0];
}

// Batched reductions: vectors are [nrhs][n]; block (blk, rhs) writes
// partial[rhs * 1024 + blk] = sum_i a_i (b_i - c_i) over its strided share of right-hand
// side rhs (b, c may be null: b := a, c := 0), accumulated in FP64.
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
dot_partial_kernel(int64_t n, const T* __restrict__ a, const T* __restrict__ b, const T* __restrict__ c,
                   double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const int64_t off = (int64_t)blockIdx.y * n;
  a += off;
  if (b) b += off;
  if (c) c += off;
  double s = 0;
  const int64_t stride = (int64_t)gridDim.x * kRedThreads;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
    const double bv = b ? (double)b[i] : (double)a[i];
    s += (double)a[i] * (c ? bv - (double)c[i] : bv);
  }
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.y * 1024 + blockIdx.x] = t;
}

template <typename T>
void dot_partials(int64_t n, int nrhs, const T* a, const T* b, const T* c, double* partial, int nblocks,
                  hipStream_t st) {
  hipLaunchKernelGGL((dot_partial_kernel<T>), dim3(nblocks, nrhs), dim3(kRedThreads), 0, st, n, a, b, c, partial);
}
template void dot_partials<double>(int64_t, int, const double*, const double*, const double*, double*, int,
                                   hipStream_t);
template void dot_partials<float>(int64_t, int, const float*, const float*, const float*, double*, int, hipStream_t);

// Second stage, one block per right-hand side: sums its partials (for kOpBeta also the
// second set at partial2) and applies the SCG scalar update selected by `op`.
//   scal[rhs * 8 + k]: 0 gamma (z^T r)  1 beta  2 alpha  3 r^T r  4 breakdown flag
//                      5 iterations run before convergence  6 stopping threshold on |r|
//                      (0: none)  7 converged flag
// A right-hand side whose |r| has reached its threshold is frozen (alpha = 0 from then on),
// so that in a batch every right-hand side stops at the iteration it would stop at alone.
__global__ void __launch_bounds__(1024) finish_kernel(int nblocks, const double* __restrict__ partial,
                                                      const double* __restrict__ partial2, int op,
                                                      double* __restrict__ scal, double* __restrict__ out,
                                                      int pstride) {
  __shared__ double sh[1024];
  const int tid = threadIdx.x, rhs = blockIdx.x;
  double v0 = 0, v1 = 0;
  for (int b = tid; b < nblocks; b += 1024) {
    v0 += partial[(int64_t)rhs * pstride + b];
    if (op == kOpBeta) v1 += partial2[(int64_t)rhs * pstride + b];
  }
  const double s0 = block_sum(v0, sh);
  __syncthreads();
  const double s1 = (op == kOpBeta) ? block_sum(v1, sh) : 0.0;
  if (tid != 0) return;
  double* sc = scal + rhs * 8;
  switch (op) {
    case kOpGamma:          // first iteration: gamma = z^T r
      sc[0] = s0;
      sc[1] = 0.0;
      break;
    case kOpBeta: {         // beta = z^T (r - r0) / gamma_old ; gamma = z^T r
      const double beta = s1 / sc[0];
      sc[1] = isfinite(beta) ? beta : 0.0;
      sc[0] = s0;
      if (!isfinite(beta)) sc[4] = 1.0;
      break;
    }
    case kOpAlpha: {        // alpha = gamma / p^T q; a converged right-hand side (p = 0) takes alpha = 0
      double alpha = (s0 != 0.0) ? sc[0] / s0 : 0.0;
      if (sc[7] != 0.0) alpha = 0.0;
      else if (s0 < 0.0 || !isfinite(alpha)) { sc[4] = 1.0; alpha = 0.0; }
      sc[2] = alpha;
      break;
    }
    case kOpNorm2:          // r^T r
      sc[3] = s0;
      if (!isfinite(s0)) sc[4] = 1.0;
      if (sc[7] == 0.0) {
        sc[5] += 1.0;
        if (sc[6] > 0.0 && sqrt(s0) <= sc[6]) sc[7] = 1.0;
      }
      break;
    case kOpStore:
      out[rhs] = s0;
      break;
  }
}

void finish(int nblocks, int nrhs, const double* partial, const double* partial2, int op, double* scal, double* out,
            hipStream_t st, int pstride) {
  hipLaunchKernelGGL(finish_kernel, dim3(nrhs), dim3(1024), 0, st, nblocks, partial, partial2, op, scal, out,
                     pstride);
}

// p = beta p + z   (first: p = z), per right-hand side beta
template <typename T>
__global__ void pupdate_kernel(int64_t n, int nrhs, const T* __restrict__ z, T* __restrict__ p, T* __restrict__ x,
                               const double* __restrict__ scal, int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const int rhs = (int)(i / n);
  if (first) {
    p[i] = z[i];
    return;
  }
  const T po = p[i];
  if (x) x[i] += (T)scal[rhs * 8 + 2] * po;     // the previous iteration's u += alpha p
  p[i] = (T)scal[rhs * 8 + 1] * po + z[i];
}

// x += alpha p (the last iteration's update)
template <typename T>
__global__ void xupdate_kernel(int64_t n, int nrhs, T* __restrict__ x, const T* __restrict__ p,
                               const double* __restrict__ scal) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  x[i] += (T)scal[(i / n) * 8 + 2] * p[i];
}

// y += (double)(x + alpha p): the last SCG update of an FP32 correction added straight to the
// FP64 iterate (the correction itself is not needed afterwards)
__global__ void xupdate_acc_kernel(int64_t n, int nrhs, const float* __restrict__ x, const float* __restrict__ p,
                                   const double* __restrict__ scal, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const float xn = x[i] + (float)scal[(i / n) * 8 + 2] * p[i];
  y[i] = y[i] + (double)xn;
}

void xupdate_acc(int64_t n, int nrhs, const float* x, const float* p, const double* scal, double* y, hipStream_t st) {
  const int64_t tot = n * nrhs;
  hipLaunchKernelGGL(xupdate_acc_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, nrhs, x, p, scal, y);
}

// rout = rin - alpha q (rout may be rin); partial[rhs*1024 + blk] = sum rout^2 (partial null: no sums)
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
cg_update_kernel(int64_t n, const T* __restrict__ rin, T* __restrict__ rout, const T* __restrict__ q,
                 const double* __restrict__ scal, double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const int rhs = blockIdx.y;
  const int64_t off = (int64_t)rhs * n;
  rin += off; rout += off; q += off;
  const T alpha = (T)scal[rhs * 8 + 2];
  double s = 0;
  const int64_t stride = (int64_t)gridDim.x * kRedThreads;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
    const T rn = rin[i] - alpha * q[i];
    rout[i] = rn;
    s += (double)rn * (double)rn;
  }
  if (!partial) return;   // no norm wanted (uniform over the grid)
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[rhs * 1024 + blockIdx.x] = t;
}

template <typename T>
void pupdate(int64_t n, int nrhs, const T* z, T* p, T* x, const double* scal, int first, hipStream_t st) {
  const int64_t tot = n * nrhs;
  hipLaunchKernelGGL((pupdate_kernel<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, nrhs, z, p, x,
                     scal, first);
}

template <typename T>
void xupdate(int64_t n, int nrhs, T* x, const T* p, const double* scal, hipStream_t st) {
  const int64_t tot = n * nrhs;
  hipLaunchKernelGGL((xupdate_kernel<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, nrhs, x, p, scal);
}

template <typename T>
void cg_update(int64_t n, int nrhs, const T* rin, T* rout, const T* q, const double* scal, double* partial,
               int nblocks, hipStream_t st) {
  hipLaunchKernelGGL((cg_update_kernel<T>), dim3(nblocks, nrhs), dim3(kRedThreads), 0, st, n, rin, rout, q, scal,
                     partial);
}
template void pupdate<double>(int64_t, int, const double*, double*, double*, const double*, int, hipStream_t);
template void pupdate<float>(int64_t, int, const float*, float*, float*, const double*, int, hipStream_t);
template void xupdate<double>(int64_t, int, double*, const double*, const double*, hipStream_t);
template void xupdate<float>(int64_t, int, float*, const float*, const double*, hipStream_t);
template void cg_update<double>(int64_t, int, const double*, double*, const double*, const double*, double*, int,
                                hipStream_t);
template void cg_update<float>(int64_t, int, const float*, float*, const float*, const double*, double*, int,
                               hipStream_t);

// y = x (with optional conversion) / y += x
template <typename TI, typename TO>
__global__ void convert_kernel(int64_t n, const TI* __restrict__ x, TO* __restrict__ y, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = accumulate ? (TO)(y[i] + (TO)x[i]) : (TO)x[i];
}

template <typename TI, typename TO>
void convert(int64_t n, const TI* x, TO* y, int accumulate, hipStream_t st) {
  hipLaunchKernelGGL((convert_kernel<TI, TO>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, y,
                     accumulate);
}
template void convert<double, double>(int64_t, const double*, double*, int, hipStream_t);
template void convert<double, float>(int64_t, const double*, float*, int, hipStream_t);
template void convert<float, double>(int64_t, const float*, double*, int, hipStream_t);
template void convert<float, float>(int64_t, const float*, float*, int, hipStream_t);

__global__ void mask_mul_kernel(int64_t n, double* __restrict__ y, const double* __restrict__ m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] *= m[i];
}
void mask_mul(int64_t n, double* y, const double* m, hipStream_t st) {
  hipLaunchKernelGGL(mask_mul_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, y, m);
}

__global__ void fill_kernel(int64_t n, double* __restrict__ y, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}
void fill(int64_t n, double* y, double v, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, y, v);
}
__global__ void fillf_kernel(int64_t n, float* __restrict__ y, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}
void fill(int64_t n, float* y, float v, hipStream_t st) {
  hipLaunchKernelGGL(fillf_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, y, v);
}

}  // namespace dgfas
