// Weighted overlapping Schwarz method on unstructured meshes (Sec. 4.3.1, design principles
// 4-6 and 8-10, with the oriented neighbour data of Sec. 5.1).
//
// The subdomain of an element is the structured tile (the element plus its overlap layers,
// ns^3 slots, smaller variants zero-padded), but which node fills a slot is decided on the
// host by walking across oriented faces: a slot holds one node, the mean of several merged
// nodes (surplus neighbours at an irregular edge or vertex), or zero (no counterpart).
//   topo_solve:   one workgroup per subdomain gathers r_s = R_s r through the slot table,
//                 applies the fast-diagonalisation solve of the surrogate, stores the tile;
//   topo_scatter: one thread per node sums its weighted contributions from the stored tiles
//                 in a fixed order (deterministic, no atomics).
#include "device.hpp"
#include "kernels.hpp"

namespace dgfas {

template <int NS>
struct TopoShape {
  static constexpr int LS = NS | 1;   // odd pitch of xi_1 rows
  static constexpr int NT = NS * NS * NS;
  static constexpr int THREADS = NS * NS <= 64 ? 64 : ((NS * NS + 63) / 64) * 64;
};

// one 1D contraction of every tile line along one direction: line <- M line (M[c][q] read
// through the scalar cache, uniform over the workgroup)
template <int NS, typename T>
__device__ __forceinline__ void contract(T* tA, int base, int stride, const T* __restrict__ M, bool act) {
  if (act) {
    T line[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) line[q] = tA[base + q * stride];
#pragma unroll 1
    for (int c = 0; c < NS; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < NS; ++q) s += M[c * NS + q] * line[q];
      tA[base + c * stride] = s;
    }
  }
  __syncthreads();
}

template <int NS, typename T>
__global__ void __launch_bounds__(TopoShape<NS>::THREADS) topo_solve_kernel(TopoArgs<T> a) {
  using Sh = TopoShape<NS>;
  constexpr int LS = Sh::LS, NT = Sh::NT;
  __shared__ T tA[NS * NS * LS];
  const int lbr = blockIdx.x;
  const int e = lbr / a.nrhs, rhs = lbr - e * a.nrhs;   // right-hand side fastest
  const T* __restrict__ r = a.r + (int64_t)rhs * a.ndof;
  // the 1D variants, made uniform where the contractions need them
  const int v0r = a.var[(int64_t)e * 3 + 0], v1r = a.var[(int64_t)e * 3 + 1], v2r = a.var[(int64_t)e * 3 + 2];
  const T g0 = a.gco[(int64_t)e * 4 + 0], g1 = a.gco[(int64_t)e * 4 + 1];
  const T g2 = a.gco[(int64_t)e * 4 + 2], g3 = a.gco[(int64_t)e * 4 + 3];
  const int tid = threadIdx.x;
  const bool act = tid < NS * NS;
  const int c1 = tid % NS, c2 = tid / NS;   // the thread's xi_3 column (s1, s2)

  // gather r_s = R_s r: the column's slot entries go out in one batch, then the values of
  // every slot at once (a zero or merged slot reads node 0 and discards it), so that the
  // column waits for memory twice; the rare merged slots (means over several nodes) follow
  if (act) {
    const int* __restrict__ gt = a.gather + (int64_t)e * NT + c2 * NS + c1;
    int gi[NS];
#pragma unroll
    for (int s3 = 0; s3 < NS; ++s3) gi[s3] = gt[s3 * NS * NS];
    T vals[NS];
#pragma unroll
    for (int s3 = 0; s3 < NS; ++s3) vals[s3] = r[gi[s3] >= 0 ? gi[s3] : 0];
#pragma unroll
    for (int s3 = 0; s3 < NS; ++s3) {
      if (gi[s3] >= 0) continue;
      T v = 0;
      if (gi[s3] < -1) {
        const int j = -2 - gi[s3], b = a.mptr[j], en = a.mptr[j + 1];
        const T share = T(1) / T(en - b);
        for (int k = b; k < en; ++k) v += share * r[a.midx[k]];
      }
      vals[s3] = v;
    }
#pragma unroll
    for (int s3 = 0; s3 < NS; ++s3) tA[(s3 * NS + c2) * LS + c1] = vals[s3];
  }
  __syncthreads();

  const int v0 = __builtin_amdgcn_readfirstlane(v0r);
  const int v1 = __builtin_amdgcn_readfirstlane(v1r);
  const int v2 = __builtin_amdgcn_readfirstlane(v2r);
  const T* __restrict__ S1 = a.S + v0 * NS * NS;
  const T* __restrict__ S2 = a.S + v1 * NS * NS;
  const T* __restrict__ S3 = a.S + v2 * NS * NS;
  const T* __restrict__ S1T = a.ST + v0 * NS * NS;
  const T* __restrict__ S2T = a.ST + v1 * NS * NS;
  const T* __restrict__ S3T = a.ST + v2 * NS * NS;
  const int tlo = c1, thi = c2;
  // (S1^T, S2^T), then S3^T, D^-1, S3 along xi_3, then (S2, S1)
  contract<NS, T>(tA, (thi * NS + tlo) * LS, 1, S1T, act);
  contract<NS, T>(tA, thi * NS * LS + tlo, LS, S2T, act);
  if (act) {
    const int b = thi * LS + tlo, sd = NS * LS;
    T line[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) line[q] = tA[b + q * sd];
    const T base = g0 + g1 * a.lam[v0 * NS + tlo] + g2 * a.lam[v1 * NS + thi];
    const T* __restrict__ L3 = a.lam + v2 * NS;
#pragma unroll 1
    for (int c = 0; c < NS; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < NS; ++q) s += S3T[c * NS + q] * line[q];
      tA[b + c * sd] = s / (base + g3 * L3[c]);
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) line[q] = tA[b + q * sd];
#pragma unroll 1
    for (int c = 0; c < NS; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < NS; ++q) s += S3[c * NS + q] * line[q];
      tA[b + c * sd] = s;
    }
  }
  __syncthreads();
  contract<NS, T>(tA, thi * NS * LS + tlo, LS, S2, act);
  contract<NS, T>(tA, (thi * NS + tlo) * LS, 1, S1, act);

  if (act) {
    T* __restrict__ zt = a.Zt + ((int64_t)rhs * a.nel + e) * NT + c2 * NS + c1;
#pragma unroll
    for (int s3 = 0; s3 < NS; ++s3) zt[s3 * NS * NS] = tA[(s3 * NS + c2) * LS + c1];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) topo_scatter_kernel(TopoArgs<T> a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.ndof * a.nrhs) return;
  const int64_t rhs = t / a.ndof, g = t - rhs * a.ndof;
  const T* __restrict__ Z = a.Zt + rhs * a.nel * (int64_t)a.nt;
  T acc = 0;
  const int64_t b = a.sptr[g], en = a.sptr[g + 1];
  // four contributions per step: their slot entries in one batch, then their values, summed
  // in list order (entries past the end repeat the last one and are not added)
  for (int64_t k0 = b; k0 < en; k0 += 4) {
    int sl[4];
    T cf[4], zv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t k = k0 + j < en ? k0 + j : en - 1;
      sl[j] = a.sslot[k];
      cf[j] = a.scoef[k];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) zv[j] = Z[sl[j]];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (k0 + j < en) acc += cf[j] * zv[j];
  }
  if (a.mode == 0) a.z[t] = acc;
  else a.z[t] += acc;
}

template <int NS, typename T>
void launch_topo(const TopoArgs<T>& a, hipStream_t st) {
  const int nb = a.nel * a.nrhs;
  if (nb > 0) hipLaunchKernelGGL((topo_solve_kernel<NS, T>), dim3(nb), dim3(TopoShape<NS>::THREADS), 0, st, a);
}

template <typename T>
void topo_schwarz_solve(int ns, const TopoArgs<T>& a, hipStream_t st) {
  switch (ns) {
    case 2: launch_topo<2, T>(a, st); break;
    case 3: launch_topo<3, T>(a, st); break;
    case 4: launch_topo<4, T>(a, st); break;
    case 5: launch_topo<5, T>(a, st); break;
    case 6: launch_topo<6, T>(a, st); break;
    case 7: launch_topo<7, T>(a, st); break;
    case 8: launch_topo<8, T>(a, st); break;
    case 9: launch_topo<9, T>(a, st); break;
    case 10: launch_topo<10, T>(a, st); break;
    case 11: launch_topo<11, T>(a, st); break;
    case 13: launch_topo<13, T>(a, st); break;
    case 15: launch_topo<15, T>(a, st); break;
    default: break;
  }
}

template <typename T>
void topo_schwarz_scatter(const TopoArgs<T>& a, hipStream_t st) {
  const int64_t n = a.ndof * a.nrhs;
  if (n > 0) hipLaunchKernelGGL((topo_scatter_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
}

template void topo_schwarz_solve<double>(int, const TopoArgs<double>&, hipStream_t);
template void topo_schwarz_solve<float>(int, const TopoArgs<float>&, hipStream_t);
template void topo_schwarz_scatter<double>(const TopoArgs<double>&, hipStream_t);
template void topo_schwarz_scatter<float>(const TopoArgs<float>&, hipStream_t);

}  // namespace dgfas
