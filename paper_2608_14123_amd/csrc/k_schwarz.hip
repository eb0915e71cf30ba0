// K2: weighted overlapping Schwarz application z = sum_e R_s^T W^e (A~_s^e)^-1 R_s r
// (Sec. 4.3.1, eq. schwarz:correction) with fast-diagonalisation subdomain solves
//   (A~_s)^-1 = (S3 x S2 x S1) D^-1 (S3^T x S2^T x S1^T),
//   D = g0 + g1 lam1_i + g2 lam2_j + g3 lam3_k.
//
// schwarz_solve: one workgroup per subdomain.  The NS^3 tile (NS = N + 2M, smaller
// variants zero-padded) is gathered from the element and its 26 neighbours into
// LDS; each 1D contraction runs with one thread per tile line, the other two
// tile indices spread over the threads so that LDS accesses are unit-stride
// across the wavefront (the xi_1 lines use an odd row pitch).  The weighted own
// part goes straight to z (or is added to u), the weighted overlap parts go to a
// per-element overlap buffer.
// schwarz_overlap_add: gather form of the scatter, z[node] += contributions of
// the neighbours' subdomains in a fixed order -- deterministic, no atomics.
#include "device.hpp"
#include "kernels.hpp"

namespace dgfas {

template <int N, int M>
struct SzShape {
  static constexpr int NS = N + 2 * M;
  static constexpr int LS = NS | 1;                 // odd pitch of xi_1 rows
  static constexpr int TILE = NS * NS * LS;
  static constexpr int THREADS = ((NS * NS + 63) / 64) * 64 < 64 ? 64 : ((NS * NS + 63) / 64) * 64;
};

// first DOF of element e, and first inbox slot of element e
template <int N, typename T>
__device__ __forceinline__ int64_t elem_base(const SchwarzArgs<T>& a, int e) {
  return a.off ? a.off[e] : (int64_t)e * (N * N * N);
}
template <int N, int M, typename T>
__device__ __forceinline__ int64_t inbox_base(const SchwarzArgs<T>& a, int e) {
  constexpr Regions<N, M> R{};
  return a.offO ? a.offO[e] : (int64_t)e * R.size;
}

int overlap_size(int p, int m) {
  const int n = p + 1;
  return 6 * m * n * n + 12 * m * m * n + 8 * m * m * m;
}

template <int N, int M, typename T>
struct SzSmem {
  using Sh = SzShape<N, M>;
  T tA[Sh::TILE];             // the subdomain tile; every contraction updates its own lines in place
  T sW[3][Sh::NS];
  int sMap[3][Sh::NS];
  int sNb[27];
  int sOff[27];
};

// One subdomain solve (logical block lbr = element in the list, right-hand side fastest).
// Threads at or beyond THR (wider batched workgroups) only pass the barriers.
template <int N, int M, typename T>
__device__ __forceinline__ void schwarz_tile(SchwarzArgs<T> a, const int lbr, SzSmem<N, M, T>& sm, int tid_in = -1) {
  using Sh = SzShape<N, M>;
  constexpr int NS = Sh::NS, LS = Sh::LS, THR = Sh::THREADS;
  constexpr Regions<N, M> R{};
  const int li = lbr / a.nrhs, rhs = lbr - li * a.nrhs;   // right-hand side fastest
  const int e = a.elist ? a.elist[li] : li;
  if (a.sel && !a.sel[e]) return;
  a.r += (int64_t)rhs * a.ndof;
  a.z += (int64_t)rhs * a.ndof;
  a.O += (int64_t)rhs * a.nin;
  const int tid = tid_in >= 0 ? tid_in : (int)threadIdx.x;   // tid_in: from a persistent batch

  T(&tA)[Sh::TILE] = sm.tA;
  T(&sW)[3][NS] = sm.sW;
  int(&sMap)[3][NS] = sm.sMap;
  int(&sNb)[27] = sm.sNb;
  int(&sOff)[27] = sm.sOff;

  // variant per direction: uniform over the workgroup, so the eigenvector tables
  // are read through the scalar cache straight into SGPR operands
  const int v0 = __builtin_amdgcn_readfirstlane(a.var[(int64_t)e * 3 + 0]);
  const int v1 = __builtin_amdgcn_readfirstlane(a.var[(int64_t)e * 3 + 1]);
  const int v2 = __builtin_amdgcn_readfirstlane(a.var[(int64_t)e * 3 + 2]);
  const T* __restrict__ S1 = a.S + v0 * NS * NS;
  const T* __restrict__ S2 = a.S + v1 * NS * NS;
  const T* __restrict__ S3 = a.S + v2 * NS * NS;
  const T* __restrict__ L3 = a.lam + v2 * NS;
  for (int t = tid; t < 3 * NS; t += THR) {
    const int d = t / NS, q = t - d * NS;
    const int v = d == 0 ? v0 : (d == 1 ? v1 : v2);
    sW[d][q] = a.W[v * NS + q];
    sMap[d][q] = a.map1d[v * NS + q];
  }
  if (tid < 27) {
    int nb = a.nb27[(int64_t)e * 27 + tid];
    if (nb >= 0 && a.deg && a.deg[nb] != N - 1) nb = -1;   // another degree: zero fill, no scatter
    sNb[tid] = nb;
    sOff[tid] = R.off[tid];
  }
  const T g0 = a.gco[(int64_t)e * 4 + 0], g1 = a.gco[(int64_t)e * 4 + 1];
  const T g2 = a.gco[(int64_t)e * 4 + 2], g3 = a.gco[(int64_t)e * 4 + 3];
  __syncthreads();

  // gather r_s = R_s r, one thread per xi_3 column (s1, s2) of the tile: the column's
  // node (l1, l2) in each of the three elements it crosses is found once, the xi_3
  // positions (uniform over the workgroup) then only select the element and the layer.
  // Every load of a thread is issued before its LDS stores.
  const bool act = tid < NS * NS;
  const int c1 = tid % NS, c2 = tid / NS;
  int m3u[NS];
#pragma unroll
  for (int s3 = 0; s3 < NS; ++s3) m3u[s3] = __builtin_amdgcn_readfirstlane(sMap[2][s3]);
  if (act) {
    const int m1 = sMap[0][c1], m2 = sMap[1][c2];
    int64_t cb[3];
#pragma unroll
    for (int d3 = 0; d3 < 3; ++d3) {
      cb[d3] = -1;
      if (m1 >= 0 && m2 >= 0) {
        const int src = sNb[d3 * 9 + (m2 >> 6) * 3 + (m1 >> 6)];   // absent neighbour: zeros
        if (src >= 0) cb[d3] = elem_base<N>(a, src) + (m2 & 63) * N + (m1 & 63);
      }
    }
    T vals[NS];
#pragma unroll
    for (int s3 = 0; s3 < NS; ++s3) {
      const int m3 = m3u[s3];
      vals[s3] = 0;
      if (m3 >= 0) {
        const int64_t cbase = cb[m3 >> 6];
        if (cbase >= 0) vals[s3] = a.r[cbase + (m3 & 63) * (N * N)];
      }
    }
#pragma unroll
    for (int s3 = 0; s3 < NS; ++s3) tA[(s3 * NS + c2) * LS + c1] = vals[s3];
  }
  __syncthreads();

  // Each contraction: one thread per tile line, out_c = sum_q M[c][q] line_q with the
  // row M[c][:] read through the scalar cache (uniform over the workgroup).
  const int tlo = c1, thi = c2;
  const T* __restrict__ S1T = a.ST + v0 * NS * NS;
  const T* __restrict__ S2T = a.ST + v1 * NS * NS;
  const T* __restrict__ S3T = a.ST + v2 * NS * NS;
  T line[NS];
  // phase 1: xi_1 with S1^T   (thread: s2 = tlo, s3 = thi)
  if (act) {
    const int b = (thi * NS + tlo) * LS;
#pragma unroll
    for (int q = 0; q < NS; ++q) line[q] = tA[b + q];
#pragma unroll 1
    for (int c = 0; c < NS; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < NS; ++q) s += S1T[c * NS + q] * line[q];
      tA[b + c] = s;
    }
  }
  __syncthreads();
  // phase 2: xi_2 with S2^T   (thread: s1 = tlo, s3 = thi)
  if (act) {
#pragma unroll
    for (int q = 0; q < NS; ++q) line[q] = tA[(thi * NS + q) * LS + tlo];
#pragma unroll 1
    for (int c = 0; c < NS; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < NS; ++q) s += S2T[c * NS + q] * line[q];
      tA[(thi * NS + c) * LS + tlo] = s;
    }
  }
  __syncthreads();
  // phase 3: xi_3 with S3^T, divide by D, xi_3 with S3   (thread: s1 = tlo, s2 = thi);
  // the thread's own k-line of tA holds the intermediate
  if (act) {
#pragma unroll
    for (int q = 0; q < NS; ++q) line[q] = tA[(q * NS + thi) * LS + tlo];
    const T base = g0 + g1 * a.lam[v0 * NS + tlo] + g2 * a.lam[v1 * NS + thi];
#pragma unroll 1
    for (int c = 0; c < NS; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < NS; ++q) s += S3T[c * NS + q] * line[q];
      tA[(c * NS + thi) * LS + tlo] = s / (base + g3 * L3[c]);
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) line[q] = tA[(q * NS + thi) * LS + tlo];
#pragma unroll 1
    for (int c = 0; c < NS; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < NS; ++q) s += S3[c * NS + q] * line[q];
      tA[(c * NS + thi) * LS + tlo] = s;
    }
  }
  __syncthreads();
  // phase 4: xi_2 with S2   (thread: s1 = tlo, s3 = thi)
  if (act) {
#pragma unroll
    for (int q = 0; q < NS; ++q) line[q] = tA[(thi * NS + q) * LS + tlo];
#pragma unroll 1
    for (int c = 0; c < NS; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < NS; ++q) s += S2[c * NS + q] * line[q];
      tA[(thi * NS + c) * LS + tlo] = s;
    }
  }
  __syncthreads();
  // phase 5: xi_1 with S1   (thread: s2 = tlo, s3 = thi)
  if (act) {
    const int b = (thi * NS + tlo) * LS;
#pragma unroll
    for (int q = 0; q < NS; ++q) line[q] = tA[b + q];
#pragma unroll 1
    for (int c = 0; c < NS; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < NS; ++q) s += S1[c * NS + q] * line[q];
      tA[b + c] = s;
    }
  }
  __syncthreads();
  // weighted scatter, one thread per xi_3 column (s1, s2): own part to z, each overlap part
  // into the receiving element's inbox (region seen from the receiver), read back by
  // overlap_add.  The destination of the column in each of the three xi_3 elements is
  // found once; the xi_3 positions select it.
  if (act) {
    const int m1 = sMap[0][c1], m2 = sMap[1][c2];
    if (m1 >= 0 && m2 >= 0) {
      const int d1 = (m1 >> 6) - 1, d2 = (m2 >> 6) - 1, l1 = m1 & 63, l2 = m2 & 63;
      const T w12 = sW[0][c1] * sW[1][c2];
      int64_t db[3], nbase[3];   // nbase: the column's node (l1, l2, 0) in the receiving element
      int ds[3];
#pragma unroll
      for (int d3i = 0; d3i < 3; ++d3i) {
        const int d3 = d3i - 1;
        db[d3i] = -1;
        ds[d3i] = 0;
        nbase[d3i] = 0;
        if (d1 == 0 && d2 == 0 && d3 == 0) {
          db[d3i] = elem_base<N>(a, e) + l2 * N + l1;
          ds[d3i] = N * N;
          nbase[d3i] = db[d3i];
        } else {
          const int dest = sNb[d3i * 9 + (d2 + 1) * 3 + (d1 + 1)];
          if (dest >= 0) {
            nbase[d3i] = elem_base<N>(a, dest) + l2 * N + l1;
            const int r = (1 - d3) * 9 + (1 - d2) * 3 + (1 - d1);      // direction from dest back to e
            const int cc1 = d1 < 0 ? l1 - (N - M) : l1, cc2 = d2 < 0 ? l2 - (N - M) : l2;
            const int x1 = d1 ? M : N, x2 = d2 ? M : N;
            ds[d3i] = x2 * x1;
            db[d3i] = inbox_base<N, M>(a, dest) + sOff[r] + cc2 * x1 + cc1;
          }
        }
      }
#pragma unroll
      for (int s3 = 0; s3 < NS; ++s3) {
        const int m3 = m3u[s3];
        if (m3 < 0) continue;
        const int d3i = m3 >> 6, l3 = m3 & 63;
        T t = tA[(s3 * NS + c2) * LS + c1];
        if (a.corr) t += (T)(a.cscale[e] * (double)a.corr[(int64_t)e * (NS * NS * NS) + (s3 * NS + c2) * NS + c1]);
        T v = a.unweighted ? t : w12 * sW[2][s3] * t;
        const int64_t base = db[d3i];
        if (base < 0) continue;
        if (a.cinv && !a.unweighted) v *= a.cinv[nbase[d3i] + l3 * (N * N)];   // normalised weight
        const int c3 = d3i == 0 ? l3 - (N - M) : l3;   // layer index inside the receiver's region
        const int64_t gi = base + (int64_t)c3 * ds[d3i];
        if (d1 == 0 && d2 == 0 && d3i == 1) {
          if (a.mode == 0) a.z[gi] = v;
          else a.z[gi] += v;
        } else {
          a.O[gi] = v;
        }
      }
    }
  }
}

// Small subdomains (n <= 3, ns^3 <= 125): one thread per tile point, looping over the
// points when the workgroup is narrower than the tile; the three directions' tables are
// staged in LDS.  The contraction order and arithmetic are those of schwarz_tile.
template <int N, int M, typename T>
struct PtSmem {
  static constexpr int NS = N + 2 * M, NT = NS * NS * NS;
  T tile[NT];
  T S[3][NS * NS];
  T lam[3][NS];
  T W[3][NS];
  int map[3][NS];
  int nb[27];
  int off[27];
};

template <int N, int M, typename T>
__device__ __forceinline__ void schwarz_point_tile(SchwarzArgs<T> a, const int lbr, PtSmem<N, M, T>& sm,
                                                   const int nthr, int tid_in = -1) {
  constexpr int NS = N + 2 * M, NT = NS * NS * NS, MAXP = (NT + 63) / 64;
  constexpr Regions<N, M> R{};
  const int li = lbr / a.nrhs, rhs = lbr - li * a.nrhs;
  const int e = a.elist ? a.elist[li] : li;
  if (a.sel && !a.sel[e]) return;
  a.r += (int64_t)rhs * a.ndof;
  a.z += (int64_t)rhs * a.ndof;
  a.O += (int64_t)rhs * a.nin;
  const int tid = tid_in >= 0 ? tid_in : (int)threadIdx.x;
  const int vv[3] = {__builtin_amdgcn_readfirstlane(a.var[(int64_t)e * 3 + 0]),
                     __builtin_amdgcn_readfirstlane(a.var[(int64_t)e * 3 + 1]),
                     __builtin_amdgcn_readfirstlane(a.var[(int64_t)e * 3 + 2])};
  for (int t = tid; t < 3 * NS * NS; t += nthr) {
    const int d = t / (NS * NS), q = t - d * NS * NS;
    sm.S[d][q] = a.S[vv[d] * NS * NS + q];
  }
  for (int t = tid; t < 3 * NS; t += nthr) {
    const int d = t / NS, q = t - d * NS;
    sm.lam[d][q] = a.lam[vv[d] * NS + q];
    sm.W[d][q] = a.W[vv[d] * NS + q];
    sm.map[d][q] = a.map1d[vv[d] * NS + q];
  }
  if (tid < 27) {
    int nb = a.nb27[(int64_t)e * 27 + tid];
    if (nb >= 0 && a.deg && a.deg[nb] != N - 1) nb = -1;   // another degree: zero fill, no scatter
    sm.nb[tid] = nb;
    sm.off[tid] = R.off[tid];
  }
  const T g0 = a.gco[(int64_t)e * 4 + 0], g1 = a.gco[(int64_t)e * 4 + 1];
  const T g2 = a.gco[(int64_t)e * 4 + 2], g3 = a.gco[(int64_t)e * 4 + 3];
  __syncthreads();
  T v[MAXP];
  // gather r_s = R_s r
#pragma unroll
  for (int pp = 0; pp < MAXP; ++pp) {
    const int q = tid + pp * nthr;
    v[pp] = 0;
    if (q < NT) {
      const int s1 = q % NS, s2 = (q / NS) % NS, s3 = q / (NS * NS);
      const int m1 = sm.map[0][s1], m2 = sm.map[1][s2], m3 = sm.map[2][s3];
      if (m1 >= 0 && m2 >= 0 && m3 >= 0) {
        const int src = sm.nb[(m3 >> 6) * 9 + (m2 >> 6) * 3 + (m1 >> 6)];
        if (src >= 0) v[pp] = a.r[elem_base<N>(a, src) + ((m3 & 63) * N + (m2 & 63)) * N + (m1 & 63)];
      }
    }
  }
#pragma unroll
  for (int pp = 0; pp < MAXP; ++pp) {
    const int q = tid + pp * nthr;
    if (q < NT) sm.tile[q] = v[pp];
  }
  __syncthreads();
  // six contractions: xi_1 S1^T, xi_2 S2^T, xi_3 S3^T and 1/D, xi_3 S3, xi_2 S2, xi_1 S1
#pragma unroll 1
  for (int step = 0; step < 6; ++step) {
    const int dir = step < 3 ? step : 5 - step;
    const bool tr = step < 3;
#pragma unroll
    for (int pp = 0; pp < MAXP; ++pp) {
      const int q = tid + pp * nthr;
      if (q >= NT) continue;
      const int s[3] = {q % NS, (q / NS) % NS, q / (NS * NS)};
      const int c = s[dir];
      const int stride = dir == 0 ? 1 : (dir == 1 ? NS : NS * NS);
      const int q0 = q - c * stride;
      T acc = 0;
#pragma unroll
      for (int k = 0; k < NS; ++k) acc += (tr ? sm.S[dir][k * NS + c] : sm.S[dir][c * NS + k]) * sm.tile[q0 + k * stride];
      if (step == 2) acc = acc / (g0 + g1 * sm.lam[0][s[0]] + g2 * sm.lam[1][s[1]] + g3 * sm.lam[2][s[2]]);
      v[pp] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int pp = 0; pp < MAXP; ++pp) {
      const int q = tid + pp * nthr;
      if (q < NT) sm.tile[q] = v[pp];
    }
    __syncthreads();
  }
  // weighted scatter: own part to z, overlap parts into the receivers' inboxes
#pragma unroll
  for (int pp = 0; pp < MAXP; ++pp) {
    const int q = tid + pp * nthr;
    if (q >= NT) continue;
    const int s1 = q % NS, s2 = (q / NS) % NS, s3 = q / (NS * NS);
    const int m1 = sm.map[0][s1], m2 = sm.map[1][s2], m3 = sm.map[2][s3];
    if (m1 < 0 || m2 < 0 || m3 < 0) continue;
    T t = sm.tile[q];
    if (a.corr) t += (T)(a.cscale[e] * (double)a.corr[(int64_t)e * NT + q]);
    T val = a.unweighted ? t : sm.W[0][s1] * sm.W[1][s2] * sm.W[2][s3] * t;
    const int d1 = (m1 >> 6) - 1, d2 = (m2 >> 6) - 1, d3 = (m3 >> 6) - 1;
    const int l1 = m1 & 63, l2 = m2 & 63, l3 = m3 & 63;
    if (d1 == 0 && d2 == 0 && d3 == 0) {
      const int64_t gi = elem_base<N>(a, e) + (l3 * N + l2) * N + l1;
      if (a.cinv && !a.unweighted) val *= a.cinv[gi];   // normalised weight
      if (a.mode == 0) a.z[gi] = val;
      else a.z[gi] += val;
    } else {
      const int dest = sm.nb[(d3 + 1) * 9 + (d2 + 1) * 3 + (d1 + 1)];
      if (dest < 0) continue;
      if (a.cinv && !a.unweighted) val *= a.cinv[elem_base<N>(a, dest) + (l3 * N + l2) * N + l1];
      const int r = (1 - d3) * 9 + (1 - d2) * 3 + (1 - d1);      // direction from dest back to e
      const int c1 = d1 < 0 ? l1 - (N - M) : l1, c2 = d2 < 0 ? l2 - (N - M) : l2, c3 = d3 < 0 ? l3 - (N - M) : l3;
      const int x1 = d1 ? M : N, x2 = d2 ? M : N;
      a.O[inbox_base<N, M>(a, dest) + sm.off[r] + (c3 * x2 + c2) * x1 + c1] = val;
    }
  }
}

template <int N, int M, typename T>
__global__ void __launch_bounds__(((N + 2 * M) * (N + 2 * M) * (N + 2 * M) + 63) / 64 * 64)
schwarz_point_kernel(SchwarzArgs<T> a) {
  __shared__ PtSmem<N, M, T> sm;
  const int lbr = xcd_block(a.nel * a.nrhs);
  if (lbr < 0) return;
  schwarz_point_tile<N, M, T>(a, lbr, sm, blockDim.x);
}

template <int N>
struct AddShape {
  static constexpr int N3 = N * N * N;
  static constexpr int EPB = (N3 >= 256) ? 1 : (256 / N3);
  static constexpr int THREADS = ((EPB * N3 + 63) / 64) * 64;
};

template <int N, int M, typename T>
__global__ void __launch_bounds__((SzShape<N, M>::THREADS))
schwarz_solve_kernel(SchwarzArgs<T> a) {
  __shared__ SzSmem<N, M, T> sm;
  const int lbr = xcd_block(a.nel * a.nrhs);
  if (lbr < 0) return;
  schwarz_tile<N, M, T>(a, lbr, sm);
}

struct AddSmem {
  int sOff[27];
  double red[2][16];   // per-wavefront partial sums of the fused dot products
};

// z[node] += sum of the neighbours' overlap contributions in the element's own
// inbox, in a fixed order.  Inbox regions of absent neighbours stay zero.  With dotz set,
// also the tile's sums of z dr and z (dr - dr0) over every node (deterministic order).
template <int N, int M, typename T>
__device__ __forceinline__ void overlap_add_tile(SchwarzArgs<T> a, const int lbr, AddSmem& sm, int tid_in = -1) {
  using Sh = AddShape<N>;
  constexpr int N3 = Sh::N3, EPB = Sh::EPB;
  constexpr Regions<N, M> R{};
  const int lb = lbr / a.nrhs, rhs = lbr - lb * a.nrhs;
  a.z += (int64_t)rhs * a.ndof;
  a.O += (int64_t)rhs * a.nin;
  const int tid = tid_in >= 0 ? tid_in : (int)threadIdx.x;
  int(&sOff)[27] = sm.sOff;
  if (tid < 27) sOff[tid] = R.off[tid];
  const int le = tid / N3, node = tid - le * N3;
  const int li = lb * EPB + le;
  const bool act = le < EPB && li < a.nel;
  // the loads that need no region table go out ahead of the barrier
  int64_t gi = 0;
  int e = 0, l[3] = {0, 0, 0}, od[3] = {0, 0, 0};
  bool any = false;
  T z0 = 0;
  double rv = 0, r0v = 0;
  if (act) {
    e = a.elist ? a.elist[li] : li;
    gi = elem_base<N>(a, e) + node;
    l[0] = node % N;
    l[1] = (node / N) % N;
    l[2] = node / (N * N);
    // per direction the offset towards the one neighbour whose overlap can cover this node
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      od[d] = (l[d] < M) ? -1 : ((l[d] >= N - M) ? 1 : 0);
      any = any || od[d] != 0;
    }
    if (any || a.dotz) z0 = a.z[gi];
    if (a.dotz) {
      const int64_t ri = (int64_t)rhs * a.ndof + gi;
      rv = (double)a.dr[ri];
      if (a.dr0) r0v = (double)a.dr0[ri];
    }
  }
  __syncthreads();
  double pz = 0, pz2 = 0;
  if (act) {
    T zv = z0;
    if (any) {
      const T* __restrict__ box = a.O + inbox_base<N, M>(a, e);
      // the up to 7 candidates (subsets of the non-zero directions): every load is issued
      // unconditionally (invalid ones read entry 0 and are masked) so that none waits on another
      T vals[7];
      bool ok[7];
#pragma unroll
      for (int bits = 1; bits < 8; ++bits) {
        const int dd[3] = {(bits & 1) ? od[0] : 0, (bits & 2) ? od[1] : 0, (bits & 4) ? od[2] : 0};
        const bool valid = ((bits & 1) == 0 || od[0] != 0) && ((bits & 2) == 0 || od[1] != 0) &&
                           ((bits & 4) == 0 || od[2] != 0);
        int off = 0;
        if (valid) {
          const int r = (dd[2] + 1) * 9 + (dd[1] + 1) * 3 + (dd[0] + 1);
          const int c1 = dd[0] > 0 ? l[0] - (N - M) : l[0];
          const int c2 = dd[1] > 0 ? l[1] - (N - M) : l[1];
          const int c3 = dd[2] > 0 ? l[2] - (N - M) : l[2];
          const int x1 = dd[0] ? M : N, x2 = dd[1] ? M : N;
          off = sOff[r] + (c3 * x2 + c2) * x1 + c1;
        }
        ok[bits - 1] = valid;
        vals[bits - 1] = box[off];
      }
      T acc = 0;
#pragma unroll
      for (int t = 0; t < 7; ++t) acc += ok[t] ? vals[t] : T(0);
      zv = z0 + acc;
      a.z[gi] = zv;
    }
    if (a.dotz) {
      pz = (double)zv * rv;
      if (a.dr0) pz2 = (double)zv * (rv - r0v);
    }
  }
  if (a.dotz) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      pz += __shfl_xor(pz, off);
      pz2 += __shfl_xor(pz2, off);
    }
    if ((tid & 63) == 0 && tid < Sh::THREADS) {
      sm.red[0][tid >> 6] = pz;
      sm.red[1][tid >> 6] = pz2;
    }
    __syncthreads();
    if (tid == 0) {
      double s = 0, s2 = 0;
      for (int w = 0; w < Sh::THREADS / 64; ++w) {
        s += sm.red[0][w];
        s2 += sm.red[1][w];
      }
      const int ntiles = (a.nel + EPB - 1) / EPB;
      a.dotz[(int64_t)rhs * ntiles + lb] = s;
      if (a.dotz2) a.dotz2[(int64_t)rhs * ntiles + lb] = s2;
    }
  }
}

template <int N, int M, typename T>
__global__ void __launch_bounds__(AddShape<N>::THREADS)
schwarz_overlap_add_kernel(SchwarzArgs<T> a) {
  using Sh = AddShape<N>;
  __shared__ AddSmem sm;
  const int lbr = xcd_block(((a.nel + Sh::EPB - 1) / Sh::EPB) * a.nrhs);
  if (lbr < 0) return;
  overlap_add_tile<N, M, T>(a, lbr, sm);
}

// ---------------------------------------------------------------------------
// Tile helpers for the learned correction.  A tile is the NS^3 subdomain block of a
// vector in the layout of the FD solve (padded positions zero).
template <int N, int M>
struct TileCtx {
  static constexpr int NS = N + 2 * M, NT = NS * NS * NS;
  int map[3][NS];
  int nb[27];
};

template <int N, int M, typename T>
__device__ void load_tile_ctx(const SchwarzArgs<T>& a, int e, TileCtx<N, M>& c) {
  constexpr int NS = N + 2 * M;
  for (int t = threadIdx.x; t < 3 * NS; t += blockDim.x) {
    const int d = t / NS, q = t - d * NS;
    c.map[d][q] = a.map1d[a.var[(int64_t)e * 3 + d] * NS + q];
  }
  for (int t = threadIdx.x; t < 27; t += blockDim.x) c.nb[t] = a.nb27[(int64_t)e * 27 + t];
}

// global index of tile position q of the element, or -1 (padding / absent neighbour)
template <int N, int M>
__device__ __forceinline__ int64_t tile_index(const TileCtx<N, M>& c, int q) {
  constexpr int NS = N + 2 * M;
  const int s1 = q % NS, s2 = (q / NS) % NS, s3 = q / (NS * NS);
  const int m1 = c.map[0][s1], m2 = c.map[1][s2], m3 = c.map[2][s3];
  if (m1 < 0 || m2 < 0 || m3 < 0) return -1;
  const int src = c.nb[(m3 >> 6) * 9 + (m2 >> 6) * 3 + (m1 >> 6)];
  if (src < 0) return -1;
  return (int64_t)src * (N * N * N) + ((m3 & 63) * N + (m2 & 63)) * N + (m1 & 63);
}

// X[row] = [tile(v) / |tile(v)|, J9[e]], norms[row] = |tile(v)|
template <int N, int M, typename T>
__global__ void __launch_bounds__(256) tile_features_kernel(SchwarzArgs<T> a, const int* ids, int n,
                                                            const double* __restrict__ v, const double* __restrict__ J9,
                                                            float* __restrict__ X, double* __restrict__ norms) {
  using C = TileCtx<N, M>;
  __shared__ C c;
  __shared__ double tile[C::NT];
  __shared__ double red[256];
  const int row = blockIdx.x;
  if (row >= n) return;
  const int e = ids ? ids[row] : row;
  load_tile_ctx<N, M, T>(a, e, c);
  __syncthreads();
  double s = 0;
  for (int q = threadIdx.x; q < C::NT; q += 256) {
    const int64_t gi = tile_index<N, M>(c, q);
    const double x = gi >= 0 ? v[gi] : 0.0;
    tile[q] = x;
    s += x * x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const double nrm = sqrt(red[0]);
  const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
  const int64_t in = C::NT + 9;
  for (int q = threadIdx.x; q < C::NT; q += 256) X[(int64_t)row * in + q] = (float)(tile[q] * inv);
  if (threadIdx.x < 9) X[(int64_t)row * in + C::NT + threadIdx.x] = (float)J9[(int64_t)e * 9 + threadIdx.x];
  if (threadIdx.x == 0) norms[row] = nrm;
}

// out[row] = (tile(v1) - tile(v2)) / norms[row]
template <int N, int M, typename T>
__global__ void __launch_bounds__(256) tile_diff_kernel(SchwarzArgs<T> a, const int* ids, int n,
                                                        const double* __restrict__ v1, const double* __restrict__ v2,
                                                        const double* __restrict__ norms, float* __restrict__ out) {
  using C = TileCtx<N, M>;
  __shared__ C c;
  const int row = blockIdx.x;
  if (row >= n) return;
  const int e = ids ? ids[row] : row;
  load_tile_ctx<N, M, T>(a, e, c);
  __syncthreads();
  const double inv = norms[row] > 0 ? 1.0 / norms[row] : 0.0;
  for (int q = threadIdx.x; q < C::NT; q += 256) {
    const int64_t gi = tile_index<N, M>(c, q);
    out[(int64_t)row * C::NT + q] = gi >= 0 ? (float)((v1[gi] - v2[gi]) * inv) : 0.f;
  }
}

// mask = 1 on every node of the listed subdomains
template <int N, int M, typename T>
__global__ void __launch_bounds__(256) mark_kernel(SchwarzArgs<T> a, const int* ids, int n, double* __restrict__ mask) {
  using C = TileCtx<N, M>;
  __shared__ C c;
  const int row = blockIdx.x;
  if (row >= n) return;
  const int e = ids ? ids[row] : row;
  load_tile_ctx<N, M, T>(a, e, c);
  __syncthreads();
  for (int q = threadIdx.x; q < C::NT; q += 256) {
    const int64_t gi = tile_index<N, M>(c, q);
    if (gi >= 0) mask[gi] = 1.0;
  }
}

template <int N, int M, typename T>
void launch_features(const SchwarzArgs<T>& a, const int* ids, int n, const double* v, const double* J9, float* X,
                     double* norms, hipStream_t st) {
  hipLaunchKernelGGL((tile_features_kernel<N, M, T>), dim3(n), dim3(256), 0, st, a, ids, n, v, J9, X, norms);
}
template <int N, int M, typename T>
void launch_diff(const SchwarzArgs<T>& a, const int* ids, int n, const double* v1, const double* v2,
                 const double* norms, float* out, hipStream_t st) {
  hipLaunchKernelGGL((tile_diff_kernel<N, M, T>), dim3(n), dim3(256), 0, st, a, ids, n, v1, v2, norms, out);
}
template <int N, int M, typename T>
void launch_mark(const SchwarzArgs<T>& a, const int* ids, int n, double* mask, hipStream_t st) {
  hipLaunchKernelGGL((mark_kernel<N, M, T>), dim3(n), dim3(256), 0, st, a, ids, n, mask);
}

#define DGFAS_TILE_CASES(CALL)                           \
  switch (p * 16 + m) {                                  \
    case 1 * 16 + 1: CALL(2, 1); break;                  \
    case 2 * 16 + 1: CALL(3, 1); break;                  \
    case 3 * 16 + 1: CALL(4, 1); break;                  \
    case 4 * 16 + 1: CALL(5, 1); break;                  \
    case 5 * 16 + 1: CALL(6, 1); break;                  \
    case 6 * 16 + 1: CALL(7, 1); break;                  \
    case 7 * 16 + 1: CALL(8, 1); break;                  \
    case 8 * 16 + 1: CALL(9, 1); break;                  \
    default: break;                                      \
  }

template <typename T>
void tile_features(int p, int m, const SchwarzArgs<T>& a, const int* ids, int n, const double* v, const double* J9,
                   float* X, double* norms, hipStream_t st) {
#define CALLF(NN, MM) launch_features<NN, MM, T>(a, ids, n, v, J9, X, norms, st)
  DGFAS_TILE_CASES(CALLF)
#undef CALLF
}
template <typename T>
void tile_diff(int p, int m, const SchwarzArgs<T>& a, const int* ids, int n, const double* v1, const double* v2,
               const double* norms, float* out, hipStream_t st) {
#define CALLD(NN, MM) launch_diff<NN, MM, T>(a, ids, n, v1, v2, norms, out, st)
  DGFAS_TILE_CASES(CALLD)
#undef CALLD
}
template <typename T>
void mark_subdomains(int p, int m, const SchwarzArgs<T>& a, const int* ids, int n, double* mask, hipStream_t st) {
#define CALLM(NN, MM) launch_mark<NN, MM, T>(a, ids, n, mask, st)
  DGFAS_TILE_CASES(CALLM)
#undef CALLM
}
template void tile_features<double>(int, int, const SchwarzArgs<double>&, const int*, int, const double*,
                                    const double*, float*, double*, hipStream_t);
template void tile_diff<double>(int, int, const SchwarzArgs<double>&, const int*, int, const double*, const double*,
                                const double*, float*, hipStream_t);
template void mark_subdomains<double>(int, int, const SchwarzArgs<double>&, const int*, int, double*, hipStream_t);

template <int N, int M, typename T>
void launch_schwarz(const SchwarzArgs<T>& a, hipStream_t st) {
  if constexpr (N <= 3) {
    constexpr int NS = N + 2 * M, THR = (NS * NS * NS + 63) / 64 * 64;
    hipLaunchKernelGGL((schwarz_point_kernel<N, M, T>), dim3(xcd_grid(a.nel * a.nrhs)), dim3(THR), 0, st, a);
  } else {
    hipLaunchKernelGGL((schwarz_solve_kernel<N, M, T>), dim3(xcd_grid(a.nel * a.nrhs)), dim3(SzShape<N, M>::THREADS),
                       0, st, a);
  }
}

template <int N, int M, typename T>
void launch_overlap(const SchwarzArgs<T>& a, hipStream_t st) {
  using Sh = AddShape<N>;
  const int nb = ((a.nel + Sh::EPB - 1) / Sh::EPB) * a.nrhs;
  hipLaunchKernelGGL((schwarz_overlap_add_kernel<N, M, T>), dim3(xcd_grid(nb)), dim3(Sh::THREADS), 0, st, a);
}

#define DGFAS_SZ_CASES(F)                                                       \
  switch (p * 16 + m) {                                                         \
    case 1 * 16 + 0: F<2, 0, T>(a, st); break;                                  \
    case 1 * 16 + 1: F<2, 1, T>(a, st); break;                                  \
    case 2 * 16 + 0: F<3, 0, T>(a, st); break;                                  \
    case 2 * 16 + 1: F<3, 1, T>(a, st); break;                                  \
    case 3 * 16 + 0: F<4, 0, T>(a, st); break;                                  \
    case 3 * 16 + 1: F<4, 1, T>(a, st); break;                                  \
    case 4 * 16 + 0: F<5, 0, T>(a, st); break;                                  \
    case 4 * 16 + 1: F<5, 1, T>(a, st); break;                                  \
    case 4 * 16 + 2: F<5, 2, T>(a, st); break;                                  \
    case 5 * 16 + 0: F<6, 0, T>(a, st); break;                                  \
    case 5 * 16 + 1: F<6, 1, T>(a, st); break;                                  \
    case 6 * 16 + 0: F<7, 0, T>(a, st); break;                                  \
    case 6 * 16 + 1: F<7, 1, T>(a, st); break;                                  \
    case 7 * 16 + 0: F<8, 0, T>(a, st); break;                                  \
    case 7 * 16 + 1: F<8, 1, T>(a, st); break;                                  \
    case 8 * 16 + 0: F<9, 0, T>(a, st); break;                                  \
    case 8 * 16 + 1: F<9, 1, T>(a, st); break;                                  \
    case 8 * 16 + 2: F<9, 2, T>(a, st); break;                                  \
    case 8 * 16 + 3: F<9, 3, T>(a, st); break;                                  \
    default: break;                                                             \
  }

template <typename T>
void schwarz_solve(int p, int m, const SchwarzArgs<T>& a, hipStream_t st) {
  DGFAS_SZ_CASES(launch_schwarz)
}
template <typename T>
void schwarz_overlap_add(int p, int m, const SchwarzArgs<T>& a, hipStream_t st) {
  if (m == 0) return;
  DGFAS_SZ_CASES(launch_overlap)
}

// ---------------------------------------------------------------------------
// Batched launches over the degree buckets of a mixed-degree level (overlap m = 1).
template <typename T, int N>
constexpr size_t sz_smem_upto() {
  if constexpr (N < 2) {
    return 0;
  } else {
    constexpr size_t a = N <= 3 ? sizeof(PtSmem<N, 1, T>) : sizeof(SzSmem<N, 1, T>), b = sz_smem_upto<T, N - 1>();
    return a > b ? a : b;
  }
}

template <int NMAX, typename T, bool PERSIST>
__global__ void __launch_bounds__((SzShape<NMAX, 1>::THREADS))
schwarz_batched_kernel(SchwarzArgs<T> a, const BucketDesc<T>* __restrict__ bd, int nb, int ntiles) {
  __shared__ __align__(16) char smem[sz_smem_upto<T, NMAX>()];
  // tiles dealt round-robin over the XCDs (the hardware order): the work list runs from the
  // largest degree to the smallest, and contiguous ranges per XCD would leave one XCD all
  // the large tiles.  The persistent form strides through the list, with a barrier between
  // tiles for the shared memory.
  auto tile = [&](int t) {
    int tid = -1;   // persistent form: an opaque copy per tile (see sipg_batched_kernel)
    if constexpr (PERSIST) {
      tid = threadIdx.x;
      asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(tid));
    }
    const int k = find_bucket(bd, nb, kStageSolve, t);
    SchwarzArgs<T> x = a;
    x.nel = bd[k].nel;
    x.elist = bd[k].elist;
    x.S = bd[k].S;
    x.ST = bd[k].ST;
    x.lam = bd[k].lam;
    x.W = bd[k].W;
    x.map1d = bd[k].map1d;
    const int lbr = t - bd[k].tile0[kStageSolve];
    switch (bd[k].p) {
#define DGFAS_SZB(P)                                                                                  \
  case P:                                                                                             \
    if constexpr (P + 1 <= 3) schwarz_point_tile<P + 1, 1, T>(x, lbr, *reinterpret_cast<PtSmem<P + 1, 1, T>*>(smem), blockDim.x, tid); \
    else if constexpr (P + 1 <= NMAX) schwarz_tile<P + 1, 1, T>(x, lbr, *reinterpret_cast<SzSmem<P + 1, 1, T>*>(smem), tid); \
    break;
      DGFAS_SZB(1) DGFAS_SZB(2) DGFAS_SZB(3) DGFAS_SZB(4) DGFAS_SZB(5) DGFAS_SZB(6) DGFAS_SZB(7) DGFAS_SZB(8)
#undef DGFAS_SZB
      default: break;
    }
  };
  if constexpr (PERSIST) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
      if (t != (int)blockIdx.x) __syncthreads();
      tile(t);
    }
  } else {
    if ((int)blockIdx.x < ntiles) tile(blockIdx.x);
  }
}

template <int NMAX, typename T, bool PERSIST>
__global__ void __launch_bounds__(AddShape<NMAX>::THREADS)
overlap_add_batched_kernel(SchwarzArgs<T> a, const BucketDesc<T>* __restrict__ bd, int nb, int ntiles) {
  __shared__ AddSmem sm;
  // tiles dealt round-robin over the XCDs (the hardware order), strided in the persistent form
  auto tile = [&](int t) {
    int tid = -1;   // persistent form: an opaque copy per tile (see sipg_batched_kernel)
    if constexpr (PERSIST) {
      tid = threadIdx.x;
      asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(tid));
    }
    const int k = find_bucket(bd, nb, kStageAdd, t);
    SchwarzArgs<T> x = a;
    x.nel = bd[k].nel;
    x.elist = bd[k].elist;
    const int lbr = t - bd[k].tile0[kStageAdd];
    switch (bd[k].p) {
#define DGFAS_ADB(P)                                                          \
  case P:                                                                     \
    if constexpr (P + 1 <= NMAX) overlap_add_tile<P + 1, 1, T>(x, lbr, sm, tid);  \
    break;
      DGFAS_ADB(1) DGFAS_ADB(2) DGFAS_ADB(3) DGFAS_ADB(4) DGFAS_ADB(5) DGFAS_ADB(6) DGFAS_ADB(7) DGFAS_ADB(8)
#undef DGFAS_ADB
      default: break;
    }
  };
  if constexpr (PERSIST) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
      if (t != (int)blockIdx.x) __syncthreads();
      tile(t);
    }
  } else {
    if ((int)blockIdx.x < ntiles) tile(blockIdx.x);
  }
}

#define DGFAS_BATCH_ONE(KERNEL, NM)                                                                     \
  if (l.persistent) hipLaunchKernelGGL((KERNEL<NM, T, true>), g, b, 0, st, a, bd, l.nb, l.ntiles);     \
  else hipLaunchKernelGGL((KERNEL<NM, T, false>), g, b, 0, st, a, bd, l.nb, l.ntiles);
#define DGFAS_BATCH_LAUNCH(KERNEL, STAGE)                                                              \
  if (l.ntiles <= 0) return;                                                                           \
  const dim3 g(l.grid), b(stage_threads(STAGE, pmax));                                                 \
  if (pmax <= 5) { DGFAS_BATCH_ONE(KERNEL, 6) }                                                        \
  else if (pmax == 6) { DGFAS_BATCH_ONE(KERNEL, 7) }                                                   \
  else if (pmax == 7) { DGFAS_BATCH_ONE(KERNEL, 8) }                                                   \
  else { DGFAS_BATCH_ONE(KERNEL, 9) }

template <typename T>
void schwarz_solve_batched(int pmax, const SchwarzArgs<T>& a, const BucketDesc<T>* bd, const BatchLaunch& l,
                           hipStream_t st) {
  DGFAS_BATCH_LAUNCH(schwarz_batched_kernel, kStageSolve)
}
template <typename T>
void schwarz_overlap_add_batched(int pmax, const SchwarzArgs<T>& a, const BucketDesc<T>* bd, const BatchLaunch& l,
                                 hipStream_t st) {
  DGFAS_BATCH_LAUNCH(overlap_add_batched_kernel, kStageAdd)
}
#undef DGFAS_BATCH_LAUNCH
#undef DGFAS_BATCH_ONE

template void schwarz_solve_batched<double>(int, const SchwarzArgs<double>&, const BucketDesc<double>*,
                                            const BatchLaunch&, hipStream_t);
template void schwarz_solve_batched<float>(int, const SchwarzArgs<float>&, const BucketDesc<float>*,
                                           const BatchLaunch&, hipStream_t);
template void schwarz_overlap_add_batched<double>(int, const SchwarzArgs<double>&, const BucketDesc<double>*,
                                                  const BatchLaunch&, hipStream_t);
template void schwarz_overlap_add_batched<float>(int, const SchwarzArgs<float>&, const BucketDesc<float>*,
                                                 const BatchLaunch&, hipStream_t);

template void schwarz_solve<double>(int, int, const SchwarzArgs<double>&, hipStream_t);
template void schwarz_solve<float>(int, int, const SchwarzArgs<float>&, hipStream_t);
template void schwarz_overlap_add<double>(int, int, const SchwarzArgs<double>&, hipStream_t);
template void schwarz_overlap_add<float>(int, int, const SchwarzArgs<float>&, hipStream_t);

}  // namespace dgfas
