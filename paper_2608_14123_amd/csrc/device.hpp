// Device-side helpers shared by the HIP kernels of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgfas {

// XCD-aware block remap: the hardware deals consecutive workgroup ids round-robin
// over the 8 XCDs; remapping gives every XCD a contiguous range of logical blocks
// so that neighbouring elements share an L2.  Returns -1 for padding blocks.
__device__ __forceinline__ int xcd_block(int n_logical) {
  const int per = (n_logical + 7) / 8;
  const int b = blockIdx.x;
  const int lb = (b & 7) * per + (b >> 3);
  return lb < n_logical ? lb : -1;
}

inline int xcd_grid(int n_logical) { return 8 * ((n_logical + 7) / 8); }

// bucket of tile t (buckets ordered by their first tile; uniform over the workgroup)
template <typename D>
__device__ __forceinline__ int find_bucket(const D* __restrict__ bd, int nb, int stage, int t) {
  int k = 0;
  while (k + 1 < nb && bd[k + 1].tile0[stage] <= t) ++k;
  return k;
}

// Volume index of face node f = (a, b) of face phi (layout: phi 0/1 -> (k, j),
// 2/3 -> (k, i), 4/5 -> (j, i)) with the normal index set to `t`.
template <int N>
__device__ __forceinline__ int face_node(int phi, int f, int t) {
  const int a = f / N, b = f % N;
  const int ax = phi >> 1;
  if (ax == 0) return (a * N + b) * N + t;
  if (ax == 1) return (a * N + t) * N + b;
  return (t * N + a) * N + b;
}

// stride of the normal line of axis ax
template <int N>
__device__ __forceinline__ constexpr int axis_stride(int ax) {
  return ax == 0 ? 1 : (ax == 1 ? N : N * N);
}

// index of symmetric metric component (b, c) in G[6] = {00, 01, 02, 11, 12, 22}; written
// without recursion, which the compiler turns into a per-lane loop for run-time axes
__device__ __forceinline__ constexpr int sym_index(int b, int c) {
  const int lo = b < c ? b : c, hi = b < c ? c : b;
  return lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
}

// offsets of the 26 overlap regions (region index (d3+1)*9 + (d2+1)*3 + (d1+1); 13 unused)
template <int N, int M>
struct Regions {
  int off[27];
  int size;
  __host__ __device__ constexpr Regions() : off(), size(0) {
    int o = 0;
    for (int r = 0; r < 27; ++r) {
      off[r] = o;
      if (r == 13) continue;
      const int d1 = r % 3 - 1, d2 = (r / 3) % 3 - 1, d3 = r / 9 - 1;
      o += (d1 ? M : N) * (d2 ? M : N) * (d3 ? M : N);
    }
    size = o;
  }
};

}  // namespace dgfas
