// K2m: the subdomain solve of the FP32 correction-form smoother with its six tensor
// contractions (Sec. 4.3.1, fast diagonalisation) on the matrix cores, in two forms:
//  - BF16: v_mfma_f32_16x16x16bf16_1k, operands rounded to BF16, products accumulated in
//    FP32; the division by the surrogate eigenvalue sums is done on the registers between
//    the two xi_3 contractions, whose result layout is the next B operand layout;
//  - FP32: v_mfma_f32_16x16x4f32 with FP32 operands, ceil(ns / 4) products per block and
//    every contraction through the LDS tile.
// One xi_3 column per thread in gather and scatter (one wavefront per subdomain for
// ns^2 <= 64, else two taking alternate blocks of 16 tile lines in the contractions;
// overlap m = 1, ns <= 11).  The tile stays in LDS in FP32; a contraction along direction d
// is OUT(c, line) = sum_q M(c, q) IN(q, line) over the ns^2 tile lines of that direction,
// 16 lines per MFMA block (M = S_d^T going forward, S_d coming back); the eigenvector tables
// sit in LDS zero-padded to 16 x 16.  Gather and weighted scatter follow the vector kernel.
#include "device.hpp"
#include "kernels.hpp"

namespace dgfas {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// FP32 -> BF16 with round-to-nearest-even (the hardware conversion on gfx950)
__device__ __forceinline__ short to_bf16s(float f) {
  return __builtin_bit_cast(short, (__bf16)f);
}

// one wavefront per subdomain while a thread per xi_3 column fits in it, else two
template <int NS>
constexpr int mf_threads() { return NS * NS <= 64 ? 64 : 128; }

template <int N, int M, bool kBf16>
__global__ void __launch_bounds__(mf_threads<N + 2 * M>()) schwarz_mfma_kernel(SchwarzArgs<float> a) {
  constexpr int NS = N + 2 * M, LS = NS | 1, NL = NS * NS, NCB = (NL + 15) / 16;
  constexpr int kMfThreads = mf_threads<NS>(), NW = kMfThreads / 64, NCW = (NCB + NW - 1) / NW;
  constexpr Regions<N, M> R{};
  static_assert(NS <= 16 && NL <= kMfThreads, "one 16x16x16 MFMA per tile line, one column per thread");
  const int lbr = xcd_block(a.nel * a.nrhs);
  if (lbr < 0) return;
  const int li = lbr / a.nrhs, rhs = lbr - li * a.nrhs;
  const int e = a.elist ? a.elist[li] : li;
  a.r += (int64_t)rhs * a.ndof;
  a.z += (int64_t)rhs * a.ndof;
  a.O += (int64_t)rhs * a.nin;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, tid = threadIdx.x;
  const int64_t ebase = a.off ? a.off[e] : (int64_t)e * (N * N * N);

  constexpr int TILE = NS * NS * LS;
  __shared__ float tile[TILE + kMfThreads];   // the tile, then one dump slot per thread
  __shared__ float sS[3][16 * 16];            // eigenvector tables zero-padded to 16 x 16
  __shared__ float sW[3][NS];
  __shared__ float sLam[3][16];
  __shared__ int sMap[3][NS];
  __shared__ int sNb[27];
  __shared__ int sOff[27];

  int vv[3];
  for (int d = 0; d < 3; ++d) vv[d] = __builtin_amdgcn_readfirstlane(a.var[(int64_t)e * 3 + d]);
  for (int t = tid; t < 3 * NS; t += kMfThreads) {
    const int d = t / NS, q = t - d * NS;
    sW[d][q] = a.W[vv[d] * NS + q];
    sLam[d][q] = a.lam[vv[d] * NS + q];
    sMap[d][q] = a.map1d[vv[d] * NS + q];
  }
  for (int t = tid; t < 3 * 256; t += kMfThreads) {
    const int d = t >> 8, i = (t >> 4) & 15, j = t & 15;
    sS[d][t & 255] = (i < NS && j < NS) ? a.S[vv[d] * NS * NS + i * NS + j] : 0.f;
  }
  for (int t = tid; t < 3 * 16; t += kMfThreads)
    if ((t & 15) >= NS) sLam[t >> 4][t & 15] = 0.f;
  if (tid < 27) {
    int nb = a.nb27[(int64_t)e * 27 + tid];
    if (nb >= 0 && a.deg && a.deg[nb] != N - 1) nb = -1;   // another degree: zero fill, no scatter
    sNb[tid] = nb;
    sOff[tid] = R.off[tid];
  }
  const float g0 = a.gco[(int64_t)e * 4 + 0], g1 = a.gco[(int64_t)e * 4 + 1];
  const float g2 = a.gco[(int64_t)e * 4 + 2], g3 = a.gco[(int64_t)e * 4 + 3];
  __syncthreads();
  int m3u[NS];
#pragma unroll
  for (int s3 = 0; s3 < NS; ++s3) m3u[s3] = __builtin_amdgcn_readfirstlane(sMap[2][s3]);

  // gather r_s = R_s r, one xi_3 column (c1, c2) per lane and pass
  for (int col = tid; col < NL; col += kMfThreads) {
    const int c1 = col % NS, c2 = col / NS;
    const int m1 = sMap[0][c1], m2 = sMap[1][c2];
    int64_t cb[3];
#pragma unroll
    for (int d3 = 0; d3 < 3; ++d3) {
      cb[d3] = -1;
      if (m1 >= 0 && m2 >= 0) {
        const int src = sNb[d3 * 9 + (m2 >> 6) * 3 + (m1 >> 6)];
        if (src >= 0)
          cb[d3] = (a.off ? a.off[src] : (int64_t)src * (N * N * N)) + (m2 & 63) * N + (m1 & 63);
      }
    }
    float vals[NS];
#pragma unroll
    for (int s3 = 0; s3 < NS; ++s3) {
      const int m3 = m3u[s3];
      vals[s3] = 0.f;
      if (m3 >= 0) {
        const int64_t b = cb[m3 >> 6];
        if (b >= 0) vals[s3] = a.r[b + (m3 & 63) * (N * N)];
      }
    }
#pragma unroll
    for (int s3 = 0; s3 < NS; ++s3) tile[(s3 * NS + c2) * LS + c1] = vals[s3];
  }
  __syncthreads();

  if constexpr (!kBf16) {
    // FP32 matrix cores (v_mfma_f32_16x16x4f32): the six contractions one after another,
    // each as ceil(ns / 4) accumulating products of 16 x 4 blocks of M by 4 x 16 blocks of
    // tile lines.  A: lane holds M[row][4 c + kk], B: lane holds IN[4 c + kk][line], result:
    // lane holds OUT[4 kk + j][line] (kk = lane / 16), which is not the B layout, so every
    // contraction goes through the LDS tile.
    constexpr int KB = (NS + 3) / 4;
    const int row = lane & 15, kk = lane >> 4, kq = 4 * kk;
#pragma unroll 1
    for (int step = 0; step < 6; ++step) {
      const int dir = step < 3 ? step : 5 - step;
      const bool fwd = step < 3;
      float av[KB];
#pragma unroll
      for (int c = 0; c < KB; ++c) {
        const int q = 4 * c + kk;
        av[c] = fwd ? sS[dir][q * 16 + row] : sS[dir][row * 16 + q];
      }
      const int sh = dir == 2 ? LS : NS * LS, sl = dir == 0 ? LS : 1;
      const int sq = dir == 0 ? 1 : (dir == 1 ? LS : NS * LS);
      int lb[NCW];
      bool lok[NCW];
#pragma unroll
      for (int k = 0; k < NCW; ++k) {
        const int line = (NW * k + wv) * 16 + row;
        lok[k] = line < NL;
        lb[k] = lok[k] ? (line / NS) * sh + (line % NS) * sl : 0;
      }
      // every block is read before any is written (in-place contraction)
      float bv[NCW][KB];
#pragma unroll
      for (int k = 0; k < NCW; ++k) {
#pragma unroll
        for (int c = 0; c < KB; ++c) {
          const int q = 4 * c + kk;
          const bool ok = lok[k] && q < NS;
          const float v = tile[ok ? lb[k] + q * sq : 0];
          bv[k][c] = ok ? v : 0.f;
        }
      }
      v4f acc[NCW];
#pragma unroll
      for (int k = 0; k < NCW; ++k) {
        acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < KB; ++c) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c], bv[k][c], acc[k], 0, 0, 0);
      }
#pragma unroll
      for (int k = 0; k < NCW; ++k) {
        const int line = (NW * k + wv) * 16 + row;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = kq + j;
          const bool ok = lok[k] && c < NS;
          float v = acc[k][j];
          if (step == 2 && ok)   // divide by the surrogate eigenvalue sum of (s1, s2, s3)
            v = v / (g0 + g1 * sLam[0][line % NS] + g2 * sLam[1][line / NS] + g3 * sLam[2][c]);
          tile[ok ? lb[k] + c * sq : TILE + tid] = v;
        }
      }
      __syncthreads();
    }
  } else {
    // six contractions: xi_1 S1^T, xi_2 S2^T, xi_3 S3^T (then 1/D), xi_3 S3, xi_2 S2, xi_1 S1,
    // in five phases: the two xi_3 contractions share their lines, and the MFMA result layout
    // (lane holds OUT[kq + j][line]) is the B operand layout, so the second one takes the
    // first one's result from registers.
    const int row = lane & 15, kq = 4 * (lane >> 4);
    // A operand: lane holds M[row][kq + i], M = S_d^T (fwd) or S_d
    auto a_operand = [&](int dir, bool fwd) {
      v4s av;
  #pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = kq + i;
        av[i] = to_bf16s(fwd ? sS[dir][q * 16 + row] : sS[dir][row * 16 + q]);
      }
      return av;
    };
  #pragma unroll 1
    for (int ph = 0; ph < 5; ++ph) {
      const int dir = ph < 3 ? ph : 4 - ph;
      const v4s av = a_operand(dir, ph <= 2);
      // slot of position q on the line (hi, lo) of direction dir: hi * sh + lo * sl + q * sq
      const int sh = dir == 2 ? LS : NS * LS, sl = dir == 0 ? LS : 1;
      const int sq = dir == 0 ? 1 : (dir == 1 ? LS : NS * LS);
      int lb[NCW];
      bool lok[NCW];
  #pragma unroll
      for (int k = 0; k < NCW; ++k) {
        const int line = (NW * k + wv) * 16 + row;
        lok[k] = line < NL;
        lb[k] = lok[k] ? (line / NS) * sh + (line % NS) * sl + kq * sq : 0;
      }
      // all column blocks are read before any is written: the lines of a direction partition
      // the tile, so the contraction is done in place; the wavefronts take alternate blocks
      v4s bv[NCW];
  #pragma unroll
      for (int k = 0; k < NCW; ++k) {
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool ok = lok[k] && kq + i < NS;
          const float v = tile[ok ? lb[k] + i * sq : 0];
          bv[k][i] = to_bf16s(ok ? v : 0.f);
        }
      }
      v4f acc[NCW];
  #pragma unroll
      for (int k = 0; k < NCW; ++k)
        acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv[k], v4f{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      if (ph == 2) {
        // divide by the surrogate eigenvalue sums of (s1, s2, s3) = (line % ns, line / ns, c),
        // then contract with S3
        const v4s av3 = a_operand(2, false);
        float l3[4];
  #pragma unroll
        for (int j = 0; j < 4; ++j) l3[j] = g3 * sLam[2][kq + j];
  #pragma unroll
        for (int k = 0; k < NCW; ++k) {
          const int line = (NW * k + wv) * 16 + row;
          const bool okl = line < NL;
          const float base = g0 + g1 * sLam[0][okl ? line % NS : 0] + g2 * sLam[1][okl ? line / NS : 0];
  #pragma unroll
          for (int j = 0; j < 4; ++j) {
            // the quotient is rounded to BF16 next, so the hardware reciprocal (1 ulp) suffices
            const float v = acc[k][j] * __builtin_amdgcn_rcpf(base + l3[j]);
            bv[k][j] = to_bf16s(okl && kq + j < NS ? v : 0.f);
          }
          acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av3, bv[k], v4f{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        }
      }
  #pragma unroll
      for (int k = 0; k < NCW; ++k) {
  #pragma unroll
        for (int j = 0; j < 4; ++j) tile[(lok[k] && kq + j < NS) ? lb[k] + j * sq : TILE + tid] = acc[k][j];
      }
      __syncthreads();
    }
  }

  // weighted scatter, one xi_3 column per lane and pass
  for (int col = tid; col < NL; col += kMfThreads) {
    const int c1 = col % NS, c2 = col / NS;
    const int m1 = sMap[0][c1], m2 = sMap[1][c2];
    if (m1 < 0 || m2 < 0) continue;
    const int d1 = (m1 >> 6) - 1, d2 = (m2 >> 6) - 1, l1 = m1 & 63, l2 = m2 & 63;
    const float w12 = sW[0][c1] * sW[1][c2];
    int64_t db[3], nbase[3];   // nbase: the column's node (l1, l2, 0) in the receiving element
    int ds[3];
#pragma unroll
    for (int d3i = 0; d3i < 3; ++d3i) {
      const int d3 = d3i - 1;
      db[d3i] = -1;
      ds[d3i] = 0;
      nbase[d3i] = 0;
      if (d1 == 0 && d2 == 0 && d3 == 0) {
        db[d3i] = ebase + l2 * N + l1;
        ds[d3i] = N * N;
        nbase[d3i] = db[d3i];
      } else {
        const int dest = sNb[d3i * 9 + (d2 + 1) * 3 + (d1 + 1)];
        if (dest >= 0) {
          nbase[d3i] = (a.off ? a.off[dest] : (int64_t)dest * (N * N * N)) + l2 * N + l1;
          const int r = (1 - d3) * 9 + (1 - d2) * 3 + (1 - d1);
          const int cc1 = d1 < 0 ? l1 - (N - M) : l1, cc2 = d2 < 0 ? l2 - (N - M) : l2;
          const int x1 = d1 ? M : N, x2 = d2 ? M : N;
          ds[d3i] = x2 * x1;
          db[d3i] = (a.offO ? a.offO[dest] : (int64_t)dest * R.size) + sOff[r] + cc2 * x1 + cc1;
        }
      }
    }
#pragma unroll
    for (int s3 = 0; s3 < NS; ++s3) {
      const int m3 = m3u[s3];
      if (m3 < 0) continue;
      const int d3i = m3 >> 6, l3 = m3 & 63;
      float v = w12 * sW[2][s3] * tile[(s3 * NS + c2) * LS + c1];
      const int64_t base = db[d3i];
      if (base < 0) continue;
      if (a.cinv) v *= a.cinv[nbase[d3i] + l3 * (N * N)];   // normalised weight
      const int c3 = d3i == 0 ? l3 - (N - M) : l3;
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

template <int N>
void launch_mfma(const SchwarzArgs<float>& a, bool bf16, hipStream_t st) {
  if (bf16)
    hipLaunchKernelGGL((schwarz_mfma_kernel<N, 1, true>), dim3(xcd_grid(a.nel * a.nrhs)), dim3(mf_threads<N + 2>()),
                       0, st, a);
  else
    hipLaunchKernelGGL((schwarz_mfma_kernel<N, 1, false>), dim3(xcd_grid(a.nel * a.nrhs)), dim3(mf_threads<N + 2>()),
                       0, st, a);
}

}  // namespace

bool schwarz_solve_mfma(int p, int m, const SchwarzArgs<float>& a, bool bf16, hipStream_t st) {
  if (m != 1 || a.sel || a.corr || a.unweighted) return false;
  switch (p) {
    case 1: launch_mfma<2>(a, bf16, st); return true;
    case 2: launch_mfma<3>(a, bf16, st); return true;
    case 3: launch_mfma<4>(a, bf16, st); return true;
    case 4: launch_mfma<5>(a, bf16, st); return true;
    case 5: launch_mfma<6>(a, bf16, st); return true;
    case 6: launch_mfma<7>(a, bf16, st); return true;
    case 7: launch_mfma<8>(a, bf16, st); return true;
    case 8: launch_mfma<9>(a, bf16, st); return true;
    default: return false;
  }
}

}  // namespace dgfas
