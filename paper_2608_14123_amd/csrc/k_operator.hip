// K1: sum-factorised SIPG operator apply / residual on curvilinear hexahedra
// (eq. helmholtz:dgm) and the one-time geometry kernels (Sec. 2.2).
//
// One workgroup takes EPB elements, one thread per node.  The element's u and
// the contravariant fluxes F_b = sum_c G_bc d_c u (G_bc = w J nu grad xi_b .
// grad xi_c) live in LDS.  Face terms use the identity
//   nu * omega * s * (n_out . grad xi_c) = +-G_bc / w_end     (normal axis b)
// so the own normal flux is F_b / w_end at the face node and the lifting term
// adds sigma * G_bc / w_end to F_c there; the neighbour's flux is rebuilt from
// its normal node line (L2-resident) and its metric at the shared face.  The
// three face axes are processed one after another so that no node is written
// by two tasks at once: the result is deterministic without atomics.
// On unstructured meshes (ORIENT) the neighbour may meet a face with any of its faces and any
// relative orientation (Sec. 5.1): its node line is then read at the orientation-mapped face
// node, and its tangential derivatives are the own face grid's, exchanged and negated as the
// orientation requires.
#include "device.hpp"
#include "kernels.hpp"


namespace dgfas {

template <int N>
struct OpShape {
  static constexpr int N2 = N * N, N3 = N * N * N;
  // LDS pitch of the xi_1 rows of volume tiles and of face rows: odd, so that the lanes of a
  // wavefront that read one column of rows hit distinct banks
  static constexpr int P = N | 1, V3 = N2 * P, F2 = N * P;
  static constexpr int EPB = (N3 >= 256) ? 1 : (256 / N3);
  static constexpr int THREADS = ((EPB * N3 + 63) / 64) * 64;
};

template <int N, typename T>
struct OpSmem {
  using S = OpShape<N>;
  T sD[S::N2];                // D[i][m] at i N + m
  T sDT[S::N2];               // D[i][m] at m N + i
  T su[S::EPB][S::V3];
  T sF[S::EPB][3][S::V3];
  T sTr[S::EPB][6][S::F2];    // neighbour trace
  T sRow[S::EPB][6][S::F2];   // direct face-row term
  T sSig[S::EPB][6][S::F2];   // lifting weight sigma
  double red[(S::THREADS + 63) / 64];   // per-wavefront partial sums of the fused dot product
};

// One tile: EPB elements of one right-hand side (logical block lbr).  Every thread of the
// workgroup passes every barrier; threads beyond EPB n^3 only take part in them, so the
// tile also runs inside wider batched workgroups.
// the neighbour's face node of own face node f under orientation code o (bit 0: exchange the
// face axes, bits 1 and 2: reverse the first and the second)
template <int N>
__device__ __forceinline__ int orient_face_node(int f, int o) {
  const int a = f / N, b = f - (f / N) * N;
  const int x = (o & 1) ? b : a, y = (o & 1) ? a : b;
  return ((o & 2) ? N - 1 - x : x) * N + ((o & 4) ? N - 1 - y : y);
}

// first face axis of face phi (layout: phi 0/1 -> (xi_3, xi_2), 2/3 -> (xi_3, xi_1), 4/5 -> (xi_2, xi_1))
__device__ __forceinline__ int face_axis_first(int phi) { return phi < 4 ? 2 : 1; }

// tid_in: the thread index when the caller passes it (the persistent batches), else threadIdx.x
// MORTAR: the level has faces between degrees (OpArgs::fmapE), whose terms the tile adds.
template <int N, typename T, bool ORIENT = false, bool MORTAR = false>
__device__ __forceinline__ void sipg_tile(const OpArgs<T>& a, const int lbr, OpSmem<N, T>& sm, int tid_in = -1) {
  using S = OpShape<N>;
  const int nrhs = a.nrhs, nel = a.nel, mode = a.mode;
  const T* __restrict__ u = a.u;
  const T* __restrict__ g = a.g;
  T* __restrict__ out = a.out;
  const T* __restrict__ G = a.G;
  const T* __restrict__ WJ = a.WJ;
  const T* __restrict__ pen = a.pen;
  const int* __restrict__ nbr = a.nbr;
  const int8_t* __restrict__ bc = a.bc;
  const T* __restrict__ Dg = a.D;
  const T kappa = a.kappa, inv_wend = a.inv_wend;
  constexpr int N2 = S::N2, N3 = S::N3, EPB = S::EPB, P = S::P, V3 = S::V3, F2 = S::F2;
  constexpr int TPT = (6 * N2 + N3 - 1) / N3;     // face tasks per thread
  // logical block = (element block, right-hand side) with the right-hand side fastest, so
  // that the batch of one element reads its geometry while it is resident in L2
  const int lb = lbr / nrhs;
  const int64_t ndof = a.ndof;
  const int64_t voff = (int64_t)(lbr - lb * nrhs) * ndof;
  u += voff;
  out += voff;
  if (g) g += voff;
  const int tid = tid_in >= 0 ? tid_in : (int)threadIdx.x;
  const int le = tid / N3;
  const int node = tid - le * N3;
  const int li = lb * EPB + le;
  const bool active = (le < EPB) && (li < nel);
  const int e = active ? (a.elist ? a.elist[li] : li) : 0;

  T(&sD)[N2] = sm.sD;
  T(&sDT)[N2] = sm.sDT;
  T(&su)[EPB][V3] = sm.su;
  T(&sF)[EPB][3][V3] = sm.sF;
  T(&sTr)[EPB][6][F2] = sm.sTr;
  T(&sRow)[EPB][6][F2] = sm.sRow;
  T(&sSig)[EPB][6][F2] = sm.sSig;
  const int i = node % N, j = (node / N) % N, k = node / N2;
  const int lnode = (k * N + j) * P + i;          // padded LDS slot of the thread's node

  const int64_t base = a.off ? a.off[e] : (int64_t)e * N3;
  const int64_t fbase = a.offF ? a.offF[e] : (int64_t)e * 6 * N2;
  // prologue: every load that needs only the element goes out in one batch (the D table, u,
  // the face tasks' neighbour ids, penalties and boundary codes, the metric, g) and nothing
  // uses them before the batch is issued, so that the tile waits for memory once before the
  // neighbour loads that need the neighbour ids
  T dv = 0;
  if (tid < N2) dv = Dg[tid];
  int en_t[TPT];
  T pen_t[TPT];
  int8_t bc_t[TPT];
  int fo_t[TPT];   // ORIENT: the neighbour's face | orientation << 3
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    en_t[k] = -1;
    pen_t[k] = 0;
    bc_t[k] = 0;
    fo_t[k] = 0;
  }
  T uval = 0, gval = 0;
  T gl[6] = {0, 0, 0, 0, 0, 0};
  if (active) {
    uval = u[base + node];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      const int t = node + k * N3;
      if (t < 6 * N2) {
        const int phi = t / N2;
        en_t[k] = nbr[(int64_t)e * 6 + phi];
        pen_t[k] = pen[fbase + t];
        bc_t[k] = bc[(int64_t)e * 6 + phi];
        if constexpr (ORIENT) fo_t[k] = a.nfo[(int64_t)e * 6 + phi];
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) gl[c] = G[c * ndof + base + node];
    if (mode == 0) gval = g[base + node];
  }
  if (tid < N2) {
    sD[tid] = dv;
    sDT[(tid % N) * N + tid / N] = dv;
  }
  if (active) su[le][lnode] = uval;
  // phase 0: the neighbour data of every face node (normal node line and metric row) is
  // loaded into registers here, as soon as the neighbour ids have arrived, and used from the
  // neighbour trace on.  On levels of several degrees the neighbour's degree and offset go
  // out together; a neighbour of another degree is left to the mortar face kernel (en = -2).
  T lnv[TPT][N], gn[TPT][3];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int t = node + k * N3;
#pragma unroll
    for (int m = 0; m < N; ++m) lnv[k][m] = 0;
    gn[k][0] = gn[k][1] = gn[k][2] = 0;
    if (!active || t >= 6 * N2) continue;
    const int phi = t / N2, f = t - phi * N2, ax = phi >> 1;
    int en = en_t[k];
    if (en < 0) continue;
    const int64_t nbase = a.off ? a.off[en] : (int64_t)en * N3;
    if (a.deg && a.deg[en] != N - 1) en = -2;
    en_t[k] = en;
    if (en >= 0) {
      const int phio = ORIENT ? (fo_t[k] & 7) : (phi ^ 1);
      const int fo = ORIENT ? orient_face_node<N>(f, fo_t[k] >> 3) : f;
      const int axo = ORIENT ? (phio >> 1) : ax;
      const int endo = (phio & 1) ? N - 1 : 0;
      const T* line = u + nbase + face_node<N>(phio, fo, 0);
      const int st = axis_stride<N>(axo);
      const int64_t gi = nbase + face_node<N>(phio, fo, endo);
#pragma unroll
      for (int c = 0; c < 3; ++c) gn[k][c] = G[sym_index(axo, c) * ndof + gi];
#pragma unroll
      for (int m = 0; m < N; ++m) lnv[k][m] = line[m * st];
    }
  }
  __syncthreads();

  // a wavefront is one xi_3 layer when N^2 = 64: D[k][m] and D[m][k] are then uniform and
  // come through the scalar cache instead of LDS
  constexpr bool kLayer = N * N == 64 && EPB == 1;
  const int ku = kLayer ? __builtin_amdgcn_readfirstlane(k) : k;
  // phase 1: reference derivatives and contravariant fluxes F_b = sum_c G_bc d_c u
  if (active) {
    T d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      d0 += sDT[m * N + i] * su[le][(k * N + j) * P + m];
      d1 += sDT[m * N + j] * su[le][(k * N + m) * P + i];
      d2 += (kLayer ? Dg[ku * N + m] : sDT[m * N + k]) * su[le][(m * N + j) * P + i];
    }
    sF[le][0][lnode] = gl[0] * d0 + gl[1] * d1 + gl[2] * d2;
    sF[le][1][lnode] = gl[1] * d0 + gl[3] * d1 + gl[4] * d2;
    sF[le][2][lnode] = gl[2] * d0 + gl[4] * d1 + gl[5] * d2;
  }
  // the neighbour's trace and normal derivative at every face node
  T dn_nb[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int t = node + k * N3;
    dn_nb[k] = 0;
    if (!active || t >= 6 * N2) continue;
    const int phi = t / N2, f = t - phi * N2;
    T tr = 0;
    if (en_t[k] >= 0) {
      const int phio = ORIENT ? (fo_t[k] & 7) : (phi ^ 1);
      const int endo = (phio & 1) ? N - 1 : 0;
      T dn = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const T v = lnv[k][m];
        dn += sD[endo * N + m] * v;
        if (m == endo) tr = v;
      }
      dn_nb[k] = dn;
    }
    sTr[le][phi][(f / N) * P + f % N] = tr;
  }
  __syncthreads();

  // phase 2: face terms per face node (no two tasks share an output slot)
#pragma unroll
  for (int kk = 0; kk < TPT; ++kk) {
    const int t = node + kk * N3;
    if (!active || t >= 6 * N2) continue;
    const int phi = t / N2, f = t - phi * N2, ax = phi >> 1;
    const int vi = face_node<N>(phi, f, (phi & 1) ? N - 1 : 0);
    const int lvi = (vi / N) * P + vi % N;
    const int fa = f / N, fb = f - fa * N, lf = fa * P + fb;
    const T sgn = (phi & 1) ? T(1) : T(-1);
    const T uo = su[le][lvi];
    const T qo = sgn * inv_wend * sF[le][ax][lvi];   // nu omega s n_out . grad u
    const T pf = pen_t[kk];
    T row = 0, sigma = 0;
    if (en_t[kk] >= 0) {
      T dlast = 0, dfirst = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        dlast += sDT[m * N + fb] * sTr[le][phi][fa * P + m];
        dfirst += sDT[m * N + fa] * sTr[le][phi][m * P + fb];
      }
      T du0, du1, du2;
      T qn;
      if constexpr (ORIENT) {
        // the neighbour's reference derivatives: along its normal from its node line, along its
        // face axes from the own face grid through the orientation
        const int phio = fo_t[kk] & 7, o = fo_t[kk] >> 3;
        const T dA = ((o & 2) ? T(-1) : T(1)) * ((o & 1) ? dlast : dfirst);
        const T dB = ((o & 4) ? T(-1) : T(1)) * ((o & 1) ? dfirst : dlast);
        const int an = phio >> 1, af = face_axis_first(phio);   // the third axis takes dB
        du0 = an == 0 ? dn_nb[kk] : (af == 0 ? dA : dB);
        du1 = an == 1 ? dn_nb[kk] : (af == 1 ? dA : dB);
        du2 = an == 2 ? dn_nb[kk] : (af == 2 ? dA : dB);
        const T fl = gn[kk][0] * du0 + gn[kk][1] * du1 + gn[kk][2] * du2;
        qn = ((phio & 1) ? T(1) : T(-1)) * inv_wend * fl;   // neighbour's outward flux
      } else {
        if (ax == 0) { du0 = dn_nb[kk]; du1 = dlast; du2 = dfirst; }
        else if (ax == 1) { du0 = dlast; du1 = dn_nb[kk]; du2 = dfirst; }
        else { du0 = dlast; du1 = dfirst; du2 = dn_nb[kk]; }
        const T fl = gn[kk][0] * du0 + gn[kk][1] * du1 + gn[kk][2] * du2;
        qn = -sgn * inv_wend * fl;                   // neighbour's outward flux
      }
      const T jmp = uo - sTr[le][phi][lf];
      row = pf * jmp - T(0.5) * (qo - qn);
      sigma = T(-0.5) * jmp;
    } else if (en_t[kk] == -1 && bc_t[kk] == 1) {    // Dirichlet: 2 mu nu omega s u - q, lifting -u
      row = pf * uo - qo;
      sigma = -uo;
    }
    sRow[le][phi][lf] = row;
    sSig[le][phi][lf] = sigma;
  }
  __syncthreads();

  // phase 3: every node collects the terms of the faces it lies on (its own slots)
  T rowsum = 0;
  if (active) {
    const int fidx[3] = {k * P + j, k * P + i, j * P + i};
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      int phi = -1;
      if (idx[ax] == 0) phi = 2 * ax;
      else if (idx[ax] == N - 1) phi = 2 * ax + 1;
      if (phi < 0) continue;
      rowsum += sRow[le][phi][fidx[ax]];
      const T sg = sSig[le][phi][fidx[ax]] * ((phi & 1) ? inv_wend : -inv_wend);
      sF[le][0][lnode] += sg * gl[sym_index(ax, 0)];
      sF[le][1][lnode] += sg * gl[sym_index(ax, 1)];
      sF[le][2][lnode] += sg * gl[sym_index(ax, 2)];
      if constexpr (MORTAR) {
        // a face to another degree: its row and lifting terms from the mortar face kernel
        const int kf = a.fmapE[(int64_t)e * 6 + phi];
        if (kf >= 0) {
          const T* __restrict__ r = a.fres + (int64_t)(lbr - lb * nrhs) * a.fres_stride + (int64_t)kf * kMortarFaceRes;
          const int ff = ax == 0 ? k * N + j : (ax == 1 ? k * N + i : j * N + i);
          rowsum += r[ff];
          sF[le][0][lnode] += r[81 + ff];
          sF[le][1][lnode] += r[162 + ff];
          sF[le][2][lnode] += r[243 + ff];
        }
      }
    }
  }
  __syncthreads();

  double pq = 0;
  if (active) {
    T acc = rowsum;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      acc += sD[m * N + i] * sF[le][0][(k * N + j) * P + m];
      acc += sD[m * N + j] * sF[le][1][(k * N + m) * P + i];
      acc += (kLayer ? Dg[m * N + ku] : sD[m * N + k]) * sF[le][2][(m * N + j) * P + i];
    }
    if (WJ) acc += kappa * WJ[base + node] * uval;
    out[base + node] = mode == 0 ? gval - acc : acc;
    if (a.dotp) pq = (double)uval * (double)acc;
  }
  if (a.dotp) {
    // u^T (A u) over the tile: wavefront butterfly, then the waves in order (deterministic)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) pq += __shfl_xor(pq, off);
    if ((tid & 63) == 0 && tid < S::THREADS) sm.red[tid >> 6] = pq;
    __syncthreads();
    if (tid == 0) {
      double s = 0;
      for (int w = 0; w < (S::THREADS + 63) / 64; ++w) s += sm.red[w];
      const int nlb = (nel + EPB - 1) / EPB;
      a.dotp[(int64_t)(lbr - lb * nrhs) * nlb + lb] = s;
    }
  }
}

template <int N, typename T, bool ORIENT, bool MORTAR>
__global__ void __launch_bounds__(OpShape<N>::THREADS)
sipg_apply_kernel(OpArgs<T> a) {
  using S = OpShape<N>;
  __shared__ OpSmem<N, T> sm;
  const int lbr = xcd_block(((a.nel + S::EPB - 1) / S::EPB) * a.nrhs);
  if (lbr < 0) return;
  sipg_tile<N, T, ORIENT, MORTAR>(a, lbr, sm);
}

template <int N, typename T>
void launch_sipg(const OpArgs<T>& a, hipStream_t st) {
  using S = OpShape<N>;
  const int nb = ((a.nel + S::EPB - 1) / S::EPB) * a.nrhs;
  if (a.nfo) hipLaunchKernelGGL((sipg_apply_kernel<N, T, true, false>), dim3(xcd_grid(nb)), dim3(S::THREADS), 0, st, a);
  else if (a.fmapE) hipLaunchKernelGGL((sipg_apply_kernel<N, T, false, true>), dim3(xcd_grid(nb)), dim3(S::THREADS), 0, st, a);
  else hipLaunchKernelGGL((sipg_apply_kernel<N, T, false, false>), dim3(xcd_grid(nb)), dim3(S::THREADS), 0, st, a);
}

// largest tile workspace of the degrees with n <= N
template <typename T, int N>
constexpr size_t op_smem_upto() {
  if constexpr (N < 2) {
    return 0;
  } else {
    constexpr size_t a = sizeof(OpSmem<N, T>), b = op_smem_upto<T, N - 1>();
    return a > b ? a : b;
  }
}

// all degrees up to NMAX - 1 in one launch; the workgroup is the widest tile's
template <int NMAX, typename T, bool PERSIST>
__global__ void __launch_bounds__(OpShape<NMAX>::THREADS)
sipg_batched_kernel(OpArgs<T> a, const BucketDesc<T>* __restrict__ bd, int nb, int ntiles) {
  __shared__ __align__(16) char smem[op_smem_upto<T, NMAX>()];
  // tiles dealt round-robin over the XCDs (the hardware order): the work list runs from the
  // largest degree to the smallest, and contiguous ranges per XCD would leave one XCD all
  // the large tiles.  The persistent form (fewer workgroups than tiles) strides through the
  // list, with a barrier between tiles for the shared memory.  It takes the thread index
  // through an opaque register copy in every tile, so that no degree branch's index arithmetic
  // is hoisted above the loop and kept live across it (that cost 48 VGPRs and scratch).
  auto tile = [&](int t) {
    int tid = -1;
    if constexpr (PERSIST) {
      tid = threadIdx.x;
      asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(tid));
    }
    const int k = find_bucket(bd, nb, kStageOp, t);
    OpArgs<T> x = a;
    x.nel = bd[k].nel;
    x.elist = bd[k].elist;
    x.D = bd[k].D;
    x.inv_wend = bd[k].inv_wend;
    const int lbr = t - bd[k].tile0[kStageOp];
    switch (bd[k].p) {
#define DGFAS_OPB(P)                                                                        \
  case P:                                                                                   \
    if constexpr (P + 1 <= NMAX) sipg_tile<P + 1, T, false, true>(x, lbr, *reinterpret_cast<OpSmem<P + 1, T>*>(smem), tid); \
    break;
      DGFAS_OPB(1) DGFAS_OPB(2) DGFAS_OPB(3) DGFAS_OPB(4) DGFAS_OPB(5) DGFAS_OPB(6) DGFAS_OPB(7) DGFAS_OPB(8)
#undef DGFAS_OPB
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

int stage_tiles(int stage, int p, int nel, int nrhs) {
  const int n3 = (p + 1) * (p + 1) * (p + 1);
  const int epb = n3 >= 256 ? 1 : 256 / n3;   // elements per tile of the operator and overlap add
  if (stage == kStageSolve) return nel * nrhs;
  return ((nel + epb - 1) / epb) * nrhs;
}

int stage_threads(int stage, int pmax) {
  const int n = pmax + 1, n3 = n * n * n;
  if (stage == kStageSolve) return n + 2 >= 9 ? 128 : 64;   // overlap 1: ns^2 lines, rounded to waves
  if (n3 >= 256) return ((n3 + 63) / 64) * 64;
  return 256;
}

template <typename T>
void sipg_apply_batched(int pmax, const OpArgs<T>& a, const BucketDesc<T>* bd, const BatchLaunch& l, hipStream_t st) {
  if (l.ntiles <= 0) return;
  const dim3 g(l.grid), b(stage_threads(kStageOp, pmax));
#define DGFAS_OPL(NM)                                                                                     \
  if (l.persistent) hipLaunchKernelGGL((sipg_batched_kernel<NM, T, true>), g, b, 0, st, a, bd, l.nb, l.ntiles); \
  else hipLaunchKernelGGL((sipg_batched_kernel<NM, T, false>), g, b, 0, st, a, bd, l.nb, l.ntiles);
  if (pmax <= 5) { DGFAS_OPL(6) }
  else if (pmax == 6) { DGFAS_OPL(7) }
  else if (pmax == 7) { DGFAS_OPL(8) }
  else { DGFAS_OPL(9) }
#undef DGFAS_OPL
}

template void sipg_apply_batched<double>(int, const OpArgs<double>&, const BucketDesc<double>*, const BatchLaunch&,
                                         hipStream_t);
template void sipg_apply_batched<float>(int, const OpArgs<float>&, const BucketDesc<float>*, const BatchLaunch&,
                                        hipStream_t);

template <typename T>
void sipg_apply(int p, const OpArgs<T>& a, hipStream_t st) {
  switch (p) {
    case 1: launch_sipg<2, T>(a, st); break;
    case 2: launch_sipg<3, T>(a, st); break;
    case 3: launch_sipg<4, T>(a, st); break;
    case 4: launch_sipg<5, T>(a, st); break;
    case 5: launch_sipg<6, T>(a, st); break;
    case 6: launch_sipg<7, T>(a, st); break;
    case 7: launch_sipg<8, T>(a, st); break;
    case 8: launch_sipg<9, T>(a, st); break;
    default: break;
  }
}

template void sipg_apply<double>(int, const OpArgs<double>&, hipStream_t);
template void sipg_apply<float>(int, const OpArgs<float>&, hipStream_t);

// ---------------------------------------------------------------------------
// Geometry (one-time): G_bc = w J nu grad xi_b . grad xi_c, w J, omega*s at face
// nodes (from the cross product of the two tangential columns of the Jacobian,
// i.e. tangential derivatives only), element volume and face areas, and the
// linear Legendre coefficients of the map (surrogate cuboid, Sec. 4.3.1).
template <int N>
__global__ void __launch_bounds__(OpShape<N>::THREADS)
geometry_kernel(GeoArgs g, const double* __restrict__ Dg, const double* __restrict__ w1,
                const double* __restrict__ x1, double nu) {
  using S = OpShape<N>;
  constexpr int N2 = S::N2, N3 = S::N3, EPB = S::EPB;
  const double* __restrict__ X = g.X;
  double* __restrict__ G = g.G;
  double* __restrict__ WJ = g.WJ;
  double* __restrict__ ws = g.ws;
  double* __restrict__ vol = g.vol;
  double* __restrict__ area = g.area;
  double* __restrict__ lin = g.lin;
  const int lb = blockIdx.x;
  const int tid = threadIdx.x;
  const int le = tid / N3;
  const int node = tid - le * N3;
  const int li = lb * EPB + le;
  const bool active = (le < EPB) && (li < g.nel);
  const int e = active ? (g.elist ? g.elist[li] : li) : 0;
  const int64_t base = g.off ? g.off[e] : (int64_t)e * N3;
  const int64_t fbase = g.offF ? g.offF[e] : (int64_t)e * 6 * N2;
  __shared__ double sX[EPB][3][N3];
  __shared__ double sWJ[EPB][N3];
  __shared__ double sWJnu[EPB][N3];
  __shared__ double sws[EPB][6][N2];
  if (active)
    for (int a = 0; a < 3; ++a) sX[le][a][node] = X[3 * base + (int64_t)a * N3 + node];
  __syncthreads();
  const int i = node % N, j = (node / N) % N, k = node / N2;
  if (active) {
    double J[3][3];
    for (int a = 0; a < 3; ++a) {
      double d0 = 0, d1 = 0, d2 = 0;
      for (int m = 0; m < N; ++m) {
        d0 += Dg[i * N + m] * sX[le][a][(k * N + j) * N + m];
        d1 += Dg[j * N + m] * sX[le][a][(k * N + m) * N + i];
        d2 += Dg[k * N + m] * sX[le][a][(m * N + j) * N + i];
      }
      J[a][0] = d0; J[a][1] = d1; J[a][2] = d2;
    }
    // cofactor matrix C[a][b] = d det / d J[a][b]; column b of C = J grad(xi_b) (times det)
    double C[3][3];
    C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    if (!(det > 0)) atomicOr(g.bad, 1);
    const double wq = w1[i] * w1[j] * w1[k];
    // grad xi_b = C[:, b] / det  ->  G_bc = w nu (C[:,b] . C[:,c]) / det, nu at the node
    const int64_t ndof = g.ndof, gi = base + node;
    const double nuq = g.nun ? g.nun[gi] : nu;
    const double sc = wq * nuq / det;
    double Gb[6];
    Gb[0] = sc * (C[0][0] * C[0][0] + C[1][0] * C[1][0] + C[2][0] * C[2][0]);
    Gb[1] = sc * (C[0][0] * C[0][1] + C[1][0] * C[1][1] + C[2][0] * C[2][1]);
    Gb[2] = sc * (C[0][0] * C[0][2] + C[1][0] * C[1][2] + C[2][0] * C[2][2]);
    Gb[3] = sc * (C[0][1] * C[0][1] + C[1][1] * C[1][1] + C[2][1] * C[2][1]);
    Gb[4] = sc * (C[0][1] * C[0][2] + C[1][1] * C[1][2] + C[2][1] * C[2][2]);
    Gb[5] = sc * (C[0][2] * C[0][2] + C[1][2] * C[1][2] + C[2][2] * C[2][2]);
    for (int c = 0; c < 6; ++c) G[c * ndof + gi] = Gb[c];
    WJ[gi] = wq * det;
    sWJ[le][node] = wq * det;
    sWJnu[le][node] = wq * det * nuq;
    // face nodes: omega * s with N = dx/dxi_t1 x dx/dxi_t2 (tangential columns of J)
    const int idx[3] = {i, j, k};
    for (int ax = 0; ax < 3; ++ax) {
      const int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
      if (idx[ax] != 0 && idx[ax] != N - 1) continue;
      const double nx = J[1][t1] * J[2][t2] - J[2][t1] * J[1][t2];
      const double ny = J[2][t1] * J[0][t2] - J[0][t1] * J[2][t2];
      const double nz = J[0][t1] * J[1][t2] - J[1][t1] * J[0][t2];
      const double s = sqrt(nx * nx + ny * ny + nz * nz) * w1[idx[t1]] * w1[idx[t2]];
      int f;
      if (ax == 0) f = k * N + j;
      else if (ax == 1) f = k * N + i;
      else f = j * N + i;
      if (idx[ax] == 0) sws[le][2 * ax][f] = s;
      if (idx[ax] == N - 1) sws[le][2 * ax + 1][f] = s;
    }
  }
  __syncthreads();
  // per-element sums: tasks 0..5 face areas, 6 volume, 7..15 linear Legendre coefficients
  for (int task = node; active && task < 16; task += N3) {
    if (task < 6) {
      double a = 0;
      for (int f = 0; f < N2; ++f) a += sws[le][task][f];
      area[(int64_t)e * 6 + task] = a;
      for (int f = 0; f < N2; ++f) ws[fbase + task * N2 + f] = sws[le][task][f];
    } else if (task == 6) {
      double v = 0, vn = 0;
      for (int t = 0; t < N3; ++t) {
        v += sWJ[le][t];
        vn += sWJnu[le][t];
      }
      vol[e] = v;
      if (g.nuavg) g.nuavg[e] = vn / v;
    } else {
      // coefficient of L_1(xi_b) L_0 L_0 in the Legendre expansion of coordinate a
      const int q = task - 7, a = q / 3, b = q % 3;
      double s = 0;
      if (N > 2) {   // GLL quadrature is exact for x * xi_b when p >= 2
        for (int t = 0; t < N3; ++t) {
          const int ti = t % N, tj = (t / N) % N, tk = t / N2;
          const int idx[3] = {ti, tj, tk};
          s += w1[ti] * w1[tj] * w1[tk] * sX[le][a][t] * x1[idx[b]];
        }
        s *= 0.375;
      } else {       // p = 1: mean half-difference along b of the trilinear map
        for (int t = 0; t < N3; ++t) {
          const int ti = t % N, tj = (t / N) % N, tk = t / N2;
          const int idx[3] = {ti, tj, tk};
          s += (idx[b] == 1 ? 0.125 : -0.125) * sX[le][a][t];
        }
      }
      lin[(int64_t)e * 9 + q] = s;
    }
  }
}

template <int N>
void launch_geometry(const GeoArgs& g, const double* D, const double* w, const double* x, double nu, hipStream_t st) {
  using S = OpShape<N>;
  const int nb = (g.nel + S::EPB - 1) / S::EPB;
  if (nb > 0) hipLaunchKernelGGL((geometry_kernel<N>), dim3(nb), dim3(S::THREADS), 0, st, g, D, w, x, nu);
}

void geometry(int p, const GeoArgs& g, const double* D, const double* w, const double* x, double nu,
              hipStream_t st) {
  switch (p) {
    case 1: launch_geometry<2>(g, D, w, x, nu, st); break;
    case 2: launch_geometry<3>(g, D, w, x, nu, st); break;
    case 3: launch_geometry<4>(g, D, w, x, nu, st); break;
    case 4: launch_geometry<5>(g, D, w, x, nu, st); break;
    case 5: launch_geometry<6>(g, D, w, x, nu, st); break;
    case 6: launch_geometry<7>(g, D, w, x, nu, st); break;
    case 7: launch_geometry<8>(g, D, w, x, nu, st); break;
    case 8: launch_geometry<9>(g, D, w, x, nu, st); break;
    default: break;
  }
}

// node of face phi at face-node index f (layout of face_node) and normal index t, degree n - 1
__device__ __forceinline__ int face_node_n(int n, int phi, int f, int t) {
  const int a = f / n, b = f % n, ax = phi >> 1;
  if (ax == 0) return (a * n + b) * n + t;
  if (ax == 1) return (a * n + t) * n + b;
  return (t * n + a) * n + b;
}

// Penalty factor per element-face node: interior mu_F max(nu-, nu+) omega s with
// mu_F = mu_star avg(p(p+1)/(2 h_perp)) over the two sides (each with its own degree),
// Dirichlet 2 mu nu omega s, Neumann 0; h_perp = vol / area (eq. helmholtz:dgm).  With a nodal
// nu (one degree), nu- and nu+ are the two sides' values at the face node.
// muf[e][phi] = mu_F nu (Dirichlet: 2 mu nu) for the face integration on mixed-degree faces.
__global__ void penalty_kernel(int E, int p, const int* __restrict__ deg, const int64_t* __restrict__ offF,
                               double mu_star, double nu, const double* __restrict__ nun,
                               const int* __restrict__ nbr, const int8_t* __restrict__ nfo,
                               const int8_t* __restrict__ bc, const double* __restrict__ vol,
                               const double* __restrict__ area, const double* __restrict__ ws,
                               double* __restrict__ pen, double* __restrict__ muf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)E * 6) return;
  const int e = (int)(t / 6), phi = (int)(t % 6);
  const int pe = deg ? deg[e] : p;
  const int N2 = (pe + 1) * (pe + 1);
  const double own = pe * (pe + 1) / (2.0 * (vol[e] / area[t]));
  const int en = nbr[t];
  // the neighbour's face and the relative orientation (unstructured meshes), else aligned
  const int phio = nfo && en >= 0 ? (nfo[t] & 7) : (phi ^ 1);
  const int ori = nfo && en >= 0 ? (nfo[t] >> 3) : 0;
  double fac = 0.0;
  if (en >= 0) {
    const int pn = deg ? deg[en] : p;
    const double oth = pn * (pn + 1) / (2.0 * (vol[en] / area[(int64_t)en * 6 + phio]));
    fac = mu_star * 0.5 * (own + oth);
  } else if (bc[t] == 1) {
    fac = 2.0 * mu_star * own;
  }
  if (muf) muf[t] = fac * nu;
  const int64_t fb = (offF ? offF[e] : (int64_t)e * 6 * N2) + (int64_t)phi * N2;
  if (!nun) {
    for (int f = 0; f < N2; ++f) pen[fb + f] = fac * nu * ws[fb + f];
    return;
  }
  const int n = pe + 1, N3 = N2 * n;
  const int end = (phi & 1) ? n - 1 : 0, endo = (phio & 1) ? n - 1 : 0;
  for (int f = 0; f < N2; ++f) {
    double nf = nun[(int64_t)e * N3 + face_node_n(n, phi, f, end)];
    if (en >= 0) {
      const int a = f / n, b = f % n;
      const int x = (ori & 1) ? b : a, y = (ori & 1) ? a : b;
      const int fo = ((ori & 2) ? n - 1 - x : x) * n + ((ori & 4) ? n - 1 - y : y);
      nf = fmax(nf, nun[(int64_t)en * N3 + face_node_n(n, phio, fo, endo)]);
    }
    pen[fb + f] = fac * nf * ws[fb + f];
  }
}

void penalty(int E, int p, const int* deg, const int64_t* offF, double mu_star, double nu, const double* nun,
             const int* nbr, const int8_t* nfo, const int8_t* bc, const double* vol, const double* area,
             const double* ws, double* pen, double* muf, hipStream_t st) {
  const int64_t n = (int64_t)E * 6;
  hipLaunchKernelGGL(penalty_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, E, p, deg, offF, mu_star,
                     nu, nun, nbr, nfo, bc, vol, area, ws, pen, muf);
}

}  // namespace dgfas

namespace dgfas {

// Right-hand side of eq. helmholtz:system:
//   b = w J f + Dirichlet faces (2 mu nu omega s u_D at the face node, lifting
//   -nu omega s u_D (n . grad phi_q)) + Neumann faces (omega s q_N).
template <int N>
__global__ void __launch_bounds__(OpShape<N>::THREADS)
rhs_kernel(RhsArgs r, const double* __restrict__ Dg, double inv_wend) {
  using S = OpShape<N>;
  constexpr int N2 = S::N2, N3 = S::N3, EPB = S::EPB;
  const double* __restrict__ f = r.f;
  const double* __restrict__ uD = r.uD;
  const double* __restrict__ qN = r.qN;
  double* __restrict__ b = r.b;
  const double* __restrict__ G = r.G;
  const double* __restrict__ WJ = r.WJ;
  const double* __restrict__ pen = r.pen;
  const double* __restrict__ ws = r.ws;
  const int* __restrict__ nbr = r.nbr;
  const int8_t* __restrict__ bc = r.bc;
  const int lb = blockIdx.x;
  const int tid = threadIdx.x;
  const int le = tid / N3, node = tid - le * N3;
  const int li = lb * EPB + le;
  const bool active = (le < EPB) && (li < r.nel);
  const int e = active ? (r.elist ? r.elist[li] : li) : 0;
  __shared__ double sD[N2];
  __shared__ double sL[EPB][3][N3];
  __shared__ double sRow[EPB][N3];
  for (int t = tid; t < N2; t += S::THREADS) sD[t] = Dg[t];
  const int64_t base = r.off ? r.off[e] : (int64_t)e * N3, ndof = r.ndof;
  const int64_t fbase = r.offF ? r.offF[e] : (int64_t)e * 6 * N2;
  if (active) {
    sL[le][0][node] = sL[le][1][node] = sL[le][2][node] = 0.0;
    sRow[le][node] = 0.0;
  }
  __syncthreads();
  for (int ax = 0; ax < 3; ++ax) {
    if (active) {
      for (int t = node; t < 2 * N2; t += N3) {
        const int s = t / N2, fn = t - s * N2;
        const int phi = 2 * ax + s;
        if (nbr[(int64_t)e * 6 + phi] >= 0) continue;
        const int vi = face_node<N>(phi, fn, (phi & 1) ? N - 1 : 0);
        const int8_t code = bc[(int64_t)e * 6 + phi];
        if (code == 1 && uD) {
          const double ud = uD[base + vi];
          const double sgn = (phi & 1) ? 1.0 : -1.0;
          sRow[le][vi] += pen[fbase + phi * N2 + fn] * ud;
          for (int c = 0; c < 3; ++c) sL[le][c][vi] += -ud * sgn * inv_wend * G[sym_index(ax, c) * ndof + base + vi];
        } else if (code == 2 && qN) {
          sRow[le][vi] += ws[fbase + phi * N2 + fn] * qN[base + vi];
        }
      }
    }
    __syncthreads();
  }
  if (active) {
    const int i = node % N, j = (node / N) % N, k = node / N2;
    double acc = WJ[base + node] * f[base + node] + sRow[le][node];
    for (int m = 0; m < N; ++m) {
      acc += sD[m * N + i] * sL[le][0][(k * N + j) * N + m];
      acc += sD[m * N + j] * sL[le][1][(k * N + m) * N + i];
      acc += sD[m * N + k] * sL[le][2][(m * N + j) * N + i];
    }
    b[base + node] = acc;
  }
}

template <int N>
void launch_rhs(const RhsArgs& r, const double* D, double inv_wend, hipStream_t st) {
  using S = OpShape<N>;
  const int nb = (r.nel + S::EPB - 1) / S::EPB;
  if (nb > 0) hipLaunchKernelGGL((rhs_kernel<N>), dim3(nb), dim3(S::THREADS), 0, st, r, D, inv_wend);
}

void rhs(int p, const RhsArgs& r, const double* D, double inv_wend, hipStream_t st) {
  switch (p) {
    case 1: launch_rhs<2>(r, D, inv_wend, st); break;
    case 2: launch_rhs<3>(r, D, inv_wend, st); break;
    case 3: launch_rhs<4>(r, D, inv_wend, st); break;
    case 4: launch_rhs<5>(r, D, inv_wend, st); break;
    case 5: launch_rhs<6>(r, D, inv_wend, st); break;
    case 6: launch_rhs<7>(r, D, inv_wend, st); break;
    case 7: launch_rhs<8>(r, D, inv_wend, st); break;
    case 8: launch_rhs<9>(r, D, inv_wend, st); break;
    default: break;
  }
}

}  // namespace dgfas
