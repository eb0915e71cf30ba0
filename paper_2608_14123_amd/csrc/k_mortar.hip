// K1m: SIPG face terms of faces between elements of different degree (mixed-degree
// levels; the paper keeps one degree per level, so this is an extension of
// eq. helmholtz:dgm).  Such a face is integrated with the GLL rule of the finer side:
// each side's trace and normal flux nu n.grad u are interpolated from its own face nodes
// to that grid, the penalty mu_F uses both degrees, and the test functions of the own
// element are its basis on the finer grid, so row terms are restricted back with the
// transposed interpolation.  The lifting term uses the restricted jump times the own
// nu n.grad xi_c, written into the transposed volume contractions as in sipg_apply.
//
// One workgroup per (face between degrees, right-hand side) computes the face's row and
// lifting terms on both sides' face grids into two result slots.  The operator kernels of the
// level, launched afterwards, add them to their own face terms (row at the face node, lifting
// into the contravariant fluxes before the transposed contractions), every output node written
// by one thread, so the result is deterministic.  Degrees are runtime values; the face's D and
// interpolation tables are staged in LDS.
#include "device.hpp"
#include "kernels.hpp"

namespace dgfas {

namespace {

constexpr int kMaxN = 9, kMaxN2 = 81;
// face kernel: one thread per face node of both sides in its first phases (n^2 + nn^2 <= 162)
constexpr int kFaceThreads = 192;

__device__ __forceinline__ int fnode(int n, int phi, int f, int t) {
  const int a = f / n, b = f - a * n, ax = phi >> 1;
  if (ax == 0) return (a * n + b) * n + t;
  if (ax == 1) return (a * n + t) * n + b;
  return (t * n + a) * n + b;
}

__device__ __forceinline__ int lstride(int n, int ax) { return ax == 0 ? 1 : (ax == 1 ? n : n * n); }

// phase B (traces, line derivatives and tables in LDS): tangential derivatives and the
// normal flux nu n_out . grad u (without omega s) at face node f
template <typename T>
__device__ T face_flux(int n, int phi, int f, const T* D, const T* tr, const T* dn, const T (*gr)[kMaxN2], T sgn,
                       T inv_wend, T wsf) {
  const int ax = phi >> 1, a = f / n, b = f - a * n;
  T dlast = 0, dfirst = 0;
  for (int m = 0; m < n; ++m) {
    dlast += D[b * n + m] * tr[a * n + m];
    dfirst += D[a * n + m] * tr[m * n + b];
  }
  T du0, du1, du2;
  if (ax == 0) { du0 = dn[f]; du1 = dlast; du2 = dfirst; }
  else if (ax == 1) { du0 = dlast; du1 = dn[f]; du2 = dfirst; }
  else { du0 = dlast; du1 = dfirst; du2 = dn[f]; }
  const T fl = gr[0][f] * du0 + gr[1][f] * du1 + gr[2][f] * du2;
  return sgn * inv_wend * fl / wsf;
}

// Face results per (right-hand side, face side): the row term and the three lifting rows on
// that side's face grid; a face task writes slot 2k (its own side) and 2k + 1 (the other)
constexpr int kFaceRes = kMortarFaceRes;

// One workgroup per (face between degrees, right-hand side): phases 0 to D of the face once,
// then the restriction to both sides' grids.  Seen from the other side the jump and flux
// differences change sign, so its finer-grid row and lifting fields are the negatives of
// this side's: both sides get what a task of their own would compute.
template <typename T>
__global__ void __launch_bounds__(kFaceThreads) mortar_face_kernel(MortarArgs<T> a) {
  const int lbr = xcd_block(a.nface * a.nrhs);
  if (lbr < 0) return;
  const int task = lbr / a.nrhs, rhs = lbr - task * a.nrhs;
  // the face's descriptor, built at set-up: one scalar load in place of a chain of dependent ones
  const int64_t* __restrict__ fd = a.fdesc + (int64_t)task * 8;
  const int ep = (int)fd[0], e = ep / 6, phi = ep - e * 6;
  const int tid = threadIdx.x;
  const T* __restrict__ u = a.u + (int64_t)rhs * a.ndof;
  T* __restrict__ res = reinterpret_cast<T*>(a.fres) + ((int64_t)rhs * 2 * a.nface + 2 * task) * kFaceRes;
  T* __restrict__ resn = res + kFaceRes;
  const int po = (int)fd[2], n = po + 1, n2 = n * n;
  const int64_t base = fd[4], fbase = fd[5];
  const T inv_wend_o = (T)(0.5 * po * (po + 1));

  __shared__ T sDo[kMaxN2], sDn[kMaxN2], sIo[kMaxN2], sIn[kMaxN2];
  __shared__ T to[kMaxN2], dno[kMaxN2], qo[kMaxN2], wso[kMaxN2], go[3][kMaxN2];
  __shared__ T tn[kMaxN2], dnn[kMaxN2], qn[kMaxN2], wsn[kMaxN2], gn[3][kMaxN2];
  __shared__ T x1[4][kMaxN2];                 // half-interpolated own t, own q, nb t, nb q
  __shared__ T rF[kMaxN2], sF[kMaxN2];        // row term and lifting weight on the finer grid
  __shared__ T y1[4][kMaxN2];                 // half-restricted row and lifting weight, both sides

  const int en = (int)fd[1];
  const int pn = (int)fd[3];
  const int nn = pn + 1, nn2 = nn * nn, nF = nn > n ? nn : n, nF2 = nF * nF;
  const int phin = phi ^ 1, ax = phi >> 1, endo = (phi & 1) ? n - 1 : 0, endn = (phin & 1) ? nn - 1 : 0;
  const int pF = nF - 1;
  const T sgn = (phi & 1) ? T(1) : T(-1);
  const T inv_wend_n = (T)(0.5 * pn * (pn + 1));
  const T mu = (T)a.muf[(int64_t)e * 6 + phi];
  const int64_t nbase = fd[6], nfbase = fd[7];

  // 0: every global load of the face first (both sides' normal lines, metric rows, omega s)
  // and the face's tables into LDS; one face-node task per thread (n^2 + nn^2 <= 162)
  const bool own_t = tid < n2, nb_t = !own_t && tid < n2 + nn2;
  const int f = own_t ? tid : tid - n2;
  T line[kMaxN], g3[3] = {0, 0, 0}, wsv = 0;
  if (nb_t) {
    const int v0 = fnode(nn, phin, f, 0), st = lstride(nn, ax);
#pragma unroll
    for (int m = 0; m < kMaxN; ++m) line[m] = m < nn ? u[nbase + v0 + m * st] : T(0);
    const int vi = v0 + endn * st;
#pragma unroll
    for (int c = 0; c < 3; ++c) g3[c] = a.G[sym_index(ax, c) * a.ndof + nbase + vi];
    wsv = (T)a.ws[nfbase + phin * nn2 + f];
  } else if (own_t) {
    const int v0 = fnode(n, phi, f, 0), st = lstride(n, ax);
#pragma unroll
    for (int m = 0; m < kMaxN; ++m) line[m] = m < n ? u[base + v0 + m * st] : T(0);
    const int vi = v0 + endo * st;
#pragma unroll
    for (int c = 0; c < 3; ++c) g3[c] = a.G[sym_index(ax, c) * a.ndof + base + vi];
    wsv = (T)a.ws[fbase + phi * n2 + f];
  }
  // the four tables: every load before the LDS stores
  for (int t = tid; t < kMaxN2; t += kFaceThreads) {
    double d_o = 0, d_n = 0, i_o = 0, i_n = 0;
    if (t < n2) d_o = a.Dall[(po - 1) * kMaxN2 + t];
    if (t < nn2) d_n = a.Dall[(pn - 1) * kMaxN2 + t];
    if (t < nF * n) i_o = a.Iall[((po - 1) * 8 + (pF - 1)) * kMaxN2 + t];     // nF x n
    if (t < nF * nn) i_n = a.Iall[((pn - 1) * 8 + (pF - 1)) * kMaxN2 + t];    // nF x nn
    if (t < n2) sDo[t] = (T)d_o;
    if (t < nn2) sDn[t] = (T)d_n;
    if (t < nF * n) sIo[t] = (T)i_o;
    if (t < nF * nn) sIn[t] = (T)i_n;
  }
  __syncthreads();
  // A: traces and normal-line derivatives of both sides
  if (own_t) {
    T d = 0, tv = 0;
#pragma unroll
    for (int m = 0; m < kMaxN; ++m) {
      if (m < n) d += sDo[endo * n + m] * line[m];
      if (m == endo) tv = line[m];
    }
    to[f] = tv;
    dno[f] = d;
    wso[f] = wsv;
    for (int c = 0; c < 3; ++c) go[c][f] = g3[c];
  } else if (nb_t) {
    T d = 0, tv = 0;
#pragma unroll
    for (int m = 0; m < kMaxN; ++m) {
      if (m < nn) d += sDn[endn * nn + m] * line[m];
      if (m == endn) tv = line[m];
    }
    tn[f] = tv;
    dnn[f] = d;
    wsn[f] = wsv;
    for (int c = 0; c < 3; ++c) gn[c][f] = g3[c];
  }
  __syncthreads();
  // B: normal fluxes (each side's outward normal)
  if (own_t) qo[f] = face_flux<T>(n, phi, f, sDo, to, dno, go, sgn, inv_wend_o, wso[f]);
  else if (nb_t) qn[f] = face_flux<T>(nn, phin, f, sDn, tn, dnn, gn, -sgn, inv_wend_n, wsn[f]);
  __syncthreads();
  // C: first interpolation step X1[i][b] = sum_a I[i][a] X[a][b] for the four face fields
  for (int t = tid; t < 2 * nF * n + 2 * nF * nn; t += kFaceThreads) {
    int s = t, which, w;
    if (s < 2 * nF * n) { which = s / (nF * n); s -= which * nF * n; w = n; }
    else { s -= 2 * nF * n; which = 2 + s / (nF * nn); s -= (which - 2) * nF * nn; w = nn; }
    const int i = s / w, b = s - i * w;
    const T* I = which < 2 ? sIo : sIn;
    const T* X = which == 0 ? to : (which == 1 ? qo : (which == 2 ? tn : qn));
    T v = 0;
    for (int q = 0; q < w; ++q) v += I[i * w + q] * X[q * w + b];
    x1[which][i * w + b] = v;
  }
  __syncthreads();
  // D: second step and the differences on the finer grid
  for (int t = tid; t < nF2; t += kFaceThreads) {
    const int i = t / nF, j = t - i * nF;
    T t_o = 0, q_o = 0, t_n = 0, q_n = 0;
    for (int b = 0; b < n; ++b) {
      const T ij = sIo[j * n + b];
      t_o += x1[0][i * n + b] * ij;
      q_o += x1[1][i * n + b] * ij;
    }
    for (int b = 0; b < nn; ++b) {
      const T ij = sIn[j * nn + b];
      t_n += x1[2][i * nn + b] * ij;
      q_n += x1[3][i * nn + b] * ij;
    }
    // omega s of the finer side, in its own face-node order (shared orientation)
    const T wF = n > nn ? wso[t] : wsn[t];
    const T jt = t_o - t_n, jq = q_o - q_n;
    rF[t] = wF * (mu * jt - T(0.5) * jq);
    sF[t] = T(-0.5) * wF * jt;
  }
  __syncthreads();
  // E: restriction, first step Y1[a][j] = sum_i I[i][a] F[i][j], own side (I = Io, F) and
  // other side (I = In, -F)
  for (int t = tid; t < 2 * n * nF + 2 * nn * nF; t += kFaceThreads) {
    if (t < 2 * n * nF) {
      const int which = t / (n * nF), s = t - which * n * nF;
      const int aa = s / nF, j = s - aa * nF;
      const T* F = which == 0 ? rF : sF;
      T v = 0;
      for (int i = 0; i < nF; ++i) v += sIo[i * n + aa] * F[i * nF + j];
      y1[which][aa * nF + j] = v;
    } else {
      const int s0 = t - 2 * n * nF, which = s0 / (nn * nF), s = s0 - which * nn * nF;
      const int aa = s / nF, j = s - aa * nF;
      const T* F = which == 0 ? rF : sF;
      T v = 0;
      for (int i = 0; i < nF; ++i) v += sIn[i * nn + aa] * (-F[i * nF + j]);
      y1[2 + which][aa * nF + j] = v;
    }
  }
  __syncthreads();
  // F: second step; the lifting weight divided by the side's omega s times its metric row
  // (the other side's outward normal is -n); row and lifting rows go to the result slots
  for (int t = tid; t < n2 + nn2; t += kFaceThreads) {
    if (t < n2) {
      const int aa = t / n, b = t - aa * n;
      T r = 0, sgm = 0;
      for (int j = 0; j < nF; ++j) {
        const T ij = sIo[j * n + b];
        r += y1[0][aa * nF + j] * ij;
        sgm += y1[1][aa * nF + j] * ij;
      }
      res[t] = r;
      const T sc = sgm / wso[t] * sgn * inv_wend_o;
      for (int c = 0; c < 3; ++c) res[(1 + c) * kMaxN2 + t] = sc * go[c][t];
    } else {
      const int tn2 = t - n2, aa = tn2 / nn, b = tn2 - aa * nn;
      T r = 0, sgm = 0;
      for (int j = 0; j < nF; ++j) {
        const T ij = sIn[j * nn + b];
        r += y1[2][aa * nF + j] * ij;
        sgm += y1[3][aa * nF + j] * ij;
      }
      resn[tn2] = r;
      const T sc = sgm / wsn[tn2] * (-sgn) * inv_wend_n;
      for (int c = 0; c < 3; ++c) resn[(1 + c) * kMaxN2 + tn2] = sc * gn[c][tn2];
    }
  }
}

}  // namespace

template <typename T>
void sipg_mortar_faces(const MortarArgs<T>& a, hipStream_t st) {
  if (a.nface <= 0) return;
  hipLaunchKernelGGL((mortar_face_kernel<T>), dim3(xcd_grid(a.nface * a.nrhs)), dim3(kFaceThreads), 0, st, a);
}

template void sipg_mortar_faces<double>(const MortarArgs<double>&, hipStream_t);
template void sipg_mortar_faces<float>(const MortarArgs<float>&, hipStream_t);

}  // namespace dgfas
