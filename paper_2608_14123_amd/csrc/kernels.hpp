// Host-side launch interface of the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgfas {

template <typename T>
struct OpArgs {
  int E = 0;
  int nrhs = 1;               // vectors are [nrhs][E (p+1)^3]
  const T* u = nullptr;
  const T* g = nullptr;
  T* out = nullptr;
  int mode = 0;               // 0: out = g - A u, 1: out = A u
  const T* G = nullptr;       // [6][ndof]
  const T* WJ = nullptr;      // [ndof] or null when kappa = 0
  const T* pen = nullptr;     // [E][6][n^2]
  const int* nbr = nullptr;   // [E][6]
  const int8_t* bc = nullptr; // [E][6]
  const T* D = nullptr;       // [n][n]
  T kappa = 0;
  T inv_wend = 0;             // 1 / w_0 = p (p + 1) / 2
};

template <typename T>
void sipg_apply(int p, const OpArgs<T>& a, hipStream_t st);

void geometry(int p, int E, const double* X, const double* D, const double* w, const double* x, double nu,
              double* G, double* WJ, double* ws, double* vol, double* area, double* lin, int* bad, hipStream_t st);
void rhs(int p, int E, const double* f, const double* uD, const double* qN, double* b, const double* G,
         const double* WJ, const double* pen, const double* ws, const int* nbr, const int8_t* bc, const double* D,
         double inv_wend, hipStream_t st);
void penalty(int E, int p, double mu_star, double nu, const int* nbr, const int8_t* bc, const double* vol,
             const double* area, const double* ws, double* pen, hipStream_t st);

template <typename T>
struct SchwarzArgs {
  int E = 0;
  int nrhs = 1;               // vectors are [nrhs][E (p+1)^3], inbox [nrhs][E][osz]
  const T* r = nullptr;       // input residual
  T* z = nullptr;             // output (mode 0: z = own part; mode 1: z += own part)
  int mode = 0;
  T* O = nullptr;             // overlap buffer [E][osz]
  const int* nb27 = nullptr;  // [E][27]
  const int8_t* var = nullptr;   // [E][3] variant index (left*3+right)
  const T* gco = nullptr;     // [E][4] g0..g3
  const T* S = nullptr;       // [9][ns*ns] padded eigenvector tables, S[i*ns + a] = (s_a)_i
  const T* ST = nullptr;      // [9][ns*ns] transposes
  const T* lam = nullptr;     // [9][ns]
  const T* W = nullptr;       // [9][ns]
  const int* map1d = nullptr; // [9][ns]: (delta+1)*64 + loc, or -1 for padding
  const uint8_t* sel = nullptr;  // [E] subdomains to solve (null: all)
  int unweighted = 0;            // 1: W = I (block-diagonal local solves)
  const float* corr = nullptr;   // [E][ns^3] learned correction added to the FD tile (or null)
  const double* cscale = nullptr;  // [E] scale of corr (the subdomain residual norm)
};

// Learned-correction helpers over the subdomain tiles of a list of elements (null list: all)
template <typename T>
void tile_features(int p, int m, const SchwarzArgs<T>& a, const int* ids, int n, const double* v, const double* J9,
                   float* X, double* norms, hipStream_t st);
template <typename T>
void tile_diff(int p, int m, const SchwarzArgs<T>& a, const int* ids, int n, const double* v1, const double* v2,
               const double* norms, float* out, hipStream_t st);
template <typename T>
void mark_subdomains(int p, int m, const SchwarzArgs<T>& a, const int* ids, int n, double* mask, hipStream_t st);

template <typename T>
void schwarz_solve(int p, int m, const SchwarzArgs<T>& a, hipStream_t st);
template <typename T>
void schwarz_overlap_add(int p, int m, const SchwarzArgs<T>& a, hipStream_t st);
int overlap_size(int p, int m);

// transfers: out (=|+=) T(x)T(x)T (in - in2); T is n_out x n_in
template <typename T>
bool tensor3(int n_in, int n_out, int E, const T* Tm, const T* in, const T* in2, T* out, int accumulate,
             hipStream_t st);

int reduction_blocks(int64_t n);

}  // namespace dgfas
