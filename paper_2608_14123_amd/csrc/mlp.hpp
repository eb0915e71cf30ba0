// Launch interface of the MLP kernels (learned subdomain correction).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgfas {

void cast_bf16(int64_t n, const float* x, uint16_t* y, hipStream_t st);
// ws (ws_cap floats, may be null) holds the K-slice partial sums of a split-K launch; with
// ones_row, row M - 1 of A is a row of ones (A itself has M - 1 rows), so that row M - 1 of C
// holds the column sums of B
void gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
               int64_t sbn, float* C, uint16_t* Cb, const float* bias, int relu, int accumulate, hipStream_t st,
               float* ws = nullptr, int64_t ws_cap = 0, int ones_row = 0);
int gemm_splits(int M, int N, int K, int64_t ws_cap);
void mse_grad(int64_t n, int cols, int ldb, const float* Y, const float* T, float scale, uint16_t* dYb, double* part,
              int nblocks, hipStream_t st);
void pad_rows(int rows, int cols, int ldd, const uint16_t* src, uint16_t* dst, hipStream_t st);
void relu_back(int64_t n, float* G, const float* H, uint16_t* Gb, hipStream_t st);
void adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* wb, float lr, float b1, float b2,
          float eps, float c1, float c2, hipStream_t st);

constexpr int kLossBlocks = 1024;   // blocks (and partial sums) of the MSE kernel

// Three affine layers in -> h -> h -> out with ReLU after the first two.
// Parameters (FP32 master, one array): W1[in][h] b1[h] W2[h][h] b2[h] W3[h][out] b3[out].
struct Mlp {
  int in = 0, h = 0, out = 0;
  int outp = 0;              // out rounded up to a multiple of 8 (pitch of the padded BF16 rows)
  int64_t off_w1 = 0, off_b1 = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0, n_params = 0;
  hipStream_t st = nullptr;
  float* w = nullptr;        // master weights
  uint16_t* wb = nullptr;    // BF16 copy (same layout)
  uint16_t* w3p = nullptr;   // BF16 W3 with rows of pitch outp (8-byte aligned operand rows)
  float *g = nullptr, *m = nullptr, *v = nullptr;   // gradient and Adam moments
  int64_t step = 0;
  // activations for up to cap rows
  int cap = 0;
  uint16_t *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *dYb = nullptr, *G2b = nullptr, *G1b = nullptr;
  float *H1 = nullptr, *H2 = nullptr, *G2 = nullptr, *G1 = nullptr;   // dYb: rows of pitch outp
  double* part = nullptr;
  float* kws = nullptr;      // split-K partial sums
  int64_t kws_cap = 0;

  void reserve(int rows);
  void refresh_bf16();
  void refresh_w3p();
  // Y = f(X), X [rows][in] FP32 (device), Y [rows][out] FP32 (device)
  void forward(const float* X, int rows, float* Y);
  // forward + MSE loss (mean over rows*out) + gradient into g; returns the loss (synchronises)
  double backward(const float* X, const float* T, int rows, float* Y);
  ~Mlp();
};

}  // namespace dgfas

struct dgfas_mlp_s;
namespace dgfas {
Mlp* dgfas_mlp_impl(dgfas_mlp_s* p);   // throws on a null handle
}
