// Launch interface of the MLP kernels (learned subdomain correction).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgfas {

void cast_bf16(int64_t n, const float* x, uint16_t* y, hipStream_t st);
void gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
               int64_t sbn, float* C, uint16_t* Cb, const float* bias, int relu, int accumulate, hipStream_t st);
void mse_grad(int64_t n, const float* Y, const float* T, float scale, float* dY, uint16_t* dYb, double* part,
              int nblocks, hipStream_t st);
void relu_back(int64_t n, float* G, const float* H, uint16_t* Gb, hipStream_t st);
void colsum(int rows, int cols, const float* G, float* out, hipStream_t st);
void adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* wb, float lr, float b1, float b2,
          float eps, float c1, float c2, hipStream_t st);

// Three affine layers in -> h -> h -> out with ReLU after the first two.
// Parameters (FP32 master, one array): W1[in][h] b1[h] W2[h][h] b2[h] W3[h][out] b3[out].
struct Mlp {
  int in = 0, h = 0, out = 0;
  int64_t off_w1 = 0, off_b1 = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0, n_params = 0;
  hipStream_t st = nullptr;
  float* w = nullptr;        // master weights
  uint16_t* wb = nullptr;    // BF16 copy (same layout)
  float *g = nullptr, *m = nullptr, *v = nullptr;   // gradient and Adam moments
  int64_t step = 0;
  // activations for up to cap rows
  int cap = 0;
  uint16_t *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *dYb = nullptr, *G2b = nullptr, *G1b = nullptr;
  float *H1 = nullptr, *H2 = nullptr, *dY = nullptr, *G2 = nullptr, *G1 = nullptr;
  double* part = nullptr;

  void reserve(int rows);
  void refresh_bf16();
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
