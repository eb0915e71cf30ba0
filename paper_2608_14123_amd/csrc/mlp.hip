// Host side of the learned subdomain correction: parameter storage, forward,
// backward and Adam training on the GPU, and their C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <random>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dgfas.h"
#include "mlp.hpp"

namespace dgfas {

const char* set_error(const std::string& m);   // defined with the solver ABI

namespace {
struct MlpError : std::runtime_error {
  dgfas_status code;
  MlpError(dgfas_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};
#define MHIP(x)                                                                    \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) throw MlpError(DGFAS_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
T* mal(size_t n) {
  void* p = nullptr;
  if (n == 0) return nullptr;
  if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) throw MlpError(DGFAS_ENOMEM, "hipMalloc failed");
  return (T*)p;
}
}  // namespace

Mlp::~Mlp() {
  if (st) hipStreamSynchronize(st);
  void* ps[] = {w, wb, w3p, g, m, v, Xb, H1b, H2b, dYb, G2b, G1b, H1, H2, G2, G1, part, kws};
  for (void* p : ps)
    if (p) hipFree(p);
}

void Mlp::reserve(int rows) {
  if (rows <= cap) return;
  void* ps[] = {Xb, H1b, H2b, dYb, G2b, G1b, H1, H2, G2, G1, kws};
  MHIP(hipStreamSynchronize(st));
  for (void* p : ps)
    if (p) hipFree(p);
  cap = rows;
  Xb = mal<uint16_t>((size_t)rows * in);
  H1b = mal<uint16_t>((size_t)rows * h);
  H2b = mal<uint16_t>((size_t)rows * h);
  dYb = mal<uint16_t>((size_t)rows * outp);
  MHIP(hipMemsetAsync(dYb, 0, (size_t)rows * outp * sizeof(uint16_t), st));   // padding columns stay zero
  G2b = mal<uint16_t>((size_t)rows * h);
  G1b = mal<uint16_t>((size_t)rows * h);
  H1 = mal<float>((size_t)rows * h);
  H2 = mal<float>((size_t)rows * h);
  G2 = mal<float>((size_t)rows * h);
  G1 = mal<float>((size_t)rows * h);
  // up to 16 K-slices of the largest weight gradient (at most 2^24 floats: a slice count the
  // cap cannot hold falls back to fewer slices)
  const int64_t mn = std::max<int64_t>((int64_t)(in + 1) * h,
                                       std::max<int64_t>((int64_t)(h + 1) * h, (int64_t)(h + 1) * out));
  kws_cap = std::min<int64_t>(16 * mn, (int64_t)1 << 24);
  kws = mal<float>((size_t)kws_cap);
}

void Mlp::refresh_w3p() { pad_rows(h, out, outp, wb + off_w3, w3p, st); }

void Mlp::refresh_bf16() {
  cast_bf16(n_params, w, wb, st);
  refresh_w3p();
}

void Mlp::forward(const float* X, int rows, float* Y) {
  reserve(rows);
  cast_bf16((int64_t)rows * in, X, Xb, st);
  gemm_bf16(rows, h, in, Xb, in, 1, wb + off_w1, h, 1, H1, H1b, w + off_b1, 1, 0, st, kws, kws_cap);
  gemm_bf16(rows, h, h, H1b, h, 1, wb + off_w2, h, 1, H2, H2b, w + off_b2, 1, 0, st);
  gemm_bf16(rows, out, h, H2b, h, 1, w3p, outp, 1, Y, nullptr, w + off_b3, 0, 0, st);
}

double Mlp::backward(const float* X, const float* T, int rows, float* Y) {
  forward(X, rows, Y);
  const int64_t ny = (int64_t)rows * out;
  const int nb = kLossBlocks;
  mse_grad(ny, out, outp, Y, T, 1.0f / (float)ny, dYb, part, nb, st);
  // every weight gradient is a GEMM over the rows whose A operand gets a row of ones: its last
  // output row is the bias gradient, which follows the weights in the parameter array
  // layer 3
  gemm_bf16(h + 1, out, rows, H2b, 1, h, dYb, outp, 1, g + off_w3, nullptr, nullptr, 0, 0, st, kws, kws_cap, 1);
  gemm_bf16(rows, h, out, dYb, outp, 1, w3p, 1, outp, G2, nullptr, nullptr, 0, 0, st, kws, kws_cap);
  relu_back((int64_t)rows * h, G2, H2, G2b, st);
  // layer 2
  gemm_bf16(h + 1, h, rows, H1b, 1, h, G2b, h, 1, g + off_w2, nullptr, nullptr, 0, 0, st, kws, kws_cap, 1);
  gemm_bf16(rows, h, h, G2b, h, 1, wb + off_w2, 1, h, G1, nullptr, nullptr, 0, 0, st);
  relu_back((int64_t)rows * h, G1, H1, G1b, st);
  // layer 1
  gemm_bf16(in + 1, h, rows, Xb, 1, in, G1b, h, 1, g + off_w1, nullptr, nullptr, 0, 0, st, kws, kws_cap, 1);
  std::vector<double> hp(nb);
  MHIP(hipMemcpyAsync(hp.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, st));
  MHIP(hipStreamSynchronize(st));
  double s = 0;
  for (double v_ : hp) s += v_;
  return s / (double)ny;
}

}  // namespace dgfas

using namespace dgfas;

struct dgfas_mlp_s {
  Mlp* m;
};

#define MLP_BEGIN try {
#define MLP_END                                                     \
  }                                                                 \
  catch (const MlpError& e) {                                       \
    set_error(e.what());                                            \
    return e.code;                                                  \
  }                                                                 \
  catch (const std::exception& e) {                                 \
    set_error(e.what());                                            \
    return DGFAS_EINVAL;                                            \
  }                                                                 \
  return DGFAS_OK;

static Mlp* M_(dgfas_mlp p) {
  if (!p || !p->m) throw MlpError(DGFAS_EINVAL, "null mlp");
  return p->m;
}

namespace dgfas {
Mlp* dgfas_mlp_impl(dgfas_mlp p) { return M_(p); }
}

extern "C" {

dgfas_status dgfas_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, uint64_t seed, void* stream,
                              dgfas_mlp* out) {
  MLP_BEGIN
  if (!out) throw MlpError(DGFAS_EINVAL, "null out");
  *out = nullptr;
  if (n_in < 1 || n_hidden < 1 || n_out < 1 || n_in > 65536 || n_hidden > 65536 || n_out > 65536)
    throw MlpError(DGFAS_EINVAL, "bad layer sizes");
  Mlp* m = new Mlp();
  std::unique_ptr<Mlp> guard(m);
  m->in = n_in; m->h = n_hidden; m->out = n_out; m->st = (hipStream_t)stream;
  int64_t o = 0;
  m->off_w1 = o; o += (int64_t)n_in * n_hidden;
  m->off_b1 = o; o += n_hidden;
  m->off_w2 = o; o += (int64_t)n_hidden * n_hidden;
  m->off_b2 = o; o += n_hidden;
  m->off_w3 = o; o += (int64_t)n_hidden * n_out;
  m->off_b3 = o; o += n_out;
  m->n_params = o;
  m->w = mal<float>(o); m->wb = mal<uint16_t>(o); m->g = mal<float>(o);
  m->m = mal<float>(o); m->v = mal<float>(o);
  m->outp = (n_out + 7) / 8 * 8;
  m->w3p = mal<uint16_t>((size_t)n_hidden * m->outp);
  m->part = mal<double>(kLossBlocks);
  // He-normal weights (seeded), zero biases
  std::vector<float> hw(o, 0.f);
  std::mt19937_64 rng(seed);
  auto fill = [&](int64_t off, int fan_in, int64_t cnt) {
    std::normal_distribution<float> nd(0.f, std::sqrt(2.0f / (float)fan_in));
    for (int64_t i = 0; i < cnt; ++i) hw[off + i] = nd(rng);
  };
  fill(m->off_w1, n_in, (int64_t)n_in * n_hidden);
  fill(m->off_w2, n_hidden, (int64_t)n_hidden * n_hidden);
  fill(m->off_w3, n_hidden, (int64_t)n_hidden * n_out);
  MHIP(hipMemcpyAsync(m->w, hw.data(), o * sizeof(float), hipMemcpyHostToDevice, m->st));
  MHIP(hipMemsetAsync(m->m, 0, o * sizeof(float), m->st));
  MHIP(hipMemsetAsync(m->v, 0, o * sizeof(float), m->st));
  m->refresh_bf16();
  MHIP(hipStreamSynchronize(m->st));
  *out = new dgfas_mlp_s{guard.release()};
  MLP_END
}

void dgfas_mlp_destroy(dgfas_mlp p) {
  if (!p) return;
  delete p->m;
  delete p;
}

dgfas_status dgfas_mlp_num_params(dgfas_mlp p, int64_t* n) {
  MLP_BEGIN
  if (!n) throw MlpError(DGFAS_EINVAL, "null n");
  *n = M_(p)->n_params;
  MLP_END
}

dgfas_status dgfas_mlp_get_params(dgfas_mlp p, float* host) {
  MLP_BEGIN
  Mlp* m = M_(p);
  if (!host) throw MlpError(DGFAS_EINVAL, "null buffer");
  MHIP(hipMemcpyAsync(host, m->w, m->n_params * sizeof(float), hipMemcpyDeviceToHost, m->st));
  MHIP(hipStreamSynchronize(m->st));
  MLP_END
}

dgfas_status dgfas_mlp_set_params(dgfas_mlp p, const float* host) {
  MLP_BEGIN
  Mlp* m = M_(p);
  if (!host) throw MlpError(DGFAS_EINVAL, "null buffer");
  MHIP(hipMemcpyAsync(m->w, host, m->n_params * sizeof(float), hipMemcpyHostToDevice, m->st));
  m->refresh_bf16();
  MHIP(hipMemsetAsync(m->m, 0, m->n_params * sizeof(float), m->st));
  MHIP(hipMemsetAsync(m->v, 0, m->n_params * sizeof(float), m->st));
  m->step = 0;
  MHIP(hipStreamSynchronize(m->st));
  MLP_END
}

dgfas_status dgfas_mlp_forward(dgfas_mlp p, const float* X, int32_t rows, float* Y) {
  MLP_BEGIN
  Mlp* m = M_(p);
  if (!X || !Y || rows < 1) throw MlpError(DGFAS_EINVAL, "bad forward arguments");
  m->forward(X, rows, Y);
  MHIP(hipGetLastError());
  MLP_END
}

dgfas_status dgfas_mlp_gradient(dgfas_mlp p, const float* X, const float* T, int32_t rows, float* grad,
                                double* loss) {
  MLP_BEGIN
  Mlp* m = M_(p);
  if (!X || !T || rows < 1) throw MlpError(DGFAS_EINVAL, "bad gradient arguments");
  m->reserve(rows);
  float* Y = mal<float>((size_t)rows * m->out);
  double l = 0;
  try {
    l = m->backward(X, T, rows, Y);
  } catch (...) {
    hipFree(Y);
    throw;
  }
  MHIP(hipFree(Y));
  if (grad) MHIP(hipMemcpyAsync(grad, m->g, m->n_params * sizeof(float), hipMemcpyDeviceToDevice, m->st));
  MHIP(hipStreamSynchronize(m->st));
  if (loss) *loss = l;
  MLP_END
}

dgfas_status dgfas_mlp_train(dgfas_mlp p, const float* X, const float* T, int64_t n, int32_t batch, int32_t steps,
                             float lr0, float lr_min, int32_t total_steps, double* losses) {
  MLP_BEGIN
  Mlp* m = M_(p);
  if (!X || !T || n < 1 || batch < 1 || steps < 0 || total_steps < 1) throw MlpError(DGFAS_EINVAL, "bad train arguments");
  const int rows = (int)std::min<int64_t>(batch, n);
  m->reserve(rows);
  float* Y = mal<float>((size_t)rows * m->out);
  try {
    for (int s = 0; s < steps; ++s) {
      const int64_t first = ((m->step * (int64_t)rows) % n);
      const int64_t r0 = first + rows <= n ? first : 0;
      const double loss = m->backward(X + r0 * m->in, T + r0 * m->out, rows, Y);
      if (losses) losses[s] = loss;
      const double t = std::min<double>(1.0, (double)m->step / (double)total_steps);
      const float lr = lr_min + 0.5f * (lr0 - lr_min) * (1.0f + (float)std::cos(3.14159265358979 * t));
      ++m->step;
      const float b1 = 0.9f, b2 = 0.999f;
      const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
      adam(m->n_params, m->w, m->g, m->m, m->v, m->wb, lr, b1, b2, 1e-8f, c1, c2, m->st);
      m->refresh_w3p();
    }
    MHIP(hipStreamSynchronize(m->st));
  } catch (...) {
    hipFree(Y);
    throw;
  }
  MHIP(hipFree(Y));
  MLP_END
}

}  // extern "C"
