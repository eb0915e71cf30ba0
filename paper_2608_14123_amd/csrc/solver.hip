// Host orchestration: level hierarchy and geometry set-up, WAS (Alg. 5), SCG
// (Alg. 6), the FAS V-cycle (Alg. 2) and the C ABI of include/dgfas.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dgfas.h"
#include "blas.hpp"
#include "kernels.hpp"
#include "tables.hpp"
#include "mlp.hpp"

namespace dgfas {
namespace {

thread_local std::string g_err;

struct Error : std::runtime_error {
  dgfas_status code;
  Error(dgfas_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPC(x)                                                                                   \
  do {                                                                                            \
    hipError_t e_ = (x);                                                                          \
    if (e_ != hipSuccess)                                                                         \
      throw Error(DGFAS_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));                    \
  } while (0)

template <typename T>
void xfer(int n_in, int n_out, int E, const T* Tm, const T* in, const T* in2, T* out, int acc, hipStream_t st) {
  if (!tensor3<T>(n_in, n_out, E, Tm, in, in2, out, acc, st))
    throw Error(DGFAS_EUNSUPPORTED, "no transfer kernel for this degree pair");
}

template <typename T>
T* dalloc(size_t n) {
  if (n == 0) return nullptr;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw Error(DGFAS_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  return static_cast<T*>(p);
}

template <typename T>
T* upload(const std::vector<T>& h, hipStream_t st) {
  T* d = dalloc<T>(h.size());
  if (d) HIPC(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return d;
}

template <typename T>
std::vector<T> download(const T* d, size_t n, hipStream_t st) {
  std::vector<T> h(n);
  if (n) HIPC(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  return h;
}

std::vector<float> to_float(const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); }

struct Level {
  int p = 0, n = 0, N2 = 0, N3 = 0, E = 0, m = 0, ns = 0;
  int64_t ndof = 0;
  double inv_wend = 0;
  // geometry
  double *X = nullptr, *G = nullptr, *WJ = nullptr, *ws = nullptr, *pen = nullptr;
  double *vol = nullptr, *area = nullptr, *lin = nullptr, *D = nullptr;
  float *G32 = nullptr, *WJ32 = nullptr, *pen32 = nullptr, *D32 = nullptr;
  // Schwarz
  int* nb27 = nullptr;
  int8_t* var = nullptr;
  double *gco = nullptr, *S = nullptr, *ST = nullptr, *lam = nullptr, *W = nullptr, *O = nullptr;
  float *gco32 = nullptr, *S32 = nullptr, *ST32 = nullptr, *lam32 = nullptr, *W32 = nullptr, *O32 = nullptr;
  int* map1d = nullptr;
  double* J9 = nullptr;          // [E][9] linear map Jacobian / det^(1/3) (network input)
  std::vector<int> h_nb27;       // host copy of the 26-neighbourhood
  // transfer matrices to the next coarser level (this = fine)
  double *Pm = nullptr, *Im = nullptr, *Rm = nullptr;
  // vectors
  double *u = nullptr, *g = nullptr, *ubar = nullptr, *r = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr,
         *r0 = nullptr;
  float *r32 = nullptr, *du32 = nullptr, *rc32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr,
        *r0_32 = nullptr;

  template <typename T>
  void scg_vectors(T*& r_, T*& z_, T*& p_, T*& q_, T*& r0_) {
    if constexpr (sizeof(T) == 8) { r_ = r; z_ = z; p_ = pv; q_ = q; r0_ = r0; }
    else { r_ = rc32; z_ = z32; p_ = p32; q_ = q32; r0_ = r0_32; }
  }
};

struct Solver {
  dgfas_options opt{};
  hipStream_t st = nullptr;
  int E = 0;
  int* nbr = nullptr;
  int8_t* bc = nullptr;
  std::vector<int> h_nbr;
  std::vector<int8_t> h_bc;
  std::vector<Level> lv;   // lv[0] = root (level 1)
  int nrhs = 1;            // right-hand sides per batch; vectors are [nrhs][ndof]
  double* partial = nullptr;   // [2][nrhs][1024] first-stage sums
  double* scal = nullptr;      // [nrhs][8] SCG scalars
  double* partial2() { return partial + (size_t)1024 * nrhs; }
  double* scratch = nullptr;
  std::vector<void*> owned;
  // learned correction on the finest level (FP64 Schwarz applications)
  Mlp* mlp = nullptr;
  bool learned = false;
  float *lX = nullptr, *lY = nullptr;
  double* lnorm = nullptr;
  double plain_rho = -1.0;       // first-cycle reduction factor of the plain smoother (fallback judge)
  double* usave = nullptr;       // finest-level copy of u taken before every learned cycle
  bool judge = true;             // apply the fallback rule (off only for diagnostics)
  // masked local solves (data generation): Schwarz restricted to selected subdomains, unweighted
  const uint8_t* msel = nullptr;
  const double* mmask = nullptr;

  template <typename T>
  T* own(T* p) {
    if (p) owned.push_back(p);
    return p;
  }
  ~Solver() {
    if (st) hipStreamSynchronize(st);
    for (void* p : owned) hipFree(p);
  }

  Level& level(int l) {
    if (l < 1 || l > (int)lv.size()) throw Error(DGFAS_EINVAL, "level out of range");
    return lv[l - 1];
  }

  // ---------------------------------------------------------------- operator
  template <typename T>
  OpArgs<T> op_args(Level& L, int mode, const T* u, const T* g, T* out);

  void apply(Level& L, const double* u, double* Au) {
    OpArgs<double> a = op_args<double>(L, 1, u, nullptr, Au);
    sipg_apply<double>(L.p, a, st);
  }
  void residual(Level& L, const double* u, const double* g, double* r) {
    OpArgs<double> a = op_args<double>(L, 0, u, g, r);
    sipg_apply<double>(L.p, a, st);
  }
  void residual32(Level& L, const float* u, const float* g, float* r) {
    OpArgs<float> a = op_args<float>(L, 0, u, g, r);
    sipg_apply<float>(L.p, a, st);
  }

  template <typename T>
  SchwarzArgs<T> sz_args(Level& L, const T* r, T* z, int mode);

  // z = B r (mode 0) or z += B r (mode 1)
  void schwarz(Level& L, const double* r, double* z, int mode) {
    SchwarzArgs<double> a = sz_args<double>(L, r, z, mode);
    if (msel) {
      // block-diagonal local solves on the selected subdomains only (their supports are disjoint)
      a.sel = msel;
      a.unweighted = 1;
      fill(L.ndof, z, 0.0, st);
      HIPC(hipMemsetAsync(L.O, 0, (size_t)L.E * overlap_size(L.p, L.m) * sizeof(double), st));
    } else if (learned && &L == &lv.back()) {
      // FD solve plus the network correction |r_s| MLP(r_s / |r_s|, J9)
      tile_features<double>(L.p, L.m, a, nullptr, L.E, r, L.J9, lX, lnorm, st);
      mlp->forward(lX, L.E, lY);
      a.corr = lY;
      a.cscale = lnorm;
    }
    schwarz_solve<double>(L.p, L.m, a, st);
    schwarz_overlap_add<double>(L.p, L.m, a, st);
  }
  void schwarz32(Level& L, const float* r, float* z, int mode) {
    SchwarzArgs<float> a = sz_args<float>(L, r, z, mode);
    schwarz_solve<float>(L.p, L.m, a, st);
    schwarz_overlap_add<float>(L.p, L.m, a, st);
  }

  // ---------------------------------------------------------------- smoothers
  void was(Level& L, double* u, const double* g, int n) {
    for (int i = 0; i < n; ++i) {
      residual(L, u, g, L.r);
      schwarz(L, L.r, u, 1);
    }
  }

  // Correction-form smoothing in FP32: r = g - A u (FP64); n WAS steps on
  // A du = r in FP32 from du = 0; u += du (FP64).
  void ensure_mixed_vectors(Level& L) {
    const size_t nv = (size_t)L.ndof * nrhs;
    if (!L.r32) L.r32 = own(dalloc<float>(nv));
    if (!L.du32) L.du32 = own(dalloc<float>(nv));
    if (!L.rc32) L.rc32 = own(dalloc<float>(nv));
    if (!L.O32) {
      const size_t nin = (size_t)L.E * overlap_size(L.p, L.m) * nrhs;
      L.O32 = own(dalloc<float>(nin));
      if (nin) HIPC(hipMemsetAsync(L.O32, 0, nin * sizeof(float), st));
    }
  }

  void was_mixed(Level& L, double* u, const double* g, int n) {
    if (n <= 0) return;
    ensure_mixed_vectors(L);
    residual(L, u, g, L.r);
    convert<double, float>(L.ndof * nrhs, L.r, L.r32, 0, st);
    schwarz32(L, L.r32, L.du32, 0);
    for (int i = 1; i < n; ++i) {
      residual32(L, L.du32, L.r32, L.rc32);
      schwarz32(L, L.rc32, L.du32, 1);
    }
    convert<float, double>(L.ndof * nrhs, L.du32, u, 1, st);
  }

  // per right-hand side dot products a^T b, synchronously
  std::vector<double> dots_sync(Level& L, const double* a, const double* b) {
    const int nb = reduction_blocks(L.ndof);
    dot_partials<double>(L.ndof, nrhs, a, b, nullptr, partial, nb, st);
    finish(nb, nrhs, partial, nullptr, kOpStore, scal, scratch, st);
    std::vector<double> h(nrhs);
    HIPC(hipMemcpyAsync(h.data(), scratch, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    return h;
  }

  void apply_t(Level& L, const double* u, double* Au) {
    apply(L, u, Au);
    if (mmask) mask_mul(L.ndof, Au, mmask, st);
  }
  void apply_t(Level& L, const float* u, float* Au) {
    OpArgs<float> a = op_args<float>(L, 1, u, nullptr, Au);
    sipg_apply<float>(L.p, a, st);
  }
  void residual_t(Level& L, const double* u, const double* g, double* r) { residual(L, u, g, r); }
  void residual_t(Level& L, const float* u, const float* g, float* r) { residual32(L, u, g, r); }
  void schwarz_t(Level& L, const double* r, double* z, int mode) { schwarz(L, r, z, mode); }
  void schwarz_t(Level& L, const float* r, float* z, int mode) { schwarz32(L, r, z, mode); }

  // Alg. 6 with p = z in the first iteration, every right-hand side with its own scalars.
  // r_max empty: exactly n iterations, no synchronisation; otherwise stop once
  // ||r_k|| <= r_max[k] for every right-hand side k (one synchronisation per iteration).
  // zero_start: x = 0 and r = f without an operator application (correction form).
  // SCG work vectors are allocated at set-up only where the configured cycle runs SCG;
  // other callers (data generation, dgfas_root_solve on any level) get them on first use
  void ensure_scg_vectors(Level& L, bool fp32) {
    const size_t nv = (size_t)L.ndof * nrhs;
    if (!fp32) {
      if (!L.z) L.z = own(dalloc<double>(nv));
      if (!L.pv) L.pv = own(dalloc<double>(nv));
      if (!L.q) L.q = own(dalloc<double>(nv));
      if (!L.r0) L.r0 = own(dalloc<double>(nv));
    } else {
      if (!L.rc32) L.rc32 = own(dalloc<float>(nv));
      if (!L.z32) L.z32 = own(dalloc<float>(nv));
      if (!L.p32) L.p32 = own(dalloc<float>(nv));
      if (!L.q32) L.q32 = own(dalloc<float>(nv));
      if (!L.r0_32) L.r0_32 = own(dalloc<float>(nv));
    }
  }

  template <typename T>
  int scg(Level& L, T* x, const T* f, int n, const std::vector<double>& r_max, bool* breakdown,
          bool zero_start = false) {
    ensure_scg_vectors(L, sizeof(T) == 4);
    const int nb = reduction_blocks(L.ndof);
    const int64_t nv = L.ndof * nrhs;
    T *r, *z, *pv, *q, *r0;
    L.scg_vectors<T>(r, z, pv, q, r0);
    if (zero_start) {
      fill(nv, x, (T)0, st);
      convert<T, T>(nv, f, r, 0, st);
    } else {
      residual_t(L, x, f, r);
    }
    HIPC(hipMemsetAsync(scal, 0, (size_t)8 * nrhs * sizeof(double), st));
    std::vector<double> h((size_t)8 * nrhs);
    int it = 0;
    for (int i = 1; i <= n; ++i) {
      schwarz_t(L, r, z, 0);
      if (i > 1) {
        dot_partials<T>(L.ndof, nrhs, z, r, nullptr, partial, nb, st);
        dot_partials<T>(L.ndof, nrhs, z, r, r0, partial2(), nb, st);
        finish(nb, nrhs, partial, partial2(), kOpBeta, scal, nullptr, st);
        pupdate<T>(L.ndof, nrhs, z, pv, scal, 0, st);
      } else {
        dot_partials<T>(L.ndof, nrhs, z, r, nullptr, partial, nb, st);
        finish(nb, nrhs, partial, nullptr, kOpGamma, scal, nullptr, st);
        pupdate<T>(L.ndof, nrhs, z, pv, scal, 1, st);
      }
      apply_t(L, pv, q);
      dot_partials<T>(L.ndof, nrhs, pv, q, nullptr, partial, nb, st);
      finish(nb, nrhs, partial, nullptr, kOpAlpha, scal, nullptr, st);
      cg_update<T>(L.ndof, nrhs, r, r0, q, x, pv, scal, partial, nb, st);
      finish(nb, nrhs, partial, nullptr, kOpNorm2, scal, nullptr, st);
      it = i;
      if (!r_max.empty()) {
        HIPC(hipMemcpyAsync(h.data(), scal, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        bool done = true, bad = false;
        for (int k = 0; k < nrhs; ++k) {
          bad = bad || h[k * 8 + 4] != 0.0;
          done = done && std::sqrt(h[k * 8 + 3]) <= r_max[k];
        }
        if (bad) { if (breakdown) *breakdown = true; break; }
        if (done) break;
      }
    }
    return it;
  }

  // Correction-form SCG smoothing in FP32: r = g - A u (FP64), n SCG iterations
  // on A du = r in FP32 from du = 0, u += du (FP64).
  void scg_mixed(Level& L, double* u, const double* g, int n) {
    ensure_mixed_vectors(L);
    residual(L, u, g, L.r);
    convert<double, float>(L.ndof * nrhs, L.r, L.r32, 0, st);
    scg<float>(L, L.du32, L.r32, n, {}, nullptr, true);
    convert<float, double>(L.ndof * nrhs, L.du32, u, 1, st);
  }

  void smooth(Level& L, double* u, const double* g, int n) {
    if (n <= 0) return;
    const bool mixed = opt.precision == DGFAS_FP32;
    if (opt.smoother == DGFAS_SCG) {
      if (mixed) scg_mixed(L, u, g, n);
      else scg<double>(L, u, g, n, {}, nullptr);
    } else if (mixed) {
      was_mixed(L, u, g, n);
    } else {
      was(L, u, g, n);
    }
  }

  int root_solve(double* u, const double* g, bool* breakdown) {
    Level& L = lv[0];
    residual(L, u, g, L.r);
    std::vector<double> rmax = dots_sync(L, L.r, L.r);
    bool any = false;
    for (double& v : rmax) {
      v = opt.root_rtol * std::sqrt(v);
      any = any || v > 0.0;
    }
    if (!any) return 0;
    return scg<double>(L, u, g, opt.root_max_iter, rmax, breakdown);
  }

  // Alg. 2 with global p-coarsening.
  void vcycle(double* u_top, const double* f_top) {
    const int Lc = (int)lv.size();
    Level& T = lv[Lc - 1];
    double* u_save = T.u;
    const double* g_save = T.g;
    T.u = u_top;
    T.g = const_cast<double*>(f_top);
    bool bd = false;
    for (int l = Lc - 1; l >= 1; --l) {
      Level& F = lv[l];
      Level& C = lv[l - 1];
      smooth(F, F.u, F.g, opt.ns1);
      residual(F, F.u, F.g, F.r);
      xfer<double>(F.n, C.n, C.E * nrhs, F.Pm, F.u, nullptr, C.ubar, 0, st);   // ubar = P u
      HIPC(hipMemcpyAsync(C.u, C.ubar, C.ndof * nrhs * sizeof(double), hipMemcpyDeviceToDevice, st));
      apply(C, C.ubar, C.g);                                                     // g = A ubar
      xfer<double>(F.n, C.n, C.E * nrhs, F.Rm, F.r, nullptr, C.g, 1, st);      //   + R r
    }
    root_solve(lv[0].u, lv[0].g, &bd);
    for (int l = 1; l < Lc; ++l) {
      Level& F = lv[l];
      Level& C = lv[l - 1];
      xfer<double>(C.n, F.n, C.E * nrhs, F.Im, C.u, C.ubar, F.u, 1, st);   // u += I (u_c - ubar)
      smooth(F, F.u, F.g, opt.ns2);
    }
    T.u = u_save;
    T.g = const_cast<double*>(g_save);
  }
};

template <typename T>
OpArgs<T> Solver::op_args(Level& L, int mode, const T* u, const T* g, T* out) {
  OpArgs<T> a;
  a.E = L.E;
  a.nrhs = nrhs;
  a.u = u;
  a.g = g;
  a.out = out;
  a.mode = mode;
  a.nbr = nbr;
  a.bc = bc;
  a.kappa = (T)opt.kappa;
  a.inv_wend = (T)L.inv_wend;
  if constexpr (sizeof(T) == 8) {
    a.G = L.G; a.WJ = opt.kappa != 0.0 ? L.WJ : nullptr; a.pen = L.pen; a.D = L.D;
  } else {
    a.G = L.G32; a.WJ = opt.kappa != 0.0 ? L.WJ32 : nullptr; a.pen = L.pen32; a.D = L.D32;
  }
  return a;
}

template <typename T>
SchwarzArgs<T> Solver::sz_args(Level& L, const T* r, T* z, int mode) {
  SchwarzArgs<T> a;
  a.E = L.E;
  a.nrhs = nrhs;
  a.r = r;
  a.z = z;
  a.mode = mode;
  a.nb27 = L.nb27;
  a.var = L.var;
  a.map1d = L.map1d;
  if constexpr (sizeof(T) == 8) {
    a.O = L.O; a.gco = L.gco; a.S = L.S; a.ST = L.ST; a.lam = L.lam; a.W = L.W;
  } else {
    a.O = L.O32; a.gco = L.gco32; a.S = L.S32; a.ST = L.ST32; a.lam = L.lam32; a.W = L.W32;
  }
  return a;
}

const int kFace[3][2] = {{0, 1}, {2, 3}, {4, 5}};

void build_level(Solver& s, Level& L, int p, const double* dX) {
  hipStream_t st = s.st;
  const Gll& gl = gll_table(p);
  L.p = p; L.n = p + 1; L.N2 = L.n * L.n; L.N3 = L.N2 * L.n; L.E = s.E;
  L.ndof = (int64_t)L.E * L.N3;
  L.inv_wend = 1.0 / gl.w[0];
  L.m = std::min(s.opt.overlap, p);
  L.ns = L.n + 2 * L.m;
  L.D = s.own(upload(gl.D, st));
  L.D32 = s.own(upload(to_float(gl.D), st));
  double* w1 = s.own(upload(gl.w, st));
  double* x1 = s.own(upload(gl.x, st));
  L.G = s.own(dalloc<double>(6 * L.ndof));
  L.WJ = s.own(dalloc<double>(L.ndof));
  L.ws = s.own(dalloc<double>((size_t)L.E * 6 * L.N2));
  L.pen = s.own(dalloc<double>((size_t)L.E * 6 * L.N2));
  L.vol = s.own(dalloc<double>(L.E));
  L.area = s.own(dalloc<double>((size_t)L.E * 6));
  L.lin = s.own(dalloc<double>((size_t)L.E * 9));
  int* bad = s.own(dalloc<int>(1));
  HIPC(hipMemsetAsync(bad, 0, sizeof(int), st));
  geometry(p, L.E, dX, L.D, w1, x1, s.opt.nu, L.G, L.WJ, L.ws, L.vol, L.area, L.lin, bad, st);
  HIPC(hipGetLastError());
  penalty(L.E, p, s.opt.mu_star, s.opt.nu, s.nbr, s.bc, L.vol, L.area, L.ws, L.pen, st);
  HIPC(hipGetLastError());
  int hbad = 0;
  HIPC(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (hbad) throw Error(DGFAS_EINVAL, "element map with det J <= 0 at degree " + std::to_string(p));
  // FP32 copies for the correction-form smoother
  L.G32 = s.own(dalloc<float>(6 * L.ndof));
  L.WJ32 = s.own(dalloc<float>(L.ndof));
  L.pen32 = s.own(dalloc<float>((size_t)L.E * 6 * L.N2));
  convert<double, float>(6 * L.ndof, L.G, L.G32, 0, st);
  convert<double, float>(L.ndof, L.WJ, L.WJ32, 0, st);
  convert<double, float>((int64_t)L.E * 6 * L.N2, L.pen, L.pen32, 0, st);

  // surrogate cuboid (Sec. 4.3.1 steps 1-3): Delta x_b = 2|a_b| (vol / prod)^(1/3)
  std::vector<double> vol = download(L.vol, L.E, st), lin = download(L.lin, (size_t)L.E * 9, st);
  std::vector<double> gco((size_t)L.E * 4);
  for (int e = 0; e < L.E; ++e) {
    double ell[3];
    for (int b = 0; b < 3; ++b) {
      double s2 = 0;
      for (int a = 0; a < 3; ++a) s2 += lin[e * 9 + a * 3 + b] * lin[e * 9 + a * 3 + b];
      ell[b] = 2.0 * std::sqrt(s2);
    }
    const double sc = std::cbrt(vol[e] / (ell[0] * ell[1] * ell[2]));
    const double dx[3] = {ell[0] * sc, ell[1] * sc, ell[2] * sc};
    gco[e * 4 + 0] = s.opt.kappa * dx[0] * dx[1] * dx[2] / 8.0;
    gco[e * 4 + 1] = s.opt.nu * dx[1] * dx[2] / (2.0 * dx[0]);
    gco[e * 4 + 2] = s.opt.nu * dx[2] * dx[0] / (2.0 * dx[1]);
    gco[e * 4 + 3] = s.opt.nu * dx[0] * dx[1] / (2.0 * dx[2]);
  }
  L.gco = s.own(upload(gco, st));
  {
    std::vector<double> j9((size_t)L.E * 9);
    for (int e = 0; e < L.E; ++e) {
      const double* A = &lin[e * 9];   // A[a][b] = coefficient of coordinate a along xi_b
      const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                         A[2] * (A[3] * A[7] - A[4] * A[6]);
      const double sc = 1.0 / std::cbrt(det);
      for (int q = 0; q < 9; ++q) j9[e * 9 + q] = A[q] * sc;
    }
    L.J9 = s.own(upload(j9, st));
  }
  L.gco32 = s.own(upload(to_float(gco), st));

  // variant tables (left, right) in {I, D, N}^2, zero padded to ns
  const int NS = L.ns;
  std::vector<double> S(9 * NS * NS, 0.0), lam(9 * NS, 1.0), W(9 * NS, 0.0);
  std::vector<int> map(9 * NS, -1);
  for (int left = 0; left < 3; ++left)
    for (int right = 0; right < 3; ++right) {
      const int v = left * 3 + right;
      Variant1D t = make_variant_1d(p, L.m, left, right, s.opt.mu_star);
      for (int i = 0; i < t.ns; ++i) {
        for (int a = 0; a < t.ns; ++a) S[v * NS * NS + i * NS + a] = t.S[i * t.ns + a];
        lam[v * NS + i] = t.lam[i];
        W[v * NS + i] = t.W[i];
        map[v * NS + i] = (t.delta[i] + 1) * 64 + t.loc[i];
      }
    }
  std::vector<double> ST(S.size());
  for (int v = 0; v < 9; ++v)
    for (int i = 0; i < NS; ++i)
      for (int a = 0; a < NS; ++a) ST[v * NS * NS + a * NS + i] = S[v * NS * NS + i * NS + a];
  L.S = s.own(upload(S, st)); L.S32 = s.own(upload(to_float(S), st));
  L.ST = s.own(upload(ST, st)); L.ST32 = s.own(upload(to_float(ST), st));
  L.lam = s.own(upload(lam, st)); L.lam32 = s.own(upload(to_float(lam), st));
  L.W = s.own(upload(W, st)); L.W32 = s.own(upload(to_float(W), st));
  L.map1d = s.own(upload(map, st));
  // per element: variant code per direction and the 27-neighbourhood
  std::vector<int8_t> var((size_t)L.E * 3);
  std::vector<int> nb27((size_t)L.E * 27, -1);
  for (int e = 0; e < L.E; ++e) {
    for (int d = 0; d < 3; ++d) {
      int code[2];
      for (int sd = 0; sd < 2; ++sd) {
        const int f = kFace[d][sd];
        code[sd] = s.h_nbr[e * 6 + f] >= 0 ? kInterior : (s.h_bc[e * 6 + f] == DGFAS_NEUMANN ? kNeumann : kDirichlet);
      }
      var[e * 3 + d] = (int8_t)(code[0] * 3 + code[1]);
    }
    for (int d3 = -1; d3 <= 1; ++d3)
      for (int d2 = -1; d2 <= 1; ++d2)
        for (int d1 = -1; d1 <= 1; ++d1) {
          int cur = e;
          const int dd[3] = {d1, d2, d3};
          for (int d = 0; d < 3 && cur >= 0; ++d)
            if (dd[d]) cur = s.h_nbr[cur * 6 + kFace[d][dd[d] > 0]];
          nb27[e * 27 + (d3 + 1) * 9 + (d2 + 1) * 3 + (d1 + 1)] = cur;
        }
  }
  L.var = s.own(upload(var, st));
  L.nb27 = s.own(upload(nb27, st));
  L.h_nb27 = nb27;
  const int osz = overlap_size(p, L.m);
  const size_t nin = (size_t)L.E * osz * s.nrhs;
  const bool fp32 = s.opt.precision == DGFAS_FP32;
  L.O = s.own(dalloc<double>(nin));
  if (fp32) L.O32 = s.own(dalloc<float>(nin));
  // inbox regions of absent neighbours are never written and must read as zero
  if (osz) {
    HIPC(hipMemsetAsync(L.O, 0, nin * sizeof(double), st));
    if (fp32) HIPC(hipMemsetAsync(L.O32, 0, nin * sizeof(float), st));
  }
  // work vectors
  const size_t nv = (size_t)L.ndof * s.nrhs;
  L.r = s.own(dalloc<double>(nv));
  const bool scg_here = s.opt.smoother == DGFAS_SCG || &L == &s.lv[0];
  const bool dbl_scg = scg_here && !(fp32 && &L != &s.lv[0]);
  if (dbl_scg || !fp32) L.z = s.own(dalloc<double>(nv));
  if (dbl_scg) {
    L.pv = s.own(dalloc<double>(nv));
    L.q = s.own(dalloc<double>(nv));
    L.r0 = s.own(dalloc<double>(nv));
  }
  if (fp32 && &L != &s.lv[0]) {
    L.r32 = s.own(dalloc<float>(nv));
    L.du32 = s.own(dalloc<float>(nv));
    L.rc32 = s.own(dalloc<float>(nv));
    if (s.opt.smoother == DGFAS_SCG) {
      L.z32 = s.own(dalloc<float>(nv));
      L.p32 = s.own(dalloc<float>(nv));
      L.q32 = s.own(dalloc<float>(nv));
      L.r0_32 = s.own(dalloc<float>(nv));
    }
  }
  HIPC(hipStreamSynchronize(st));
}

void validate(const dgfas_mesh_desc* m, const dgfas_options* o) {
  if (!m || !o) throw Error(DGFAS_EINVAL, "null mesh or options");
  if (m->n_elem <= 0 || !m->degree || !m->coords || !m->face_nbr || !m->face_bc)
    throw Error(DGFAS_EINVAL, "mesh arrays missing or n_elem <= 0");
  const int p = m->degree[0];
  for (int e = 0; e < m->n_elem; ++e)
    if (m->degree[e] != p) throw Error(DGFAS_EUNSUPPORTED, "mixed degrees are not supported by dgfas_create");
  if (p < 1 || p > 8) throw Error(DGFAS_EUNSUPPORTED, "degree must be 1..8");
  for (int e = 0; e < m->n_elem; ++e)
    for (int f = 0; f < 6; ++f) {
      const int en = m->face_nbr[e * 6 + f];
      if (en >= m->n_elem) throw Error(DGFAS_EINVAL, "face neighbour out of range");
      if (en >= 0 && m->face_nbr[en * 6 + (f ^ 1)] != e)
        throw Error(DGFAS_EUNSUPPORTED, "face neighbours must be aligned and mutual");
      if (en < 0 && m->face_bc[e * 6 + f] != DGFAS_DIRICHLET && m->face_bc[e * 6 + f] != DGFAS_NEUMANN)
        throw Error(DGFAS_EINVAL, "boundary face without a Dirichlet/Neumann code");
    }
  if (!(o->nu > 0) || !(o->kappa >= 0) || !(o->mu_star > 0)) throw Error(DGFAS_EINVAL, "bad coefficients");
  if (o->overlap < 0 || o->overlap > 1 + (p >= 4 ? 1 : 0))
    throw Error(DGFAS_EUNSUPPORTED, "overlap must be 0 or 1 (2 for p = 4, 8)");
  if (o->overlap == 2 && p != 4 && p != 8) throw Error(DGFAS_EUNSUPPORTED, "overlap 2 needs p = 4 or 8");
  if (o->smoother != DGFAS_WAS && o->smoother != DGFAS_SCG) throw Error(DGFAS_EINVAL, "unknown smoother");
  if (o->ns1 < 0 || o->ns2 < 0 || o->root_max_iter < 1) throw Error(DGFAS_EINVAL, "bad step counts");
  if (o->precision != DGFAS_FP64 && o->precision != DGFAS_FP32) throw Error(DGFAS_EINVAL, "unknown precision");
  if (o->n_rhs < 1 || o->n_rhs > 64) throw Error(DGFAS_EINVAL, "n_rhs must be 1..64");
  if ((int64_t)m->n_elem * o->n_rhs > (int64_t)1 << 30) throw Error(DGFAS_EUNSUPPORTED, "n_elem * n_rhs too large");
}

Solver* create(const dgfas_mesh_desc* m, const dgfas_options* o, void* stream) {
  validate(m, o);
  std::unique_ptr<Solver> s(new Solver());
  s->opt = *o;
  s->st = (hipStream_t)stream;
  s->E = m->n_elem;
  const int p = m->degree[0];
  s->h_nbr.assign(m->face_nbr, m->face_nbr + (size_t)s->E * 6);
  s->h_bc.assign(m->face_bc, m->face_bc + (size_t)s->E * 6);
  for (int e = 0; e < s->E; ++e)
    for (int f = 0; f < 6; ++f)
      if (s->h_nbr[e * 6 + f] >= 0) s->h_bc[e * 6 + f] = DGFAS_INTERIOR;
  s->nbr = s->own(upload(s->h_nbr, s->st));
  s->bc = s->own(upload(s->h_bc, s->st));
  s->nrhs = o->n_rhs;
  s->partial = s->own(dalloc<double>((size_t)2048 * s->nrhs));
  s->scal = s->own(dalloc<double>((size_t)8 * s->nrhs));
  s->scratch = s->own(dalloc<double>((size_t)8 * s->nrhs));
  std::vector<int> chain{p};
  while (chain.back() > 1) chain.push_back(std::max(1, chain.back() / 2));
  std::reverse(chain.begin(), chain.end());
  const int Lc = (int)chain.size();
  s->lv.resize(Lc);
  const int n = p + 1;
  const size_t nX = (size_t)s->E * 3 * n * n * n;
  double* X = s->own(dalloc<double>(nX));
  HIPC(hipMemcpyAsync(X, m->coords, nX * sizeof(double), hipMemcpyHostToDevice, s->st));
  for (int li = Lc - 1; li >= 0; --li) {
    Level& L = s->lv[li];
    if (li < Lc - 1) {
      Level& F = s->lv[li + 1];
      const int pc = chain[li], pf = chain[li + 1];
      std::vector<double> P = interp_matrix(pf, pc), I = interp_matrix(pc, pf);
      std::vector<double> R((size_t)(pc + 1) * (pf + 1));
      for (int a = 0; a <= pc; ++a)
        for (int b = 0; b <= pf; ++b) R[a * (pf + 1) + b] = I[b * (pc + 1) + a];
      F.Pm = s->own(upload(P, s->st));
      F.Im = s->own(upload(I, s->st));
      F.Rm = s->own(upload(R, s->st));
      // coarse geometry: fine coordinates evaluated at the coarse GLL nodes
      const size_t nXc = (size_t)s->E * 3 * (pc + 1) * (pc + 1) * (pc + 1);
      double* Xc = s->own(dalloc<double>(nXc));
      xfer<double>(pf + 1, pc + 1, 3 * s->E, F.Pm, X, nullptr, Xc, 0, s->st);
      HIPC(hipGetLastError());
      X = Xc;
    }
    build_level(*s, L, chain[li], X);
    L.X = X;
    if (li < Lc - 1) {
      L.u = s->own(dalloc<double>((size_t)L.ndof * s->nrhs));
      L.g = s->own(dalloc<double>((size_t)L.ndof * s->nrhs));
      L.ubar = s->own(dalloc<double>((size_t)L.ndof * s->nrhs));
    }
  }
  HIPC(hipStreamSynchronize(s->st));
  return s.release();
}

}  // namespace

const char* set_error(const std::string& m) {
  g_err = m;
  return g_err.c_str();
}

namespace {

dgfas_status fail(const Error& e) {
  g_err = e.what();
  return e.code;
}

}  // namespace
}  // namespace dgfas

using namespace dgfas;

struct dgfas_solver_s {
  Solver* s;
};

#define API_BEGIN try {
#define API_END                                           \
  }                                                       \
  catch (const Error& e) { return fail(e); }              \
  catch (const std::exception& e) {                       \
    g_err = e.what();                                     \
    return DGFAS_EINVAL;                                  \
  }                                                       \
  return DGFAS_OK;

static Solver* S_(dgfas_solver s) {
  if (!s || !s->s) throw Error(DGFAS_EINVAL, "null solver");
  return s->s;
}
static void need(const void* p, const char* what) {
  if (!p) throw Error(DGFAS_EINVAL, std::string("null pointer: ") + what);
}

extern "C" {

void dgfas_default_options(dgfas_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->kappa = 0.0;
  o->nu = 1.0;
  o->mu_star = 2.0;
  o->overlap = 1;
  o->smoother = DGFAS_WAS;
  o->ns1 = 2;
  o->ns2 = 2;
  o->root_max_iter = 500;
  o->root_rtol = 1e-12;
  o->precision = DGFAS_FP64;
  o->n_rhs = 1;
}

dgfas_status dgfas_gll(int32_t p, double* x, double* w) {
  API_BEGIN
  need(x, "x");
  need(w, "w");
  if (p < 1 || p > kMaxDegree) throw Error(DGFAS_EINVAL, "degree out of range");
  const Gll& g = gll_table(p);
  for (int i = 0; i <= p; ++i) { x[i] = g.x[i]; w[i] = g.w[i]; }
  API_END
}

dgfas_status dgfas_schwarz_tables_1d(int32_t p, int32_t m, int32_t left, int32_t right, double mu_star, int32_t* ns,
                                     double* S, double* lam, double* weights) {
  API_BEGIN
  need(ns, "ns"); need(S, "S"); need(lam, "lam"); need(weights, "weights");
  if (p < 1 || p > kMaxDegree || m < 0 || m > p) throw Error(DGFAS_EINVAL, "p or m out of range");
  if (left < 0 || left > 2 || right < 0 || right > 2) throw Error(DGFAS_EINVAL, "bad side code");
  Variant1D v = make_variant_1d(p, m, left, right, mu_star);
  *ns = v.ns;
  for (int i = 0; i < v.ns * v.ns; ++i) S[i] = v.S[i];
  for (int i = 0; i < v.ns; ++i) { lam[i] = v.lam[i]; weights[i] = v.W[i]; }
  API_END
}

dgfas_status dgfas_create(const dgfas_mesh_desc* mesh, const dgfas_options* opt, void* stream, dgfas_solver* out) {
  API_BEGIN
  need(out, "out");
  *out = nullptr;
  Solver* s = create(mesh, opt, stream);
  *out = new dgfas_solver_s{s};
  API_END
}

void dgfas_destroy(dgfas_solver s) {
  if (!s) return;
  delete s->s;
  delete s;
}

dgfas_status dgfas_levels(dgfas_solver s, int32_t* n) {
  API_BEGIN
  need(n, "n_levels");
  *n = (int32_t)S_(s)->lv.size();
  API_END
}

dgfas_status dgfas_level_info(dgfas_solver s, int32_t level, int32_t* degree, int64_t* n_dof) {
  API_BEGIN
  Level& L = S_(s)->level(level);
  if (degree) *degree = L.p;
  if (n_dof) *n_dof = L.ndof;
  API_END
}

dgfas_status dgfas_rhs(dgfas_solver sv, const double* f, const double* uD, const double* qN, double* b) {
  API_BEGIN
  Solver* s = S_(sv);
  need(f, "f"); need(b, "b");
  Level& T = s->lv.back();
  for (int k = 0; k < s->nrhs; ++k) {
    const int64_t o = (int64_t)k * T.ndof;
    rhs(T.p, T.E, f + o, uD ? uD + o : nullptr, qN ? qN + o : nullptr, b + o, T.G, T.WJ, T.pen, T.ws, s->nbr, s->bc,
        T.D, T.inv_wend, s->st);
  }
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_apply(dgfas_solver sv, int32_t level, const double* u, double* Au) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(Au, "Au");
  s->apply(s->level(level), u, Au);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_residual(dgfas_solver sv, int32_t level, const double* u, const double* g, double* r) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(g, "g"); need(r, "r");
  s->residual(s->level(level), u, g, r);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_schwarz(dgfas_solver sv, int32_t level, const double* r, double* z) {
  API_BEGIN
  Solver* s = S_(sv);
  need(r, "r"); need(z, "z");
  s->schwarz(s->level(level), r, z, 0);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_smooth(dgfas_solver sv, int32_t level, double* u, const double* g, int32_t n) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(g, "g");
  if (n < 0) throw Error(DGFAS_EINVAL, "negative step count");
  s->smooth(s->level(level), u, g, n);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_restrict(dgfas_solver sv, int32_t level, const double* rf, double* rc) {
  API_BEGIN
  Solver* s = S_(sv);
  need(rf, "r_fine"); need(rc, "r_coarse");
  if (level < 2) throw Error(DGFAS_EINVAL, "restrict needs level >= 2");
  Level& F = s->level(level);
  Level& C = s->level(level - 1);
  xfer<double>(F.n, C.n, C.E * s->nrhs, F.Rm, rf, nullptr, rc, 0, s->st);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_project(dgfas_solver sv, int32_t level, const double* uf, double* uc) {
  API_BEGIN
  Solver* s = S_(sv);
  need(uf, "u_fine"); need(uc, "u_coarse");
  if (level < 2) throw Error(DGFAS_EINVAL, "project needs level >= 2");
  Level& F = s->level(level);
  Level& C = s->level(level - 1);
  xfer<double>(F.n, C.n, C.E * s->nrhs, F.Pm, uf, nullptr, uc, 0, s->st);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_prolong_add(dgfas_solver sv, int32_t level, const double* uc, const double* ubar, double* uf) {
  API_BEGIN
  Solver* s = S_(sv);
  need(uc, "u_coarse"); need(uf, "u_fine");
  if (level < 2) throw Error(DGFAS_EINVAL, "prolong needs level >= 2");
  Level& F = s->level(level);
  Level& C = s->level(level - 1);
  xfer<double>(C.n, F.n, C.E * s->nrhs, F.Im, uc, ubar, uf, 1, s->st);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_root_solve(dgfas_solver sv, double* u, const double* g, int32_t* iters) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(g, "g");
  bool bd = false;
  const int it = s->root_solve(u, g, &bd);
  HIPC(hipStreamSynchronize(s->st));
  if (iters) *iters = it;
  if (bd) throw Error(DGFAS_EBREAKDOWN, "SCG breakdown in the root solve");
  API_END
}

dgfas_status dgfas_vcycle(dgfas_solver sv, double* u, const double* f) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(f, "f");
  s->vcycle(u, f);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_solve(dgfas_solver sv, double* u, const double* f, int32_t max_cycles, double rtol, double* hist,
                         int32_t* n_done) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(f, "f");
  if (max_cycles < 0) throw Error(DGFAS_EINVAL, "negative max_cycles");
  Level& T = s->lv.back();
  s->residual(T, u, f, T.r);
  std::vector<double> r0 = s->dots_sync(T, T.r, T.r);
  for (double& v : r0) v = std::sqrt(v);
  if (hist) hist[0] = 1.0;
  int k = 0;
  auto worst = [&](const std::vector<double>& rr) {
    double w = 0.0;
    for (int j = 0; j < s->nrhs; ++j) {
      const double rel = r0[j] > 0.0 ? std::sqrt(rr[j]) / r0[j] : 0.0;
      if (!std::isfinite(rel)) return rel;
      w = std::max(w, rel);
    }
    return w;
  };
  bool conv = worst(std::vector<double>(s->nrhs, 0.0)) == 0.0 &&
              *std::max_element(r0.begin(), r0.end()) == 0.0;
  // learned correction: the plain smoother is the judge.  The first solve after attaching runs
  // its first two cycles plain; the second cycle's reduction factor is the reference (the first
  // cycle of any solve reduces far more than later ones).  A learned cycle that reduces less than
  // the reference, or goes non-finite, is undone and the solve continues plain.
  const bool attached = s->learned;
  bool use_learned = attached, fell_back = false;
  if (attached && !s->usave) s->usave = s->own(dalloc<double>(T.ndof * s->nrhs));
  double* usave = s->usave;
  double prev = 1.0;
  while (!conv && k < max_cycles) {
    const bool plain_probe = use_learned && s->plain_rho < 0.0;
    s->learned = use_learned && !plain_probe;
    if (s->learned)
      HIPC(hipMemcpyAsync(usave, u, T.ndof * s->nrhs * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    s->vcycle(u, f);
    s->residual(T, u, f, T.r);
    double rk = worst(s->dots_sync(T, T.r, T.r));
    if (plain_probe && k == 1) s->plain_rho = rk / prev;
    if (s->learned && s->judge && (!std::isfinite(rk) || rk / prev > s->plain_rho)) {
      HIPC(hipMemcpyAsync(u, usave, T.ndof * s->nrhs * sizeof(double), hipMemcpyDeviceToDevice, s->st));
      use_learned = false;
      fell_back = true;
      s->learned = false;
      s->vcycle(u, f);
      s->residual(T, u, f, T.r);
      rk = worst(s->dots_sync(T, T.r, T.r));
    }
    ++k;
    if (hist) hist[k] = rk;
    if (!std::isfinite(rk)) { s->learned = attached; throw Error(DGFAS_EBREAKDOWN, "non-finite residual"); }
    prev = rk;
    conv = rk <= rtol;
  }
  s->learned = attached;
  if (n_done) *n_done = k;
  if (!conv) { g_err = "tolerance not reached"; return DGFAS_ENOTCONV; }
  if (fell_back) { g_err = "learned correction disabled by the fallback rule"; return DGFAS_EFALLBACK; }
  API_END
}

#if 0
#endif

dgfas_status dgfas_norm(dgfas_solver sv, int32_t level, const double* v, double* out) {
  API_BEGIN
  Solver* s = S_(sv);
  need(v, "v"); need(out, "out");
  std::vector<double> d = s->dots_sync(s->level(level), v, v);
  for (int k = 0; k < s->nrhs; ++k) out[k] = std::sqrt(d[k]);
  API_END
}

dgfas_status dgfas_set_learned(dgfas_solver sv, dgfas_mlp m, int32_t enabled) {
  API_BEGIN
  Solver* s = S_(sv);
  Level& T = s->lv.back();
  if (!enabled) { s->learned = false; return DGFAS_OK; }
  if (!m) throw Error(DGFAS_EINVAL, "null network");
  Mlp* net = dgfas_mlp_impl(m);
  const int nt = T.ns * T.ns * T.ns;
  if (net->in != nt + 9 || net->out != nt)
    throw Error(DGFAS_EINVAL, "network shape must be (ns^3 + 9) -> ns^3 = " + std::to_string(nt + 9) + " -> " +
                                  std::to_string(nt));
  if (s->nrhs != 1) throw Error(DGFAS_EUNSUPPORTED, "learned correction needs n_rhs = 1");
  if (s->opt.precision != DGFAS_FP64) throw Error(DGFAS_EUNSUPPORTED, "learned correction runs in the FP64 smoother");
  if (!s->lX) {
    s->lX = s->own(dalloc<float>((size_t)T.E * (nt + 9)));
    s->lY = s->own(dalloc<float>((size_t)T.E * nt));
    s->lnorm = s->own(dalloc<double>(T.E));
  }
  net->st = s->st;
  s->mlp = net;
  s->learned = true;
  s->judge = enabled != 2;
  s->plain_rho = -1.0;
  API_END
}

dgfas_status dgfas_learned_pairs(dgfas_solver sv, const double* r, const int32_t* centers, int32_t n, float* X,
                                 float* T, int32_t* pcg_iters) {
  API_BEGIN
  Solver* s = S_(sv);
  need(r, "r"); need(centers, "centers"); need(X, "X"); need(T, "T");
  if (s->nrhs != 1) throw Error(DGFAS_EUNSUPPORTED, "pairs need n_rhs = 1");
  Level& L = s->lv.back();
  if (n < 1 || n > L.E) throw Error(DGFAS_EINVAL, "bad number of centres");
  // centres must be 4 apart in the 26-neighbourhood graph: their 3x3x3 patches then neither
  // overlap nor touch, so the masked operator is block diagonal over the subdomains
  std::vector<char> is_center(L.E, 0);
  for (int c = 0; c < n; ++c) {
    const int e0 = centers[c];
    if (e0 < 0 || e0 >= L.E) throw Error(DGFAS_EINVAL, "centre out of range");
    if (is_center[e0]) throw Error(DGFAS_EINVAL, "repeated centre");
    is_center[e0] = 1;
  }
  for (int c = 0; c < n; ++c) {
    const int e0 = centers[c];
    std::vector<int> front{e0}, seen{e0};
    for (int hop = 0; hop < 3; ++hop) {
      std::vector<int> nxt;
      for (int e : front)
        for (int q = 0; q < 27; ++q) {
          const int en = L.h_nb27[(size_t)e * 27 + q];
          if (en < 0 || std::find(seen.begin(), seen.end(), en) != seen.end()) continue;
          if (is_center[en]) throw Error(DGFAS_EINVAL, "centres closer than 4 elements");
          seen.push_back(en);
          nxt.push_back(en);
        }
      front.swap(nxt);
    }
  }
  std::vector<int> ids(centers, centers + n);
  std::vector<uint8_t> sel(L.E, 0);
  for (int e : ids) sel[e] = 1;
  int* d_ids = upload(ids, s->st);
  uint8_t* d_sel = upload(sel, s->st);
  double *mask = nullptr, *b = nullptr, *z0 = nullptr, *x = nullptr, *nrm = nullptr;
  auto cleanup = [&]() {
    s->msel = nullptr;
    s->mmask = nullptr;
    hipStreamSynchronize(s->st);
    void* ps[] = {d_ids, d_sel, mask, b, z0, x, nrm};
    for (void* p : ps)
      if (p) hipFree(p);
  };
  try {
    mask = dalloc<double>(L.ndof);
    b = dalloc<double>(L.ndof);
    z0 = dalloc<double>(L.ndof);
    x = dalloc<double>(L.ndof);
    nrm = dalloc<double>(n);
    SchwarzArgs<double> a = s->sz_args<double>(L, r, z0, 0);
    fill(L.ndof, mask, 0.0, s->st);
    mark_subdomains<double>(L.p, L.m, a, d_ids, n, mask, s->st);
    convert<double, double>(L.ndof, r, b, 0, s->st);
    mask_mul(L.ndof, b, mask, s->st);
    s->msel = d_sel;
    s->mmask = mask;
    s->schwarz(L, b, z0, 0);                      // FD solutions of the local problems
    const double bn = std::sqrt(s->dots_sync(L, b, b)[0]);
    bool bd = false;
    const int it = s->scg<double>(L, x, b, 1000, {1e-11 * bn}, &bd, true);   // exact local solves
    if (bd) throw Error(DGFAS_EBREAKDOWN, "breakdown in the local solves");
    s->msel = nullptr;
    s->mmask = nullptr;
    tile_features<double>(L.p, L.m, a, d_ids, n, b, L.J9, X, nrm, s->st);
    tile_diff<double>(L.p, L.m, a, d_ids, n, x, z0, nrm, T, s->st);
    HIPC(hipGetLastError());
    if (pcg_iters) *pcg_iters = it;
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
  API_END
}

const char* dgfas_last_error(void) { return g_err.c_str(); }

}  // extern "C"
