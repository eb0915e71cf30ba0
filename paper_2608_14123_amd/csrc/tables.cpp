// Host FP64 tables: GLL points (Newton on P_p'), barycentric differentiation and
// interpolation, 1D SIPG subdomain matrices and their generalized eigenproblem by
// cyclic Jacobi rotations.
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>

namespace dgfas {
namespace {

// Legendre P_p, P_p' at x (three-term recurrence).
void legendre(int p, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (p == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 1; k < p; ++k) {
    double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    double d2 = d0 + (2 * k + 1) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  P = p1; dP = d1;
}

std::vector<double> bary_weights(const std::vector<double>& x) {
  size_t n = x.size();
  std::vector<double> lam(n, 1.0);
  for (size_t j = 0; j < n; ++j)
    for (size_t k = 0; k < n; ++k)
      if (k != j) lam[j] /= (x[j] - x[k]);
  return lam;
}

Gll build_gll(int p) {
  Gll g;
  g.p = p;
  int n = p + 1;
  g.x.assign(n, 0.0);
  g.w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < n; ++j) g.x[j] = -std::cos(pi * j / p);   // Chebyshev-Lobatto start
  g.x[0] = -1.0;
  g.x[p] = 1.0;
  for (int j = 1; j < p; ++j) {
    double x = g.x[j];
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, x, P, dP);
      double d2P = (2.0 * x * dP - p * (p + 1) * P) / (1.0 - x * x);
      double dx = dP / d2P;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    g.x[j] = x;
  }
  // symmetrise
  for (int j = 0; j < n / 2; ++j) {
    double a = 0.5 * (g.x[p - j] - g.x[j]);
    g.x[j] = -a;
    g.x[p - j] = a;
  }
  if (n % 2 == 1) g.x[p / 2] = 0.0;
  for (int j = 0; j < n; ++j) {
    double P, dP;
    legendre(p, g.x[j], P, dP);
    g.w[j] = 2.0 / (p * (p + 1) * P * P);
  }
  std::vector<double> lam = bary_weights(g.x);
  g.D.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      double v = (lam[j] / lam[i]) / (g.x[i] - g.x[j]);
      g.D[i * n + j] = v;
      diag -= v;
    }
    g.D[i * n + i] = diag;
  }
  return g;
}

// Symmetric eigen-decomposition C = Q diag(ev) Q^T by cyclic Jacobi rotations.
void jacobi_eigen(int n, std::vector<double> C, std::vector<double>& Q, std::vector<double>& ev) {
  Q.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += C[i * n + j] * C[i * n + j];
        if (i != j) off += C[i * n + j] * C[i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = C[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = C[p * n + p], aqq = C[q * n + q];
        double theta = 0.5 * (aqq - app) / apq;
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          double ckp = C[k * n + p], ckq = C[k * n + q];
          C[k * n + p] = c * ckp - s * ckq;
          C[k * n + q] = s * ckp + c * ckq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          double cpk = C[p * n + k], cqk = C[q * n + k];
          C[p * n + k] = c * cpk - s * cqk;
          C[q * n + k] = s * cpk + c * cqk;
        }
        for (int k = 0; k < n; ++k) {
          double qkp = Q[k * n + p], qkq = Q[k * n + q];
          Q[k * n + p] = c * qkp - s * qkq;
          Q[k * n + q] = s * qkp + c * qkq;
        }
      }
  }
  ev.assign(n, 0.0);
  for (int i = 0; i < n; ++i) ev[i] = C[i * n + i];
}

double smoothstep5(double t) {
  if (t <= 0.0) return 0.0;
  if (t >= 1.0) return 1.0;
  return t * t * t * (10.0 + t * (-15.0 + 6.0 * t));
}

}  // namespace

const Gll& gll_table(int p) {
  static std::mutex mu;
  static std::map<int, Gll> cache;
  if (p < 1 || p > kMaxDegree) throw std::invalid_argument("degree out of range");
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(p);
  if (it == cache.end()) it = cache.emplace(p, build_gll(p)).first;
  return it->second;
}

std::vector<double> interp_matrix(int p_from, int p_to) {
  const Gll& gf = gll_table(p_from);
  const Gll& gt = gll_table(p_to);
  int nf = p_from + 1, nt = p_to + 1;
  std::vector<double> lam = bary_weights(gf.x);
  std::vector<double> T(nt * nf, 0.0);
  for (int i = 0; i < nt; ++i) {
    double y = gt.x[i];
    int hit = -1;
    for (int j = 0; j < nf; ++j)
      if (y == gf.x[j]) hit = j;
    if (hit >= 0) { T[i * nf + hit] = 1.0; continue; }
    double den = 0.0;
    for (int j = 0; j < nf; ++j) den += lam[j] / (y - gf.x[j]);
    for (int j = 0; j < nf; ++j) T[i * nf + j] = (lam[j] / (y - gf.x[j])) / den;
  }
  return T;
}

// L[i*n + j] = l_j(y_i) for the degree-p GLL Lagrange basis (barycentric form)
static std::vector<double> lagrange_at(int p, const std::vector<double>& y) {
  const Gll& g = gll_table(p);
  const int n = p + 1;
  const std::vector<double> lam = bary_weights(g.x);
  std::vector<double> L(y.size() * n, 0.0);
  for (size_t i = 0; i < y.size(); ++i) {
    int hit = -1;
    for (int j = 0; j < n; ++j)
      if (y[i] == g.x[j]) hit = j;
    if (hit >= 0) { L[i * n + hit] = 1.0; continue; }
    double den = 0.0;
    for (int j = 0; j < n; ++j) den += lam[j] / (y[i] - g.x[j]);
    for (int j = 0; j < n; ++j) L[i * n + j] = (lam[j] / (y[i] - g.x[j])) / den;
  }
  return L;
}

std::vector<double> h_child_matrices(int p) {
  const Gll& g = gll_table(p);
  const int n = p + 1, n2 = n * n;
  std::vector<double> out(6 * n2, 0.0);
  for (int b = 0; b < 2; ++b) {
    std::vector<double> yi(n), yp(n);
    for (int i = 0; i < n; ++i) {
      yi[i] = (g.x[i] + (2 * b - 1)) / 2.0;
      yp[i] = std::min(1.0, std::max(-1.0, 2.0 * g.x[i] - (2 * b - 1)));
    }
    const std::vector<double> I = lagrange_at(p, yi), P = lagrange_at(p, yp);
    for (int i = 0; i < n; ++i) {
      const bool mid = std::fabs(g.x[i]) < 1e-14, inside = b == 0 ? g.x[i] < 0 : g.x[i] > 0;
      const double w = mid ? 0.5 : (inside ? 1.0 : 0.0);
      for (int j = 0; j < n; ++j) {
        out[b * n2 + i * n + j] = w * P[i * n + j];          // P_b
        out[(2 + b) * n2 + j * n + i] = I[i * n + j];        // I_b^T
        out[(4 + b) * n2 + i * n + j] = I[i * n + j];        // I_b
      }
    }
  }
  return out;
}

std::vector<double> l2_projection_matrix(int p_from, int p_to) {
  const int nf = p_from + 1, nc = p_to + 1;
  const std::vector<double> I = interp_matrix(p_to, p_from);   // nf x nc
  const std::vector<double>& w = gll_table(p_from).w;
  // normal equations M P = B with M = I^T W I (nc x nc, SPD) and B = I^T W (nc x nf)
  std::vector<double> M(nc * nc, 0.0), B(nc * nf, 0.0);
  for (int a = 0; a < nc; ++a) {
    for (int b = 0; b < nc; ++b)
      for (int q = 0; q < nf; ++q) M[a * nc + b] += I[q * nc + a] * w[q] * I[q * nc + b];
    for (int q = 0; q < nf; ++q) B[a * nf + q] = I[q * nc + a] * w[q];
  }
  // Gaussian elimination with partial pivoting on [M | B]
  for (int c = 0; c < nc; ++c) {
    int piv = c;
    for (int r = c + 1; r < nc; ++r)
      if (std::fabs(M[r * nc + c]) > std::fabs(M[piv * nc + c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < nc; ++k) std::swap(M[c * nc + k], M[piv * nc + k]);
      for (int k = 0; k < nf; ++k) std::swap(B[c * nf + k], B[piv * nf + k]);
    }
    for (int r = 0; r < nc; ++r) {
      if (r == c) continue;
      const double f = M[r * nc + c] / M[c * nc + c];
      if (f == 0.0) continue;
      for (int k = 0; k < nc; ++k) M[r * nc + k] -= f * M[c * nc + k];
      for (int k = 0; k < nf; ++k) B[r * nf + k] -= f * B[c * nf + k];
    }
  }
  for (int r = 0; r < nc; ++r)
    for (int k = 0; k < nf; ++k) B[r * nf + k] /= M[r * nc + r];
  return B;
}

Variant1D make_variant_1d(int p, int m, int left, int right, double mu_star) {
  const Gll& g = gll_table(p);
  const int n = p + 1;
  if (m < 0 || m > p) throw std::invalid_argument("overlap out of range");
  if (left < 0 || left >= kSides || right < 0 || right >= kSides) throw std::invalid_argument("bad side code");
  // overlap per side: an interior side without overlap keeps the patch element (its face
  // terms) but selects none of its nodes
  const int ml = left == kInterior ? m : 0, mr = right == kInterior ? m : 0;
  if (left == kInteriorNoOverlap) left = kInterior;
  if (right == kInteriorNoOverlap) right = kInterior;
  // Patch of reference elements (length 2, so d/dx = d/dxi and the mass is diag(w)).
  int nel = 1 + (left == kInterior) + (right == kInterior);
  int c0 = (left == kInterior) ? 1 : 0;   // index of the centre element in the patch
  int N = nel * n;
  std::vector<double> L(N * N, 0.0), M(N, 0.0);
  const double mu = mu_star * p * (p + 1) / 4.0;
  const double* D = g.D.data();
  auto at = [&](int r, int c) -> double& { return L[r * N + c]; };
  for (int e = 0; e < nel; ++e)
    for (int a = 0; a < n; ++a) {
      M[e * n + a] = g.w[a];
      for (int b = 0; b < n; ++b) {
        double s = 0.0;
        for (int q = 0; q < n; ++q) s += D[q * n + a] * g.w[q] * D[q * n + b];
        at(e * n + a, e * n + b) += s;
      }
    }
  // interior points between patch elements e and e+1: mu [v][u] - {v'}[u] - [v]{u'}
  for (int e = 0; e + 1 < nel; ++e) {
    std::vector<double> jv(N, 0.0), av(N, 0.0);
    jv[e * n + p] = 1.0;
    jv[(e + 1) * n] = -1.0;
    for (int b = 0; b < n; ++b) {
      av[e * n + b] += 0.5 * D[p * n + b];
      av[(e + 1) * n + b] += 0.5 * D[0 * n + b];
    }
    for (int r = 0; r < N; ++r)
      for (int c = 0; c < N; ++c) at(r, c) += mu * jv[r] * jv[c] - av[r] * jv[c] - jv[r] * av[c];
  }
  // Dirichlet ends of the centre element: 2 mu v u - (d_n v) u - v d_n u
  if (left == kDirichlet) {
    int r0 = c0 * n;
    at(r0, r0) += 2.0 * mu;
    for (int b = 0; b < n; ++b) {   // outward normal -1: d_n = -d/dxi
      at(c0 * n + b, r0) += D[0 * n + b];
      at(r0, c0 * n + b) += D[0 * n + b];
    }
  }
  if (right == kDirichlet) {
    int r1 = c0 * n + p;
    at(r1, r1) += 2.0 * mu;
    for (int b = 0; b < n; ++b) {
      at(c0 * n + b, r1) -= D[p * n + b];
      at(r1, c0 * n + b) -= D[p * n + b];
    }
  }
  Variant1D v;
  std::vector<int> sel;
  if (left == kInterior)
    for (int l = n - ml; l < n; ++l) { v.delta.push_back(-1); v.loc.push_back(l); sel.push_back(l); }
  for (int l = 0; l < n; ++l) { v.delta.push_back(0); v.loc.push_back(l); sel.push_back(c0 * n + l); }
  if (right == kInterior)
    for (int l = 0; l < mr; ++l) { v.delta.push_back(1); v.loc.push_back(l); sel.push_back((c0 + 1) * n + l); }
  const int ns = (int)sel.size();
  v.ns = ns;
  // C = M^-1/2 L M^-1/2 on the selected nodes
  std::vector<double> C(ns * ns), ih(ns);
  for (int a = 0; a < ns; ++a) ih[a] = 1.0 / std::sqrt(M[sel[a]]);
  for (int a = 0; a < ns; ++a)
    for (int b = 0; b < ns; ++b) C[a * ns + b] = ih[a] * at(sel[a], sel[b]) * ih[b];
  for (int a = 0; a < ns; ++a)
    for (int b = a + 1; b < ns; ++b) {
      double s = 0.5 * (C[a * ns + b] + C[b * ns + a]);
      C[a * ns + b] = C[b * ns + a] = s;
    }
  std::vector<double> Q, ev;
  jacobi_eigen(ns, C, Q, ev);
  v.S.assign(ns * ns, 0.0);
  for (int i = 0; i < ns; ++i)
    for (int a = 0; a < ns; ++a) v.S[i * ns + a] = ih[i] * Q[i * ns + a];
  v.lam = ev;
  // weights: quintic blend across each overlapped side
  v.W.assign(ns, 1.0);
  if (m > 0) {
    const double a = 0.5 * (1.0 + g.x[m]);
    for (int s = 0; s < ns; ++s) {
      double w = 1.0;
      const double xl = g.x[v.loc[s]];
      if (ml > 0) {
        if (v.delta[s] == 0) w *= smoothstep5((0.5 * (1.0 + xl) + a) / (2 * a));
        else if (v.delta[s] == -1) w *= smoothstep5((-0.5 * (1.0 - xl) + a) / (2 * a));
      }
      if (mr > 0) {
        if (v.delta[s] == 0) w *= smoothstep5((0.5 * (1.0 - xl) + a) / (2 * a));
        else if (v.delta[s] == 1) w *= smoothstep5((-0.5 * (1.0 + xl) + a) / (2 * a));
      }
      v.W[s] = w;
    }
  }
  return v;
}

}  // namespace dgfas
