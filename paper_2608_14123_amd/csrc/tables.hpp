// Host FP64 tables of the nodal GLL spectral element (Sec. 2.2) and of the
// one-dimensional Schwarz subdomain problems (Sec. 4.3.1).
#pragma once
#include <vector>

namespace dgfas {

constexpr int kMaxDegree = 16;

struct Gll {
  int p = 0;
  std::vector<double> x, w;   // p+1 nodes (ascending) and weights
  std::vector<double> D;      // (p+1)^2 row-major: D[i*n+j] = l_j'(x_i)
};

// Gauss-Lobatto-Legendre nodes/weights/differentiation matrix of degree p.
const Gll& gll_table(int p);

// T[i*n_from + j] = l_j^{p_from}(x_i^{p_to}): interpolation of a degree-p_from nodal
// polynomial at the GLL nodes of degree p_to.
std::vector<double> interp_matrix(int p_from, int p_to);

// h-coarsening matrices of degree p (Sec. 3.2), each (p+1) x (p+1) row-major, in the order
// P_0, P_1, I_0^T, I_1^T, I_0, I_1 for the children b = 0 (xi in [-1, 0] of the parent) and 1:
// I_b[i][j] = l_j((x_i + 2b - 1) / 2) (the parent's basis at the child's nodes) and
// P_b[i][j] = w_b(i) l_j(2 x_i - (2b - 1)) (the child's basis at the parent's nodes, weighted
// 1 in the child's half, 1/2 at the shared midpoint, 0 elsewhere).
std::vector<double> h_child_matrices(int p);

// Reference-element L2 projection of a degree-p_from nodal polynomial onto degree p_to < p_from
// (Sec. 3.2): P = (I^T W I)^-1 I^T W with I = interp_matrix(p_to, p_from) and W the p_from GLL
// weights, which integrate every product involved exactly.  Row-major p_to+1 x p_from+1.
std::vector<double> l2_projection_matrix(int p_from, int p_to);

// Face condition of one side of a 1D subdomain; kInteriorNoOverlap is an interior face
// whose subdomain stops at the face (neighbour of another degree): the 1D matrix keeps
// the own element's half of the interior face terms and no node of the neighbour.
enum Side { kInterior = 0, kDirichlet = 1, kNeumann = 2, kInteriorNoOverlap = 3 };
constexpr int kSides = 4;   // variant index = left * kSides + right

// 1D subdomain data of a face-condition variant (Sec. 4.3.1): node map, generalized
// eigen-decomposition L s = lambda M s (S^T M S = I, S^T L S = diag lambda) and weights.
struct Variant1D {
  int ns = 0;                   // number of subdomain nodes in this direction
  std::vector<int> delta, loc;  // per subdomain node: neighbour offset (-1,0,1), local node index
  std::vector<double> S;        // ns*ns row-major, S[i*ns + a] = component i of eigenvector a
  std::vector<double> lam;      // ns eigenvalues
  std::vector<double> W;        // ns weights
};

Variant1D make_variant_1d(int p, int m, int left, int right, double mu_star);

}  // namespace dgfas
