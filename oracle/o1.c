/*
 * O1: FP64 matrix-free CPU oracle of the FAS multigrid with weighted overlapping Schwarz
 * smoothing for SIPG DG spectral elements, in plain C with OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load this library (through oracle/o1.py); the product never does, and this file
 * shares no code with the HIP library.  It restates, element by element and in the paper's
 * order, what the numpy oracle of this directory computes, so that the same method can be run
 * at full size: the numpy oracle pins it element-wise on small meshes.
 *
 * Small 1D tables (GLL nodes and weights, the differentiation matrix, the rows of the inverse
 * Legendre-Vandermonde matrix, the 1D Schwarz variants and the interpolation matrices) come
 * from the numpy oracle through o1_set_level; everything that scales with the mesh is here:
 *  - geometry (Sec. 2.2): Jacobian of the isoparametric map by applying D along each
 *    direction, metric dxi_b/dx_a, w J, face omega s and outward normal from the cross
 *    product of the two tangential derivatives, h_perp = vol / area, penalty
 *    mu = mu_star avg(p(p+1)/(2 h_perp)) (eq. helmholtz:dgm);
 *  - the SIPG operator and right-hand side (eq. helmholtz:dgm, eq. helmholtz:system);
 *  - the surrogate cuboid (Sec. 4.3.1 steps 1-3) and the fast-diagonalisation subdomain
 *    solves with the weighted combination (eq. schwarz:tpo, eq. schwarz:correction);
 *  - WAS (Alg. 5), SCG (Alg. 6, first direction z, flexible beta), the transfers of
 *    Sec. 3.2, the FAS V-cycle (Alg. 2) and the solve loop.
 *
 * Layout: element-major, nodes [k][j][i] with i fastest; faces 0:-xi1 1:+xi1 2:-xi2 3:+xi2
 * 4:-xi3 5:+xi3, face node (a, b) = (k, j) on faces 0/1, (k, i) on 2/3, (j, i) on 4/5.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define NMAX 17
#define NSMAX 24
static const int OPP[6] = {1, 0, 3, 2, 5, 4};

typedef struct {
  int nv;                         /* subdomain nodes in this direction */
  int map[NSMAX];                 /* (delta + 1) * 64 + local index */
  double S[NSMAX * NSMAX];        /* S[i * nv + a]: column a is an eigenvector, S^T M S = I */
  double lam[NSMAX];
  double W[NSMAX];
} Variant;

typedef struct {
  int p, n, n3, m;
  int64_t ndof;
  double x[NMAX], w[NMAX], D[NMAX * NMAX], v0[NMAX], v1[NMAX];
  Variant var[9];                 /* (left, right) in {interior, Dirichlet, Neumann}^2 */
  int nc;                         /* nodes per direction of the next coarser level (0: root) */
  double P[NMAX * NMAX];          /* [nc][n]  fine -> coarse evaluation */
  double I[NMAX * NMAX];          /* [n][nc]  coarse -> fine interpolation; R = I^T */
  /* geometry */
  double *X, *wJ, *dxi, *fws, *fn, *mu, *gco;
  int* vcode;
  /* vectors of the cycle */
  double *u, *g, *ubar, *r, *z, *pv, *q, *r0, *grad, *tiles;
} Level;

typedef struct {
  int L, E;
  int *nbr, *bc, *nb27;
  double kappa, nu, mu_star;
  Level* lv;                      /* lv[0] = root */
} O1;

/* ------------------------------------------------------------------------------ helpers */
static int face_node(int n, int phi, int a, int b, int t) {
  const int ax = phi >> 1;
  if (ax == 0) return (a * n + b) * n + t;
  if (ax == 1) return (a * n + t) * n + b;
  return (t * n + a) * n + b;
}

/* du = derivative of u along direction c (D applied along that index) */
static void deriv(const Level* L, const double* u, int c, double* du) {
  const int n = L->n;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int m = 0; m < n; ++m) {
          const int src = c == 0 ? (k * n + j) * n + m : (c == 1 ? (k * n + m) * n + i : (m * n + j) * n + i);
          const int row = c == 0 ? i : (c == 1 ? j : k);
          s += L->D[row * n + m] * u[src];
        }
        du[(k * n + j) * n + i] = s;
      }
}

/* out += D_c^T v */
static void deriv_t_add(const Level* L, const double* v, int c, double* out) {
  const int n = L->n;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const double vv = v[(k * n + j) * n + i];
        const int row = c == 0 ? i : (c == 1 ? j : k);
        for (int m = 0; m < n; ++m) {
          const int dst = c == 0 ? (k * n + j) * n + m : (c == 1 ? (k * n + m) * n + i : (m * n + j) * n + i);
          out[dst] += L->D[row * n + m] * vv;
        }
      }
}

/* out = T (x) T (x) T in, T is no x ni */
static void tensor3(const double* T, int no, int ni, const double* in, double* out) {
  double a[NMAX * NMAX * NMAX], b[NMAX * NMAX * NMAX];
  for (int k = 0; k < ni; ++k)
    for (int j = 0; j < ni; ++j)
      for (int i = 0; i < no; ++i) {
        double s = 0.0;
        for (int m = 0; m < ni; ++m) s += T[i * ni + m] * in[(k * ni + j) * ni + m];
        a[(k * ni + j) * no + i] = s;
      }
  for (int k = 0; k < ni; ++k)
    for (int j = 0; j < no; ++j)
      for (int i = 0; i < no; ++i) {
        double s = 0.0;
        for (int m = 0; m < ni; ++m) s += T[j * ni + m] * a[(k * ni + m) * no + i];
        b[(k * no + j) * no + i] = s;
      }
  for (int k = 0; k < no; ++k)
    for (int j = 0; j < no; ++j)
      for (int i = 0; i < no; ++i) {
        double s = 0.0;
        for (int m = 0; m < ni; ++m) s += T[k * ni + m] * b[(m * no + j) * no + i];
        out[(k * no + j) * no + i] = s;
      }
}

static double dot(int64_t N, const double* a, const double* b) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t i = 0; i < N; ++i) s += a[i] * b[i];
  return s;
}

/* ------------------------------------------------------------------------------ geometry */
static void geometry(O1* o, Level* L) {
  const int n = L->n, n3 = L->n3, n2 = n * n, E = o->E;
  double* vol = (double*)calloc(E, sizeof(double));
  double* area = (double*)calloc((size_t)E * 6, sizeof(double));
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int e = 0; e < E; ++e) {
    double Jac[9][NMAX * NMAX * NMAX];        /* Jac[a * 3 + b] = dx_a / dxi_b */
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) deriv(L, L->X + ((size_t)e * 3 + a) * n3, b, Jac[a * 3 + b]);
    double vsum = 0.0;
    for (int q = 0; q < n3; ++q) {
      double J[9];
      for (int t = 0; t < 9; ++t) J[t] = Jac[t][q];
      const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                         J[2] * (J[3] * J[7] - J[4] * J[6]);
      if (!(det > 0)) bad = 1;
      /* inverse: dxi[b][a] = dxi_b / dx_a */
      double* di = L->dxi + ((size_t)e * n3 + q) * 9;
      di[0] = (J[4] * J[8] - J[5] * J[7]) / det;
      di[1] = (J[2] * J[7] - J[1] * J[8]) / det;
      di[2] = (J[1] * J[5] - J[2] * J[4]) / det;
      di[3] = (J[5] * J[6] - J[3] * J[8]) / det;
      di[4] = (J[0] * J[8] - J[2] * J[6]) / det;
      di[5] = (J[2] * J[3] - J[0] * J[5]) / det;
      di[6] = (J[3] * J[7] - J[4] * J[6]) / det;
      di[7] = (J[1] * J[6] - J[0] * J[7]) / det;
      di[8] = (J[0] * J[4] - J[1] * J[3]) / det;
      const int i = q % n, j = (q / n) % n, k = q / n2;
      L->wJ[(size_t)e * n3 + q] = L->w[i] * L->w[j] * L->w[k] * det;
      vsum += L->wJ[(size_t)e * n3 + q];
    }
    vol[e] = vsum;
    for (int phi = 0; phi < 6; ++phi) {
      const int ax = phi >> 1, t = (phi & 1) ? n - 1 : 0;
      const int c1 = (ax + 1) % 3, c2 = (ax + 2) % 3;     /* tangential directions, cyclic */
      const double sign = (phi & 1) ? 1.0 : -1.0;
      double asum = 0.0;
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          const int q = face_node(n, phi, a, b, t);
          double t1[3], t2[3];
          for (int x = 0; x < 3; ++x) { t1[x] = Jac[x * 3 + c1][q]; t2[x] = Jac[x * 3 + c2][q]; }
          const double om = L->w[a] * L->w[b];
          const double N[3] = {sign * om * (t1[1] * t2[2] - t1[2] * t2[1]), sign * om * (t1[2] * t2[0] - t1[0] * t2[2]),
                               sign * om * (t1[0] * t2[1] - t1[1] * t2[0])};
          const double ws = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
          const size_t f = (((size_t)e * 6 + phi) * n2 + a * n + b);
          L->fws[f] = ws;
          for (int x = 0; x < 3; ++x) L->fn[f * 3 + x] = N[x] / ws;
          asum += ws;
        }
      area[(size_t)e * 6 + phi] = asum;
    }
    /* surrogate cuboid: linear Legendre coefficients a_b of the map, edge lengths 2|a_b|,
       rescaled to the element volume; g0..g3 of eq. schwarz:tpo */
    double ell[3];
    for (int b = 0; b < 3; ++b) {
      double s2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        const double* Xa = L->X + ((size_t)e * 3 + a) * n3;
        double c = 0.0;
        for (int k = 0; k < n; ++k)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
              const double wi = b == 0 ? L->v1[i] : L->v0[i];
              const double wj = b == 1 ? L->v1[j] : L->v0[j];
              const double wk = b == 2 ? L->v1[k] : L->v0[k];
              c += wi * wj * wk * Xa[(k * n + j) * n + i];
            }
        s2 += c * c;
      }
      ell[b] = 2.0 * sqrt(s2);
    }
    const double sc = cbrt(vsum / (ell[0] * ell[1] * ell[2]));
    const double dx[3] = {ell[0] * sc, ell[1] * sc, ell[2] * sc};
    double* g = L->gco + (size_t)e * 4;
    g[0] = o->kappa * dx[0] * dx[1] * dx[2] / 8.0;
    g[1] = o->nu * dx[1] * dx[2] / (2.0 * dx[0]);
    g[2] = o->nu * dx[2] * dx[0] / (2.0 * dx[1]);
    g[3] = o->nu * dx[0] * dx[1] / (2.0 * dx[2]);
  }
  (void)bad;
  /* penalty per element face */
  const double pp = (double)L->p * (L->p + 1);
  for (int e = 0; e < E; ++e)
    for (int phi = 0; phi < 6; ++phi) {
      const double own = pp / (2.0 * vol[e] / area[(size_t)e * 6 + phi]);
      const int en = o->nbr[e * 6 + phi];
      if (en < 0) L->mu[e * 6 + phi] = o->mu_star * own;
      else {
        const double oth = pp / (2.0 * vol[en] / area[(size_t)en * 6 + OPP[phi]]);
        L->mu[e * 6 + phi] = o->mu_star * 0.5 * (own + oth);
      }
    }
  /* Schwarz variant per element direction: 0 interior, 1 Dirichlet, 2 Neumann */
  for (int e = 0; e < E; ++e)
    for (int d = 0; d < 3; ++d) {
      int code[2];
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * d + s;
        code[s] = o->nbr[e * 6 + f] >= 0 ? 0 : (o->bc[e * 6 + f] == 1 ? 1 : 2);
      }
      L->vcode[e * 3 + d] = code[0] * 3 + code[1];
    }
  free(vol);
  free(area);
}

/* ------------------------------------------------------------------------------ operator */
/* grad[e][a][q] = sum_c dxi_c/dx_a du/dxi_c */
static void gradient(const O1* o, const Level* L, const double* u, double* grad) {
  const int n3 = L->n3;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < o->E; ++e) {
    double du[3][NMAX * NMAX * NMAX];
    for (int c = 0; c < 3; ++c) deriv(L, u + (size_t)e * n3, c, du[c]);
    for (int q = 0; q < n3; ++q) {
      const double* di = L->dxi + ((size_t)e * n3 + q) * 9;
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) s += di[c * 3 + a] * du[c][q];
        grad[((size_t)e * 3 + a) * n3 + q] = s;
      }
    }
  }
}

/* out = A u (sign = 1) or out = g - A u (sign = -1, g given) */
static void apply(const O1* o, Level* L, const double* u, const double* g, double* out) {
  const int n = L->n, n3 = L->n3, n2 = n * n;
  const double nu = o->nu;
  double* grad = L->grad;
  gradient(o, L, u, grad);
#pragma omp parallel for schedule(static)
  for (int e = 0; e < o->E; ++e) {
    double res[NMAX * NMAX * NMAX], flux[NMAX * NMAX * NMAX], lift[3][NMAX * NMAX * NMAX];
    const double* ue = u + (size_t)e * n3;
    for (int q = 0; q < n3; ++q) res[q] = o->kappa * L->wJ[(size_t)e * n3 + q] * ue[q];
    /* volume: sum_b D_b^T [ w J nu grad(xi_b) . grad u ] */
    for (int b = 0; b < 3; ++b) {
      for (int q = 0; q < n3; ++q) {
        const double* di = L->dxi + ((size_t)e * n3 + q) * 9;
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += di[b * 3 + a] * grad[((size_t)e * 3 + a) * n3 + q];
        flux[q] = nu * L->wJ[(size_t)e * n3 + q] * s;
      }
      deriv_t_add(L, flux, b, res);
    }
    memset(lift, 0, sizeof(lift));
    for (int phi = 0; phi < 6; ++phi) {
      const int en = o->nbr[e * 6 + phi];
      const int dir = en < 0 && o->bc[e * 6 + phi] == 1;
      if (en < 0 && !dir) continue;                       /* Neumann: no operator terms */
      const int t = (phi & 1) ? n - 1 : 0;
      const double mu = L->mu[e * 6 + phi];
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          const size_t f = ((size_t)e * 6 + phi) * n2 + a * n + b;
          const double ws = L->fws[f], *nv = L->fn + f * 3;
          const int qi = face_node(n, phi, a, b, t);
          double dn_own = 0.0;
          for (int x = 0; x < 3; ++x) dn_own += nv[x] * grad[((size_t)e * 3 + x) * n3 + qi];
          double row, sigma;
          if (!dir) {
            const int tn = (OPP[phi] & 1) ? n - 1 : 0;
            const int qn = face_node(n, OPP[phi], a, b, tn);
            double dn_nb = 0.0;                          /* neighbour's flux, own normal */
            for (int x = 0; x < 3; ++x) dn_nb += nv[x] * grad[((size_t)en * 3 + x) * n3 + qn];
            const double jmp = ue[qi] - u[(size_t)en * n3 + qn];
            row = mu * nu * ws * jmp - 0.5 * ws * nu * (dn_own + dn_nb);
            sigma = -0.5 * nu * ws * jmp;
          } else {
            row = 2.0 * mu * nu * ws * ue[qi] - ws * nu * dn_own;
            sigma = -nu * ws * ue[qi];
          }
          res[qi] += row;
          const double* di = L->dxi + ((size_t)e * n3 + qi) * 9;
          for (int c = 0; c < 3; ++c) {
            double nc = 0.0;
            for (int x = 0; x < 3; ++x) nc += nv[x] * di[c * 3 + x];
            lift[c][qi] += sigma * nc;
          }
        }
    }
    for (int c = 0; c < 3; ++c) deriv_t_add(L, lift[c], c, res);
    double* oe = out + (size_t)e * n3;
    if (g) {
      for (int q = 0; q < n3; ++q) oe[q] = g[(size_t)e * n3 + q] - res[q];
    } else {
      for (int q = 0; q < n3; ++q) oe[q] = res[q];
    }
  }
}

/* b = w J f + Dirichlet terms (2 mu nu omega s u_D and the lifting -nu omega s u_D n.grad phi) */
static void rhs(const O1* o, Level* L, const double* f, const double* uD, double* b) {
  const int n = L->n, n3 = L->n3, n2 = n * n;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < o->E; ++e) {
    double res[NMAX * NMAX * NMAX], lift[3][NMAX * NMAX * NMAX];
    for (int q = 0; q < n3; ++q) res[q] = L->wJ[(size_t)e * n3 + q] * f[(size_t)e * n3 + q];
    memset(lift, 0, sizeof(lift));
    if (uD) {
      for (int phi = 0; phi < 6; ++phi) {
        if (o->nbr[e * 6 + phi] >= 0 || o->bc[e * 6 + phi] != 1) continue;
        const int t = (phi & 1) ? n - 1 : 0;
        for (int a = 0; a < n; ++a)
          for (int bb = 0; bb < n; ++bb) {
            const size_t fi = ((size_t)e * 6 + phi) * n2 + a * n + bb;
            const double ws = L->fws[fi], *nv = L->fn + fi * 3;
            const int qi = face_node(n, phi, a, bb, t);
            const double ud = uD[(size_t)e * n3 + qi];
            res[qi] += 2.0 * L->mu[e * 6 + phi] * o->nu * ws * ud;
            const double* di = L->dxi + ((size_t)e * n3 + qi) * 9;
            for (int c = 0; c < 3; ++c) {
              double nc = 0.0;
              for (int x = 0; x < 3; ++x) nc += nv[x] * di[c * 3 + x];
              lift[c][qi] += -o->nu * ws * ud * nc;
            }
          }
      }
    }
    for (int c = 0; c < 3; ++c) deriv_t_add(L, lift[c], c, res);
    memcpy(b + (size_t)e * n3, res, n3 * sizeof(double));
  }
}

/* ------------------------------------------------------------------------------ Schwarz */
/* z = sum_e R_s^T W^e (A~_s^e)^-1 R_s r: fast-diagonalisation solves in parallel, then the
   weighted scatter in element order */
static void schwarz(const O1* o, Level* L, const double* r, double* z) {
  const int n = L->n, n3 = L->n3, E = o->E;
  const int NS = n + 2 * L->m, T = NS * NS * NS;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < E; ++e) {
    const Variant* v[3] = {&L->var[L->vcode[e * 3 + 0]], &L->var[L->vcode[e * 3 + 1]], &L->var[L->vcode[e * 3 + 2]]};
    const int n1 = v[0]->nv, n2 = v[1]->nv, n3s = v[2]->nv;
    double rs[NSMAX * NSMAX * NSMAX], t1[NSMAX * NSMAX * NSMAX], t2[NSMAX * NSMAX * NSMAX];
    /* gather r_s = R_s r */
    for (int s3 = 0; s3 < n3s; ++s3)
      for (int s2 = 0; s2 < n2; ++s2)
        for (int s1 = 0; s1 < n1; ++s1) {
          const int m1 = v[0]->map[s1], m2 = v[1]->map[s2], m3 = v[2]->map[s3];
          const int src = o->nb27[(size_t)e * 27 + (m3 >> 6) * 9 + (m2 >> 6) * 3 + (m1 >> 6)];
          rs[(s3 * n2 + s2) * n1 + s1] = r[(size_t)src * n3 + ((m3 & 63) * n + (m2 & 63)) * n + (m1 & 63)];
        }
    /* t = (S3^T x S2^T x S1^T) r_s */
    for (int s3 = 0; s3 < n3s; ++s3)
      for (int s2 = 0; s2 < n2; ++s2)
        for (int a = 0; a < n1; ++a) {
          double s = 0.0;
          for (int i = 0; i < n1; ++i) s += v[0]->S[i * n1 + a] * rs[(s3 * n2 + s2) * n1 + i];
          t1[(s3 * n2 + s2) * n1 + a] = s;
        }
    for (int s3 = 0; s3 < n3s; ++s3)
      for (int b = 0; b < n2; ++b)
        for (int a = 0; a < n1; ++a) {
          double s = 0.0;
          for (int j = 0; j < n2; ++j) s += v[1]->S[j * n2 + b] * t1[(s3 * n2 + j) * n1 + a];
          t2[(s3 * n2 + b) * n1 + a] = s;
        }
    const double* g = L->gco + (size_t)e * 4;
    for (int c = 0; c < n3s; ++c)
      for (int b = 0; b < n2; ++b)
        for (int a = 0; a < n1; ++a) {
          double s = 0.0;
          for (int k = 0; k < n3s; ++k) s += v[2]->S[k * n3s + c] * t2[(k * n2 + b) * n1 + a];
          /* divide by g0 + g1 lam1_a + g2 lam2_b + g3 lam3_c */
          t1[(c * n2 + b) * n1 + a] = s / (g[0] + g[1] * v[0]->lam[a] + g[2] * v[1]->lam[b] + g[3] * v[2]->lam[c]);
        }
    /* du = (S3 x S2 x S1) t */
    for (int k = 0; k < n3s; ++k)
      for (int b = 0; b < n2; ++b)
        for (int a = 0; a < n1; ++a) {
          double s = 0.0;
          for (int c = 0; c < n3s; ++c) s += v[2]->S[k * n3s + c] * t1[(c * n2 + b) * n1 + a];
          t2[(k * n2 + b) * n1 + a] = s;
        }
    for (int k = 0; k < n3s; ++k)
      for (int j = 0; j < n2; ++j)
        for (int a = 0; a < n1; ++a) {
          double s = 0.0;
          for (int b = 0; b < n2; ++b) s += v[1]->S[j * n2 + b] * t2[(k * n2 + b) * n1 + a];
          t1[(k * n2 + j) * n1 + a] = s;
        }
    double* tile = L->tiles + (size_t)e * T;
    for (int k = 0; k < n3s; ++k)
      for (int j = 0; j < n2; ++j)
        for (int i = 0; i < n1; ++i) {
          double s = 0.0;
          for (int a = 0; a < n1; ++a) s += v[0]->S[i * n1 + a] * t1[(k * n2 + j) * n1 + a];
          tile[(k * n2 + j) * n1 + i] = v[2]->W[k] * v[1]->W[j] * v[0]->W[i] * s;
        }
  }
  memset(z, 0, (size_t)L->ndof * sizeof(double));
  for (int e = 0; e < E; ++e) {
    const Variant* v[3] = {&L->var[L->vcode[e * 3 + 0]], &L->var[L->vcode[e * 3 + 1]], &L->var[L->vcode[e * 3 + 2]]};
    const int n1 = v[0]->nv, n2 = v[1]->nv, n3s = v[2]->nv;
    const double* tile = L->tiles + (size_t)e * T;
    for (int s3 = 0; s3 < n3s; ++s3)
      for (int s2 = 0; s2 < n2; ++s2)
        for (int s1 = 0; s1 < n1; ++s1) {
          const int m1 = v[0]->map[s1], m2 = v[1]->map[s2], m3 = v[2]->map[s3];
          const int dst = o->nb27[(size_t)e * 27 + (m3 >> 6) * 9 + (m2 >> 6) * 3 + (m1 >> 6)];
          z[(size_t)dst * n3 + ((m3 & 63) * n + (m2 & 63)) * n + (m1 & 63)] += tile[(s3 * n2 + s2) * n1 + s1];
        }
  }
}

/* ------------------------------------------------------------------------------ transfers */
/* kind 0: out = P in; 1: out += R in (R = I^T); 2: out += I (in - in2) */
static void transfer(const O1* o, const Level* F, const Level* C, int kind, const double* in, const double* in2,
                     double* out) {
  const int nf = F->n, nc = F->nc, nf3 = F->n3, nc3 = C->n3;
  double Rm[NMAX * NMAX];
  for (int a = 0; a < nc; ++a)
    for (int b = 0; b < nf; ++b) Rm[a * nf + b] = F->I[b * nc + a];
#pragma omp parallel for schedule(static)
  for (int e = 0; e < o->E; ++e) {
    double tmp[NMAX * NMAX * NMAX], res[NMAX * NMAX * NMAX];
    if (kind == 0) {
      tensor3(F->P, nc, nf, in + (size_t)e * nf3, out + (size_t)e * nc3);
    } else if (kind == 1) {
      tensor3(Rm, nc, nf, in + (size_t)e * nf3, res);
      for (int q = 0; q < nc3; ++q) out[(size_t)e * nc3 + q] += res[q];
    } else {
      for (int q = 0; q < nc3; ++q) tmp[q] = in[(size_t)e * nc3 + q] - (in2 ? in2[(size_t)e * nc3 + q] : 0.0);
      tensor3(F->I, nf, nc, tmp, res);
      for (int q = 0; q < nf3; ++q) out[(size_t)e * nf3 + q] += res[q];
    }
  }
}

/* ------------------------------------------------------------------------------ solvers */
static void was(O1* o, Level* L, double* u, const double* g, int n_i) {
  for (int it = 0; it < n_i; ++it) {
    apply(o, L, u, g, L->r);
    schwarz(o, L, L->r, L->z);
    const int64_t N = L->ndof;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) u[i] += L->z[i];
  }
}

/* Alg. 6 with p = z in the first iteration and the flexible beta; stops after n_i iterations
   or once ||r|| <= r_max.  Returns the iteration count. */
static int scg(O1* o, Level* L, double* u, const double* f, int n_i, double r_max) {
  const int64_t N = L->ndof;
  double *r = L->r, *z = L->z, *p = L->pv, *q = L->q, *r0 = L->r0;
  apply(o, L, u, f, r);
  double gamma = 0.0;
  int it = 0;
  for (int i = 1; i <= n_i; ++i) {
    schwarz(o, L, r, z);
    if (i > 1) {
      double zr = 0.0, zr0 = 0.0;
#pragma omp parallel for reduction(+ : zr, zr0) schedule(static)
      for (int64_t k = 0; k < N; ++k) { zr += z[k] * r[k]; zr0 += z[k] * r0[k]; }
      const double beta = (zr - zr0) / gamma;
#pragma omp parallel for schedule(static)
      for (int64_t k = 0; k < N; ++k) p[k] = beta * p[k] + z[k];
    } else {
      memcpy(p, z, (size_t)N * sizeof(double));
    }
    apply(o, L, p, NULL, q);
    gamma = dot(N, z, r);
    const double alpha = gamma / dot(N, p, q);
    double rr = 0.0;
#pragma omp parallel for reduction(+ : rr) schedule(static)
    for (int64_t k = 0; k < N; ++k) {
      r0[k] = r[k];
      r[k] -= alpha * q[k];
      u[k] += alpha * p[k];
      rr += r[k] * r[k];
    }
    it = i;
    if (sqrt(rr) <= r_max) break;
  }
  return it;
}

typedef struct {
  int smoother;                   /* 0 WAS, 1 SCG */
  int ns1, ns2;
  int root_maxit;
  double root_rtol;
} CycleOpts;

static void smooth(O1* o, Level* L, double* u, const double* g, int n, const CycleOpts* c) {
  if (n <= 0) return;
  if (c->smoother == 0) was(o, L, u, g, n);
  else scg(o, L, u, g, n, 0.0);
}

static int root_solve(O1* o, double* u, const double* g, const CycleOpts* c) {
  Level* L = &o->lv[0];
  apply(o, L, u, g, L->r);
  const double r0 = sqrt(dot(L->ndof, L->r, L->r));
  return scg(o, L, u, g, c->root_maxit, c->root_rtol * r0);
}

/* Alg. 2 with global p-coarsening; u_top and f_top are the finest level's iterate and rhs */
static int vcycle(O1* o, double* u_top, const double* f_top, const CycleOpts* c) {
  const int Lc = o->L;
  double* u[64];
  const double* g[64];
  for (int l = 0; l < Lc; ++l) { u[l] = o->lv[l].u; g[l] = o->lv[l].g; }
  u[Lc - 1] = u_top;
  g[Lc - 1] = f_top;
  for (int l = Lc - 1; l >= 1; --l) {
    Level *F = &o->lv[l], *C = &o->lv[l - 1];
    smooth(o, F, u[l], g[l], c->ns1, c);
    apply(o, F, u[l], g[l], F->r);                         /* r = g - A u */
    transfer(o, F, C, 0, u[l], NULL, C->ubar);            /* ubar = P u */
    memcpy(C->u, C->ubar, (size_t)C->ndof * sizeof(double));
    apply(o, C, C->ubar, NULL, C->g);                     /* g = A ubar + R r */
    transfer(o, F, C, 1, F->r, NULL, C->g);
  }
  const int it = root_solve(o, o->lv[0].u, o->lv[0].g, c);
  for (int l = 1; l < Lc; ++l) {
    Level *F = &o->lv[l], *C = &o->lv[l - 1];
    transfer(o, F, C, 2, C->u, C->ubar, u[l]);            /* u += I (u_c - ubar) */
    smooth(o, F, u[l], g[l], c->ns2, c);
  }
  return it;
}

/* ------------------------------------------------------------------------------ C ABI */
static void* xalloc(size_t n) {
  void* p = calloc(n ? n : 1, 1);
  return p;
}

/* Create the hierarchy: L levels with degrees deg[0] (root) .. deg[L-1] (finest), E elements,
   face neighbours nbr [E][6] (-1 boundary), boundary codes bc [E][6] (1 Dirichlet, 2 Neumann).
   The finest coordinates follow with o1_set_coords after every level's tables are set. */
void* o1_create(int L, const int* deg, int E, const int* nbr, const int* bc, double kappa, double nu,
                double mu_star) {
  O1* o = (O1*)xalloc(sizeof(O1));
  o->L = L;
  o->E = E;
  o->kappa = kappa;
  o->nu = nu;
  o->mu_star = mu_star;
  o->nbr = (int*)xalloc((size_t)E * 6 * sizeof(int));
  o->bc = (int*)xalloc((size_t)E * 6 * sizeof(int));
  memcpy(o->nbr, nbr, (size_t)E * 6 * sizeof(int));
  memcpy(o->bc, bc, (size_t)E * 6 * sizeof(int));
  o->lv = (Level*)xalloc((size_t)L * sizeof(Level));
  for (int l = 0; l < L; ++l) {
    Level* V = &o->lv[l];
    V->p = deg[l];
    V->n = deg[l] + 1;
    V->n3 = V->n * V->n * V->n;
    V->ndof = (int64_t)E * V->n3;
  }
  /* 27-neighbourhood by walking face neighbours along xi_1, then xi_2, then xi_3 */
  o->nb27 = (int*)xalloc((size_t)E * 27 * sizeof(int));
  for (int e = 0; e < E; ++e)
    for (int d3 = -1; d3 <= 1; ++d3)
      for (int d2 = -1; d2 <= 1; ++d2)
        for (int d1 = -1; d1 <= 1; ++d1) {
          const int dd[3] = {d1, d2, d3};
          int cur = e;
          for (int d = 0; d < 3 && cur >= 0; ++d)
            if (dd[d]) cur = nbr[cur * 6 + 2 * d + (dd[d] > 0)];
          o->nb27[(size_t)e * 27 + (d3 + 1) * 9 + (d2 + 1) * 3 + (d1 + 1)] = cur;
        }
  return o;
}

/* Tables of level l (0 = root): GLL x, w; D [n][n]; rows 0 and 1 of the inverse Legendre
   Vandermonde matrix; overlap m and the 9 variants (nv [9], map [9][NSMAX], S [9][NSMAX^2]
   with S[i * nv + a], lam and W [9][NSMAX]); P [nc][n] and I [n][nc] to the next coarser
   level (nc = 0 on the root). */
void o1_set_level(void* h, int l, const double* x, const double* w, const double* D, const double* v0,
                  const double* v1, int m, const int* nv, const int* map, const double* S, const double* lam,
                  const double* W, int nc, const double* P, const double* I) {
  O1* o = (O1*)h;
  Level* L = &o->lv[l];
  const int n = L->n;
  memcpy(L->x, x, n * sizeof(double));
  memcpy(L->w, w, n * sizeof(double));
  memcpy(L->D, D, (size_t)n * n * sizeof(double));
  memcpy(L->v0, v0, n * sizeof(double));
  memcpy(L->v1, v1, n * sizeof(double));
  L->m = m;
  for (int v = 0; v < 9; ++v) {
    L->var[v].nv = nv[v];
    memcpy(L->var[v].map, map + v * NSMAX, NSMAX * sizeof(int));
    memcpy(L->var[v].S, S + (size_t)v * NSMAX * NSMAX, NSMAX * NSMAX * sizeof(double));
    memcpy(L->var[v].lam, lam + v * NSMAX, NSMAX * sizeof(double));
    memcpy(L->var[v].W, W + v * NSMAX, NSMAX * sizeof(double));
  }
  L->nc = nc;
  if (nc) {
    memcpy(L->P, P, (size_t)nc * n * sizeof(double));
    memcpy(L->I, I, (size_t)n * nc * sizeof(double));
  }
}

/* Finest coordinates X [E][3][n^3]; coarser levels take the fine map evaluated at their GLL
   nodes (P applied per element), then every level's geometry and work vectors are built.
   Returns 0, or -1 when a map is not orientation preserving. */
int o1_set_coords(void* h, const double* X) {
  O1* o = (O1*)h;
  const int E = o->E;
  for (int l = o->L - 1; l >= 0; --l) {
    Level* L = &o->lv[l];
    const int n3 = L->n3, n = L->n, n2 = n * n;
    L->X = (double*)xalloc((size_t)E * 3 * n3 * sizeof(double));
    if (l == o->L - 1) {
      memcpy(L->X, X, (size_t)E * 3 * n3 * sizeof(double));
    } else {
      const Level* F = &o->lv[l + 1];
#pragma omp parallel for schedule(static)
      for (int c = 0; c < 3 * E; ++c) tensor3(F->P, n, F->n, F->X + (size_t)c * F->n3, L->X + (size_t)c * n3);
    }
    L->wJ = (double*)xalloc((size_t)E * n3 * sizeof(double));
    L->dxi = (double*)xalloc((size_t)E * n3 * 9 * sizeof(double));
    L->fws = (double*)xalloc((size_t)E * 6 * n2 * sizeof(double));
    L->fn = (double*)xalloc((size_t)E * 6 * n2 * 3 * sizeof(double));
    L->mu = (double*)xalloc((size_t)E * 6 * sizeof(double));
    L->gco = (double*)xalloc((size_t)E * 4 * sizeof(double));
    L->vcode = (int*)xalloc((size_t)E * 3 * sizeof(int));
    geometry(o, L);
    const size_t nv = (size_t)L->ndof * sizeof(double);
    L->u = (double*)xalloc(nv);
    L->g = (double*)xalloc(nv);
    L->ubar = (double*)xalloc(nv);
    L->r = (double*)xalloc(nv);
    L->z = (double*)xalloc(nv);
    L->pv = (double*)xalloc(nv);
    L->q = (double*)xalloc(nv);
    L->r0 = (double*)xalloc(nv);
    L->grad = (double*)xalloc(3 * nv);
    const int NS = n + 2 * L->m;
    L->tiles = (double*)xalloc((size_t)E * NS * NS * NS * sizeof(double));
    for (int64_t q = 0; q < (int64_t)E * n3; ++q)
      if (!(L->wJ[q] > 0)) return -1;
  }
  return 0;
}

void o1_destroy(void* h) {
  O1* o = (O1*)h;
  if (!o) return;
  for (int l = 0; l < o->L; ++l) {
    Level* L = &o->lv[l];
    void* ps[] = {L->X, L->wJ, L->dxi, L->fws, L->fn, L->mu, L->gco, L->vcode, L->u, L->g, L->ubar,
                  L->r, L->z, L->pv, L->q, L->r0, L->grad, L->tiles};
    for (size_t i = 0; i < sizeof(ps) / sizeof(ps[0]); ++i) free(ps[i]);
  }
  free(o->lv);
  free(o->nbr);
  free(o->bc);
  free(o->nb27);
  free(o);
}

/* level numbers count from 1 (root) as in the paper */
void o1_apply(void* h, int level, const double* u, double* out) {
  O1* o = (O1*)h;
  apply(o, &o->lv[level - 1], u, NULL, out);
}
void o1_residual(void* h, int level, const double* u, const double* g, double* out) {
  O1* o = (O1*)h;
  apply(o, &o->lv[level - 1], u, g, out);
}
void o1_rhs(void* h, const double* f, const double* uD, double* b) {
  O1* o = (O1*)h;
  rhs(o, &o->lv[o->L - 1], f, uD, b);
}
void o1_schwarz(void* h, int level, const double* r, double* z) {
  O1* o = (O1*)h;
  schwarz(o, &o->lv[level - 1], r, z);
}
/* kind 0 project, 1 restrict (out = R in), 2 prolong_add (out += I in) between level and level-1 */
void o1_transfer(void* h, int level, int kind, const double* in, double* out) {
  O1* o = (O1*)h;
  Level *F = &o->lv[level - 1], *C = &o->lv[level - 2];
  if (kind == 1) memset(out, 0, (size_t)C->ndof * sizeof(double));
  transfer(o, F, C, kind, in, NULL, out);
}
void o1_smooth(void* h, int level, int smoother, double* u, const double* g, int n) {
  O1* o = (O1*)h;
  CycleOpts c = {smoother, 0, 0, 500, 0.0};
  smooth(o, &o->lv[level - 1], u, g, n, &c);
}

/* FAS V-cycles from u until ||f - A u|| <= rtol ||f - A u_0|| or max_cycles; hist
   [max_cycles + 1] receives the relative residuals (entry 0 = 1) and root_iters [max_cycles]
   the root SCG iteration counts.  Returns the number of cycles run. */
int o1_solve(void* h, double* u, const double* f, int smoother, int ns1, int ns2, int root_maxit, double root_rtol,
             int max_cycles, double rtol, double* hist, int* root_iters) {
  O1* o = (O1*)h;
  Level* T = &o->lv[o->L - 1];
  CycleOpts c = {smoother, ns1, ns2, root_maxit, root_rtol};
  apply(o, T, u, f, T->r);
  const double r0 = sqrt(dot(T->ndof, T->r, T->r));
  hist[0] = 1.0;
  int k = 0;
  while (k < max_cycles) {
    const int it = vcycle(o, u, f, &c);
    if (root_iters) root_iters[k] = it;
    apply(o, T, u, f, T->r);
    ++k;
    hist[k] = r0 > 0 ? sqrt(dot(T->ndof, T->r, T->r)) / r0 : 0.0;
    if (hist[k] <= rtol) break;
  }
  return k;
}

int o1_threads(void) { return omp_get_max_threads(); }
