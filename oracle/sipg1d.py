"""1D SIPG matrices on uniform meshes (oracle; test infrastructure only).

The one-dimensional restriction of eq. helmholtz:dgm with nu = 1: elements of
length h, GLL nodes, penalty mu = mu_star p(p+1)/(2h) at every interior point
and at Dirichlet ends (where the form carries the factor 2).  Used (a) to pin
the 3D operator on uniform Cartesian meshes by its Kronecker structure and
(b) to build the 1D subdomain matrices of the Schwarz method (Sec. 4.3.1),
which are principal submatrices of this operator on a 3-element patch.
"""
import numpy as np

from .gll import gll, diff_matrix


def sipg_1d(p, K, h, mu_star, left='d', right='d'):
    """Global (mass, stiffness) of K elements of length h; ends 'd' Dirichlet, 'n' Neumann, 'p' periodic."""
    x, w = gll(p)
    D = diff_matrix(p)
    n = p + 1
    N = K * n
    M = np.zeros((N, N))
    L = np.zeros((N, N))
    mu = mu_star * p * (p + 1) / (2.0 * h)
    d = 2.0 / h                                       # d/dx = (2/h) d/dxi
    for e in range(K):
        sl = slice(e * n, (e + 1) * n)
        M[sl, sl] += (h / 2.0) * np.diag(w)
        L[sl, sl] += (h / 2.0) * d * d * D.T @ np.diag(w) @ D

    def point(eL, eR):
        """interior point between the right end of eL and the left end of eR (n^- = +1)."""
        J = np.zeros(N)
        J[eL * n + p] += 1.0
        J[eR * n + 0] -= 1.0
        A = np.zeros(N)                               # functional v -> {v'}
        A[eL * n:(eL + 1) * n] += 0.5 * d * D[p, :]
        A[eR * n:(eR + 1) * n] += 0.5 * d * D[0, :]
        return mu * np.outer(J, J) - np.outer(A, J) - np.outer(J, A)

    for e in range(K - 1):
        L += point(e, e + 1)
    if left == 'p' or right == 'p':
        L += point(K - 1, 0)
    if left == 'd':                                   # outward n = -1: d_n = -d/dx
        e0 = np.zeros(N); e0[0] = 1.0
        g0 = np.zeros(N); g0[:n] = d * D[0, :]
        L += 2.0 * mu * np.outer(e0, e0) + np.outer(g0, e0) + np.outer(e0, g0)
    if right == 'd':                                  # outward n = +1
        e1 = np.zeros(N); e1[-1] = 1.0
        g1 = np.zeros(N); g1[-n:] = d * D[p, :]
        L += 2.0 * mu * np.outer(e1, e1) - np.outer(g1, e1) - np.outer(e1, g1)
    return M, L
