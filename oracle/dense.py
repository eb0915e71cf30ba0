"""Brute-force dense versions of the solver pieces (oracle; test infrastructure only).

Tiny meshes only.  Everything is an explicit matrix built by a route that
differs from the matrix-free oracle: the Schwarz matrix B is assembled from
0/1 restriction matrices R_s, the diagonal weights and the dense inverse of
the Kronecker-assembled surrogate A~ (eq. schwarz:tpo) rather than by fast
diagonalisation; transfer matrices are block-diagonal Kronecker products.
"""
import numpy as np

from . import operator as op
from . import transfer as tr


def schwarz_matrix(level):
    """B = sum_e R_s^T W^e (A~_s^e)^-1 R_s (eq. schwarz:correction), explicitly."""
    sz = level.schwarz
    N = level.mesh.n_dof()
    B = np.zeros((N, N))
    for grp in sz.groups.values():
        v = grp['v']
        M = [np.diag(v[d]['M']) for d in range(3)]
        Lm = [v[d]['L'] for d in range(3)]
        for gi, e in enumerate(grp['els']):
            g0, g1, g2, g3 = sz.g[e]
            At = (g0 * np.kron(np.kron(M[2], M[1]), M[0]) + g1 * np.kron(np.kron(M[2], M[1]), Lm[0])
                  + g2 * np.kron(np.kron(M[2], Lm[1]), M[0]) + g3 * np.kron(np.kron(Lm[2], M[1]), M[0]))
            idx = grp['idx'][gi].ravel()
            Rs = np.zeros((len(idx), N))
            Rs[np.arange(len(idx)), idx] = 1.0
            Wd = np.diag(grp['W'].ravel())
            B += Rs.T @ Wd @ np.linalg.inv(At) @ Rs
    return B


def transfer_matrices(E, pc, pf):
    """Dense (I, R, P) between degree pc and pf for E elements."""
    Ti = tr.interp_1d(pc, pf)
    Tp = tr.interp_1d(pf, pc)
    I1 = np.kron(np.kron(Ti, Ti), Ti)
    P1 = np.kron(np.kron(Tp, Tp), Tp)
    I = np.kron(np.eye(E), I1)
    P = np.kron(np.eye(E), P1)
    return I, I.T.copy(), P


class DenseHierarchy:
    def __init__(self, levels):
        self.A = [op.assemble(lv.mesh) for lv in levels]
        self.B = [schwarz_matrix(lv) for lv in levels]
        from .hmg import dense_transfers
        self.T = [None] + [dense_transfers(levels[l].down) if getattr(levels[l], 'down', None) is not None
                           else transfer_matrices(levels[l].mesh.E, levels[l - 1].p, levels[l].p)
                           for l in range(1, len(levels))]


def fas_vcycle_dense(H, u_top, f_top, ns1, ns2):
    """Alg. 2 with WAS smoothing and an exact root solve, in explicit matrices."""
    L = len(H.A)
    u = [None] * L
    g = [None] * L
    ubar = [None] * L
    u[-1], g[-1] = u_top.copy(), f_top.copy()

    def was(l, v, rhs, k):
        for _ in range(k):
            v = v + H.B[l] @ (rhs - H.A[l] @ v)
        return v

    for l in range(L - 1, 0, -1):
        I, R, P = H.T[l]
        u[l] = was(l, u[l], g[l], ns1)
        r = g[l] - H.A[l] @ u[l]
        ubar[l - 1] = P @ u[l]
        u[l - 1] = ubar[l - 1].copy()
        g[l - 1] = H.A[l - 1] @ u[l - 1] + R @ r
    u[0] = np.linalg.solve(H.A[0], g[0])
    for l in range(1, L):
        I, R, P = H.T[l]
        u[l] = u[l] + I @ (u[l - 1] - ubar[l - 1])
        u[l] = was(l, u[l], g[l], ns2)
    return u[-1]


def _was_dense(H, l, v, rhs, k):
    for _ in range(k):
        v = v + H.B[l] @ (rhs - H.A[l] @ v)
    return v


def _sub(H, l):
    """The hierarchy of levels 1..l (root first) as a new DenseHierarchy view."""
    S = DenseHierarchy.__new__(DenseHierarchy)
    S.A, S.B, S.T = H.A[:l], H.B[:l], H.T[:l]
    return S


def level_rhs_dense(H, f_top):
    fs = [None] * len(H.A)
    fs[-1] = f_top
    for l in range(len(H.A) - 1, 0, -1):
        fs[l - 1] = H.T[l][1] @ fs[l]
    return fs


def fmg_dense(H, f_top, ns1, ns2):
    """Alg. 4 from a zero start with WAS smoothing and exact root solves, in explicit matrices."""
    L = len(H.A)
    fs = level_rhs_dense(H, f_top)
    u = np.zeros(H.A[0].shape[0])
    for l in range(1, L):
        u = fas_vcycle_dense(_sub(H, l), u, fs[l - 1], ns1, ns2)
        u = H.T[l][0] @ u
    return u


def cmg_dense(H, f_top, ns0):
    """Alg. 3 from a zero start with WAS smoothing and an exact root solve, in explicit matrices."""
    L = len(H.A)
    fs = level_rhs_dense(H, f_top)
    u = np.linalg.solve(H.A[0], fs[0])
    for l in range(1, L - 1):
        u = _was_dense(H, l, H.T[l][0] @ u, fs[l], ns0)
    return H.T[L - 1][0] @ u


def crossover_cycles_dense(H, u, f_top, ns1, ns2, nsc, n):
    """n FAS V-cycles where every cycle after the first starts with nsc - ns2 top-level
    pre-smoothing steps (explicit matrices, WAS, exact root solve)."""
    L = len(H.A)
    for k in range(n):
        pre = ns1 if k == 0 else nsc - ns2
        v = [None] * L
        g = [None] * L
        ub = [None] * L
        v[-1], g[-1] = u.copy(), f_top
        for l in range(L - 1, 0, -1):
            I, R, P = H.T[l]
            v[l] = _was_dense(H, l, v[l], g[l], pre if l == L - 1 else ns1)
            r = g[l] - H.A[l] @ v[l]
            ub[l - 1] = P @ v[l]
            v[l - 1] = ub[l - 1].copy()
            g[l - 1] = H.A[l - 1] @ v[l - 1] + R @ r
        v[0] = np.linalg.solve(H.A[0], g[0])
        for l in range(1, L):
            I, R, P = H.T[l]
            v[l] = _was_dense(H, l, v[l] + I @ (v[l - 1] - ub[l - 1]), g[l], ns2)
        u = v[-1]
    return u
