"""Gauss-Lobatto-Legendre tables (oracle; test infrastructure only).

Sec. 2.2 (Remark "Basis functions, geometry and numerical integration"): the
nodal basis uses the p+1 GLL points per direction, and the same points give
the volume and face quadrature.  GLL points are -1, +1 and the roots of
P_p'; the weights are 2 / (p (p+1) P_p(x_j)^2).  All values are FP64.
"""
import numpy as np


def legendre(p, x):
    """Return (P_p(x), P_p'(x)) by the Bonnet three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    P_prev, P = np.ones_like(x), x.copy()
    dP_prev, dP = np.zeros_like(x), np.ones_like(x)
    if p == 0:
        return P_prev, dP_prev
    for k in range(1, p):
        P_next = ((2 * k + 1) * x * P - k * P_prev) / (k + 1)
        # P'_{k+1} = P'_{k-1} + (2k+1) P_k
        dP_next = dP_prev + (2 * k + 1) * P
        P_prev, P = P, P_next
        dP_prev, dP = dP, dP_next
    return P, dP


def gll(p):
    """GLL nodes (ascending) and weights of degree p >= 1."""
    if p < 1:
        raise ValueError("degree must be >= 1")
    if p == 1:
        x = np.array([-1.0, 1.0])
    else:
        c = np.zeros(p + 1)
        c[p] = 1.0
        inner = np.sort(np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c)).real)
        # polish the library roots with Newton on P_p'; P_p'' from Legendre's ODE
        for _ in range(3):
            P, dP = legendre(p, inner)
            d2P = (2.0 * inner * dP - p * (p + 1) * P) / (1.0 - inner ** 2)
            inner = inner - dP / d2P
        x = np.concatenate(([-1.0], inner, [1.0]))
    P, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * P ** 2)
    return x, w


def diff_matrix(p):
    """D[i, j] = l_j'(x_i) for the GLL Lagrange basis (closed form)."""
    x, _ = gll(p)
    P, _ = legendre(p, x)
    n = p + 1
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = P[i] / (P[j] * (x[i] - x[j]))
    D[0, 0] = -p * (p + 1) / 4.0
    D[p, p] = p * (p + 1) / 4.0
    return D


def lagrange_eval(nodes, y):
    """L[i, j] = l_j(y_i): Lagrange polynomials on `nodes` evaluated at `y`."""
    nodes = np.asarray(nodes, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    L = np.ones((len(y), len(nodes)))
    for j in range(len(nodes)):
        for m in range(len(nodes)):
            if m != j:
                L[:, j] *= (y - nodes[m]) / (nodes[j] - nodes[m])
    return L
