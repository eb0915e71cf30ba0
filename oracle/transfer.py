"""Transfer operators between p-levels (oracle; test infrastructure only).

Sec. 3.2: coarse-to-fine prolongation I is the embedded interpolation (exact
for nested spaces), the residual restriction is R = I^T, and the solution
projection P evaluates the fine polynomial at the coarse GLL nodes
(embedded interpolation).  All are per-element tensor products of 1D
matrices.
"""
import numpy as np

from .gll import gll, lagrange_eval


def interp_1d(p_from, p_to):
    """T[i, j] = l_j^{p_from}(x_i^{p_to}): evaluate a degree-p_from nodal polynomial at p_to nodes."""
    xf, _ = gll(p_from)
    xt, _ = gll(p_to)
    return lagrange_eval(xf, xt)


def tensor3(T, u):
    """Apply T in each of the three directions of u[e, k, j, i]."""
    return np.einsum('ck,bj,ai,ekji->ecba', T, T, T, u)


def prolong(pc, pf, uc):
    """I: coarse (pc) -> fine (pf) embedded interpolation."""
    return tensor3(interp_1d(pc, pf), uc)


def restrict(pc, pf, rf):
    """R = I^T: fine residual -> coarse."""
    return tensor3(interp_1d(pc, pf).T, rf)


def l2_project_1d(p_from, p_to):
    """Reference-element L2 projection of a degree-p_from nodal polynomial onto degree p_to < p_from
    (Sec. 3.2 names L2 projection beside embedded interpolation): P = (I^T W I)^-1 I^T W with
    I = interp_1d(p_to, p_from) and W the p_from GLL weights.  The p_from GLL rule integrates
    every product involved exactly (degree <= p_to + p_from <= 2 p_from - 1)."""
    I = interp_1d(p_to, p_from)
    _, w = gll(p_from)
    return np.linalg.solve(I.T @ (w[:, None] * I), I.T * w[None, :])


def project(pc, pf, uf, kind='interp'):
    """P: fine solution -> coarse, by evaluation at the coarse GLL nodes (embedded interpolation)
    or by the L2 projection of l2_project_1d (kind 'l2')."""
    T = interp_1d(pf, pc) if kind == 'interp' else l2_project_1d(pf, pc)
    return tensor3(T, uf)


def coarse_coords(pc, pf, X):
    """Coarse-level isoparametric geometry: fine nodal coordinates evaluated at coarse nodes.

    Reading: the paper represents the geometry of every level in that level's
    basis (Remark on basis functions); for p-coarsening the coarse map is the
    embedded interpolation of the fine one.
    """
    T = interp_1d(pf, pc)
    return np.einsum('ck,bj,ai,edkji->edcba', T, T, T, X)


def degree_chain(p):
    """p_L = p, p_{l-1} = max(1, floor(p_l / 2)) down to 1 (p_l = 2^(l-1) for powers of two)."""
    chain = [p]
    while chain[-1] > 1:
        chain.append(max(1, chain[-1] // 2))
    return chain[::-1]
