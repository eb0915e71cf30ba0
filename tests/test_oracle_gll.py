"""Pins of the oracle's GLL tables against textbook facts (Sec. 2.2, Remark on basis functions)."""
import numpy as np
import pytest

from oracle.gll import gll, diff_matrix, lagrange_eval
from oracle import transfer as tr


def test_closed_forms():
    x, w = gll(1)
    assert np.allclose(x, [-1, 1], atol=0) and np.allclose(w, [1, 1], atol=1e-15)
    x, w = gll(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15) and np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = gll(4)
    r = np.sqrt(3 / 7)
    assert np.allclose(x, [-1, -r, 0, r, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 7, 8, 12, 16])
def test_quadrature_exactness(p):
    x, w = gll(p)
    assert abs(w.sum() - 2) < 1e-14
    for k in range(0, 2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13 * max(1, p)
    # degree 2p is not integrated exactly (GLL has precision 2p-1)
    if p >= 1:
        k = 2 * p
        assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 4, 7, 8, 16])
def test_differentiation(p):
    x, _ = gll(p)
    D = diff_matrix(p)
    assert abs(D[0, 0] + p * (p + 1) / 4) < 1e-14 and abs(D[p, p] - p * (p + 1) / 4) < 1e-14
    assert np.abs(D @ np.ones(p + 1)).max() < 1e-12 * p * p
    for k in range(1, p + 1):
        assert np.abs(D @ x ** k - k * x ** (k - 1)).max() < 1e-11 * p ** 2


@pytest.mark.parametrize("pc,pf", [(1, 2), (2, 4), (3, 7), (4, 8), (1, 3)])
def test_transfers(pc, pf):
    I = tr.interp_1d(pc, pf)
    P = tr.interp_1d(pf, pc)
    assert np.abs(P @ I - np.eye(pc + 1)).max() < 1e-13         # nested spaces (Sec. 3.2)
    xc, _ = gll(pc)
    xf, _ = gll(pf)
    for k in range(pc + 1):                                     # I reproduces degree <= pc
        assert np.abs(I @ xc ** k - xf ** k).max() < 1e-13
    rng = np.random.default_rng(3)
    uc = rng.standard_normal((2, pc + 1, pc + 1, pc + 1))
    rf = rng.standard_normal((2, pf + 1, pf + 1, pf + 1))
    # R = I^T: <R rf, uc> = <rf, I uc>
    lhs = np.sum(tr.restrict(pc, pf, rf) * uc)
    rhs = np.sum(rf * tr.prolong(pc, pf, uc))
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_lagrange_cardinal():
    x, _ = gll(5)
    assert np.abs(lagrange_eval(x, x) - np.eye(6)).max() < 1e-14
