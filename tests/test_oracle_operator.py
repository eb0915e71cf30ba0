"""Pins of the oracle's SIPG operator (eq. helmholtz:dgm) against facts the mathematics fixes."""
import numpy as np
import pytest

from oracle import operator as op, solvers as sv
from oracle.gll import gll
from oracle.mesh import Mesh
from oracle.sipg1d import sipg_1d
from paper_2608_14123_amd import workloads as W


def mild_map(amp):
    return lambda X: W.sine_bump_map(X, amp)


def make_mesh(p, ne, map_fn=None, periodic=False, bc_code=1, mu_star=2.0, V=None, kappa=0.0):
    nbr, bc = W.box_topology(ne, ne, ne, periodic=(periodic,) * 3, bc_code=bc_code)
    V = W.box_vertices(ne, ne, ne) if V is None else V
    x, _ = gll(p)
    X = W.element_coords(V, x, map_fn)
    return Mesh(p, X, nbr, bc, mu_star=mu_star, kappa=kappa), X


@pytest.mark.parametrize("p,amp", [(2, 0.0), (3, 0.03), (4, 0.03)])
def test_symmetric_positive_definite(p, amp):
    m, _ = make_mesh(p, 2, mild_map(amp) if amp else None)
    A = op.assemble(m)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


def test_indefinite_when_penalty_too_small_on_distorted_mesh():
    """The SIPG form is coercive only for a large enough penalty: with mu_star below 1 it is not."""
    m, _ = make_mesh(3, 2, mild_map(0.03), mu_star=0.3)
    A = op.assemble(m)
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() < 0


@pytest.mark.parametrize("bc_code,periodic", [(2, False), (1, True)])
def test_constants_in_kernel(bc_code, periodic):
    """kappa = 0 with pure Neumann or periodic conditions: A 1 = 0 (curved elements)."""
    amp = 0.0 if periodic else 0.03
    fn = (lambda X: X + 0.01 * np.sin(2 * np.pi * X)) if periodic else mild_map(amp)
    m, _ = make_mesh(3, 3, fn, periodic=periodic, bc_code=bc_code)
    Au = op.apply(m, np.ones((m.E, m.n, m.n, m.n)))
    assert np.abs(Au).max() < 1e-12


@pytest.mark.parametrize("p,ne,lengths", [(3, 2, (1.0, 1.0, 1.0)), (2, 3, (1.0, 1.0, 1.0)), (4, 2, (1.0, 1.0, 1.0))])
def test_kronecker_structure_on_uniform_cartesian(p, ne, lengths):
    """Uniform cubes: A = M x M x L + M x L x M + L x M x M with the 1D SIPG matrices."""
    m, _ = make_mesh(p, ne)
    A = op.assemble(m)
    M1, L1 = sipg_1d(p, ne, 1.0 / ne, 2.0)
    K = np.kron(np.kron(M1, M1), L1) + np.kron(np.kron(M1, L1), M1) + np.kron(np.kron(L1, M1), M1)
    n = p + 1
    perm = np.empty(m.n_dof(), dtype=int)
    c = 0
    for ez in range(ne):
        for ey in range(ne):
            for ex in range(ne):
                for k in range(n):
                    for j in range(n):
                        for i in range(n):
                            perm[c] = ((ez * n + k) * ne * n + ey * n + j) * ne * n + ex * n + i
                            c += 1
    assert np.abs(A - K[np.ix_(perm, perm)]).max() <= 1e-13 * np.abs(A).max()


def test_kappa_term_is_mass():
    m0, X = make_mesh(3, 2, mild_map(0.03))
    m1 = Mesh(3, X, m0.nbr, m0.bc, kappa=2.5)
    u = np.random.default_rng(0).standard_normal((m0.E, 4, 4, 4))
    d = op.apply(m1, u) - op.apply(m0, u)
    assert np.abs(d - 2.5 * m0.w3 * m0.detJ * u).max() < 1e-13


def test_linear_patch_test_affine():
    """SIPG is consistent: a linear exact solution with its Dirichlet data is reproduced exactly."""
    p, ne = 3, 2
    Amat = np.array([[1, 0.2, 0.0], [0.1, 1.0, 0.3], [0.0, 0.1, 1.0]])
    V = W.box_vertices(ne, ne, ne, lengths=(1.0, 2.0, 0.5))
    m, X = make_mesh(p, ne, lambda Y: Y @ Amat.T, V=V)
    ul = 1 + 2 * X[:, 0] - X[:, 1] + 0.5 * X[:, 2]
    b = op.rhs(m, np.zeros_like(ul), uD=ul)
    assert np.abs(op.apply(m, ul) - b).max() < 1e-12


def test_neumann_rhs_patch():
    """Linear u with Neumann data on x=0 and x=1 and Dirichlet elsewhere is also reproduced."""
    p, ne = 2, 2
    nbr, bc = W.box_topology(ne, ne, ne)
    x, _ = gll(p)
    X = W.element_coords(W.box_vertices(ne, ne, ne), x)
    ex = np.arange(ne ** 3) % ne
    bc[(ex == 0), 0] = 2
    bc[(ex == ne - 1), 1] = 2
    m = Mesh(p, X, nbr, bc)
    ul = 0.3 + 1.5 * X[:, 0] + X[:, 1] - 2 * X[:, 2]
    qN = np.zeros_like(ul)
    qN[:, :, :, 0] = -1.5         # nu du/dn on x=0 (outward -x)
    qN[:, :, :, -1] = 1.5         # on x=1
    b = op.rhs(m, np.zeros_like(ul), uD=ul, qN=qN)
    assert np.abs(op.apply(m, ul) - b).max() < 1e-12


def _solve_error(p, ne, amp):
    m, X = make_mesh(p, ne, mild_map(amp) if amp else None)
    levels = sv.build_levels(p, X, m.nbr, m.bc, m=1)
    ue = W.sine_solution(X)
    b = op.rhs(levels[-1].mesh, 3 * np.pi ** 2 * ue)
    u, hist = sv.solve(levels, np.zeros_like(b), b, sv.Options('was', 2, 2), max_cycles=40, rtol=1e-13)
    assert hist[-1] <= 1e-12
    return op.l2_error(levels[-1].mesh, u, ue)


@pytest.mark.slow
def test_h_convergence_rate_cartesian():
    """Order p+1 on rectangular elements with constant nu (Remark on basis functions)."""
    p = 2
    e = [_solve_error(p, ne, 0.0) for ne in (2, 4, 8)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert rates[-1] > p + 1 - 0.3, rates


def test_h_convergence_rate_curved():
    """Order at least p on curved elements."""
    p = 3
    e = [_solve_error(p, ne, 0.03) for ne in (2, 4)]
    assert np.log2(e[0] / e[1]) > p - 0.2


def test_p_convergence_exponential():
    e = [_solve_error(p, 2, 0.0) for p in (2, 3, 4, 5, 6)]
    assert all(e[i + 1] < 0.5 * e[i] for i in range(len(e) - 1)), e
    assert e[-1] < 1e-4


@pytest.mark.parametrize('pf', [2, 3, 4, 7, 8])
def test_l2_projection_is_the_orthogonal_projection(pf):
    """The 1D L2 projection onto degree pc = pf // 2 reproduces coarse polynomials (P I = Id) and
    leaves a residual orthogonal to every coarse polynomial, checked with Gauss-Legendre
    quadrature of pf + 2 points (exact for the products, independent of the GLL rule)."""
    from oracle.transfer import l2_project_1d, interp_1d
    from oracle.gll import lagrange_eval
    pc = max(1, pf // 2)
    P = l2_project_1d(pf, pc)
    assert np.abs(P @ interp_1d(pc, pf) - np.eye(pc + 1)).max() < 1e-13
    xf, _ = gll(pf)
    xc, _ = gll(pc)
    xq, wq = np.polynomial.legendre.leggauss(pf + 2)
    uf = np.random.default_rng(pf).standard_normal(pf + 1)
    res = lagrange_eval(xf, xq) @ uf - lagrange_eval(xc, xq) @ (P @ uf)
    assert np.abs(lagrange_eval(xc, xq).T @ (wq * res)).max() < 1e-13
