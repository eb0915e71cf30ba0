"""Pins of the oracle's Schwarz smoother (Sec. 4.3.1) against independent facts."""
import numpy as np
import pytest

from oracle import operator as op, solvers as sv, dense as dn
from oracle.gll import gll
from oracle.mesh import Mesh
from oracle.schwarz import Schwarz, variant_1d, surrogate_dx, overlap_layers, quintic
from oracle.sipg1d import sipg_1d
from paper_2608_14123_amd import workloads as W


def cart_mesh(p, ne, lengths=(1.0, 1.0, 1.0)):
    nbr, bc = W.box_topology(ne, ne, ne)
    x, _ = gll(p)
    X = W.element_coords(W.box_vertices(ne, ne, ne, lengths=lengths), x)
    return Mesh(p, X, nbr, bc)


@pytest.mark.parametrize("p,m", [(2, 1), (4, 1), (4, 2), (7, 1), (8, 1), (8, 3)])
@pytest.mark.parametrize("lr", [('i', 'i'), ('i', 'd'), ('d', 'i'), ('d', 'd'), ('n', 'i'), ('i', 'n'), ('d', 'n')])
def test_generalized_eigen(p, m, lr):
    v = variant_1d(p, m, lr[0], lr[1], 2.0)
    S, M, L = v['S'], np.diag(v['M']), v['L']
    assert np.abs(S.T @ M @ S - np.eye(len(M))).max() < 1e-13
    assert np.abs(S.T @ L @ S - np.diag(v['lam'])).max() < 1e-12 * np.abs(v['lam']).max()
    assert np.abs(L - L.T).max() < 1e-14 * np.abs(L).max()


@pytest.mark.parametrize("p,m", [(3, 1), (4, 2), (6, 3)])
def test_principal_submatrix_ignores_far_faces(p, m):
    """With m <= p the 1D subdomain block does not depend on the far ends of the patch."""
    n = p + 1
    for far in ('d', 'n'):
        M, L = sipg_1d(p, 5, 2.0, 2.0, far, far)
        sel = list(range(2 * n - m, 2 * n)) + list(range(2 * n, 3 * n)) + list(range(3 * n, 3 * n + m))
        v = variant_1d(p, m, 'i', 'i', 2.0)
        assert np.abs(L[np.ix_(sel, sel)] - v['L']).max() < 1e-12


@pytest.mark.parametrize("p,ne", [(3, 3), (4, 3), (2, 4)])
def test_fd_equals_exact_local_solve_cartesian(p, ne):
    """Uniform Cartesian: the FD solve equals the dense solve with R_s A R_s^T (eq. schwarz:exact)."""
    mesh = cart_mesh(p, ne)
    A = op.assemble(mesh)
    sz = Schwarz(mesh, 1)
    r = np.random.default_rng(1).standard_normal(mesh.n_dof())
    worst = 0.0
    for e in range(mesh.E):
        idx, grp = sz.subdomain_indices(e)
        i = idx.ravel()
        exact = np.linalg.solve(A[np.ix_(i, i)], r[i])
        sel = np.nonzero(grp['els'] == e)[0]
        fd = sz.fd_solve(grp, r[i].reshape((1,) + idx.shape), sel).ravel()
        worst = max(worst, np.abs(fd - exact).max() / np.abs(exact).max())
    assert worst < 1e-12


def test_fd_equals_dense_surrogate_inverse_curved():
    p, ne = 3, 3
    nbr, bc = W.box_topology(ne, ne, ne)
    x, _ = gll(p)
    X = W.element_coords(W.box_vertices(ne, ne, ne), x, lambda Y: W.sine_bump_map(Y, 0.03))
    mesh = Mesh(p, X, nbr, bc)
    lv = sv.Level(mesh, 1)
    B = dn.schwarz_matrix(lv)
    r = np.random.default_rng(2).standard_normal(mesh.n_dof())
    z = lv.B(r).ravel()
    assert np.abs(z - B @ r).max() < 1e-12 * np.abs(z).max()


@pytest.mark.parametrize("p,m", [(4, 1), (7, 1), (8, 2), (5, 3)])
def test_partition_of_unity(p, m):
    mesh = cart_mesh(p, 3)
    sz = Schwarz(mesh, m)
    one = np.zeros(mesh.n_dof())
    for grp in sz.groups.values():
        np.add.at(one, grp['idx'].ravel(), np.broadcast_to(grp['W'][None], grp['idx'].shape).ravel())
    assert np.abs(one - 1).max() < 1e-14


def test_weights_one_layer():
    """m = 1: the two face-node layers of a shared face get 1/2, every other node 1."""
    v = variant_1d(5, 1, 'i', 'i', 2.0)
    assert np.allclose(v['W'], [0.5, 0.5, 1, 1, 1, 1, 0.5, 0.5])
    v = variant_1d(5, 1, 'd', 'i', 2.0)
    assert np.allclose(v['W'], [1, 1, 1, 1, 1, 0.5, 0.5])
    assert abs(quintic(0.5) - 0.5) < 1e-15 and quintic(-1) == 0 and quintic(2) == 1


def test_single_element_box_is_solved_in_one_sweep():
    """One Dirichlet box element: no overlap, A~ = A exactly, so one WAS sweep solves."""
    mesh = cart_mesh(5, 1, lengths=(1.0, 2.0, 0.5))
    lv = sv.Level(mesh, 1)
    f = np.random.default_rng(0).uniform(-1, 1, (1, 6, 6, 6))
    b = op.rhs(mesh, f)
    u = sv.was(lv, np.zeros_like(b), b, 1)
    assert sv.norm(b - lv.A(u)) < 1e-13 * sv.norm(b)


def test_surrogate_cuboid_and_parallelepiped():
    p = 4
    x, _ = gll(p)
    nbr, bc = W.box_topology(1, 1, 1)
    X = W.element_coords(W.box_vertices(1, 1, 1, lengths=(0.5, 2.0, 3.0)), x)
    dx = surrogate_dx(Mesh(p, X, nbr, bc))
    assert np.allclose(dx, [[0.5, 2.0, 3.0]], atol=1e-13)
    # rotated: invariant
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    Xr = np.einsum('ab,ebkji->eakji', Q, X)
    assert np.allclose(surrogate_dx(Mesh(p, Xr, nbr, bc)), dx, atol=1e-13)
    # sheared parallelepiped: product of edges equals the exact volume det(F)
    F = np.array([[1.0, 0.4, 0.1], [0.0, 1.2, 0.3], [0.2, 0.0, 0.9]])
    Xs = np.einsum('ab,ebkji->eakji', F, X)
    ms = Mesh(p, Xs, nbr, bc)
    dxs = surrogate_dx(ms)
    assert abs(np.prod(dxs) - np.linalg.det(F) * 0.5 * 2.0 * 3.0) < 1e-12


def test_overlap_from_delta():
    assert overlap_layers(4, 0.08) == 1       # the paper's default delta at p = 4
    assert overlap_layers(8, 0.04) == 1
    assert overlap_layers(8, 0.16) == 2
