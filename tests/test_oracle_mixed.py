"""Pins of the mixed-degree oracle (addition 2: a degree per element)."""
import numpy as np
import pytest

from oracle import mixed as mx, operator as op, solvers as sv
from oracle.gll import gll
from oracle.mesh import Mesh
from oracle.schwarz import Schwarz
from paper_2608_14123_amd import workloads as W


def mixed_mesh(ne, degrees, map_fn=None, V=None, bc_code=1, kappa=0.0, mu_star=2.0):
    nbr, bc = W.box_topology(ne, ne, ne, bc_code=bc_code)
    V = W.box_vertices(ne, ne, ne) if V is None else V
    X = W.element_coords_mixed(V, degrees, lambda p: gll(p)[0], map_fn)
    return mx.MixedMesh(degrees, X, nbr, bc, kappa=kappa, mu_star=mu_star), X, nbr, bc


def test_equal_degrees_reduce_to_the_uniform_operator():
    ne, p = 3, 3
    mp = lambda Y: W.sine_bump_map(Y, 0.03)
    mm, X, nbr, bc = mixed_mesh(ne, np.full(ne ** 3, p), mp)
    m = Mesh(p, np.stack(X), nbr, bc)
    u = np.random.default_rng(0).standard_normal(mm.n_dof())
    assert np.abs(mm.apply(u) - op.apply(m, u).ravel()).max() < 1e-12
    sz_u, sz_m = Schwarz(m, 1), mx.MixedSchwarz(mm, 1)
    assert np.abs(sz_m.apply(u) - sz_u.apply(u).ravel()).max() < 1e-12


@pytest.mark.parametrize('degs', [[2, 3, 2, 4, 3, 2, 2, 3], [1, 2, 3, 4, 4, 3, 2, 1]])
def test_mixed_operator_symmetric_positive(degs):
    mm, *_ = mixed_mesh(2, np.array(degs), lambda Y: W.sine_bump_map(Y, 0.03))
    A = mm.assemble()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


def test_mixed_constants_in_kernel_and_linear_patch():
    degs = np.array([2, 3, 4, 2, 3, 2, 4, 3, 2, 2, 3, 4, 2, 3, 4, 2, 3, 4, 2, 2, 3, 2, 4, 3, 3, 2, 4])
    # Neumann box, kappa = 0: constants are in the kernel
    mm, *_ = mixed_mesh(3, degs, lambda Y: W.sine_bump_map(Y, 0.03), bc_code=2)
    assert np.abs(mm.apply(np.ones(mm.n_dof()))).max() < 1e-12
    # affine map, linear solution with its Dirichlet data is reproduced exactly
    Amat = np.array([[1, 0.2, 0.0], [0.1, 1.0, 0.3], [0.0, 0.1, 1.0]])
    mm, X, *_ = mixed_mesh(3, degs, lambda Y: Y @ Amat.T)
    ul = np.concatenate([(1 + 2 * x[0] - x[1] + 0.5 * x[2]).ravel() for x in X])
    b = mm.rhs(np.zeros(mm.n_dof()), uD=ul)
    assert np.abs(mm.apply(ul) - b).max() < 1e-11


def test_front_degree_rule_matches_the_histogram():
    d = W.front_degrees(27)
    vals, cnt = np.unique(d, return_counts=True)
    assert dict(zip(vals.tolist(), cnt.tolist())) == {2: 11809, 3: 1190, 4: 1254, 5: 1196, 6: 1140, 7: 1103, 8: 1991}
    assert int(((d + 1) ** 3).sum()) == 3217284


def test_mixed_vcycle_converges_to_the_direct_solution():
    """Front centred outside the domain (as in the paper's wave-front test), degrees 2..4."""
    ne, c = 2, (-0.05, -0.05, -0.05)
    degs = np.array([4, 3, 3, 2, 3, 2, 2, 2])
    nbr, bc = W.box_topology(ne, ne, ne)
    V = W.box_vertices(ne, ne, ne)
    X = W.element_coords_mixed(V, degs, lambda p: gll(p)[0])
    levels = mx.build_mixed_levels(degs, X, nbr, bc, m=1)
    top = levels[-1].mesh
    f = np.concatenate([W.front_source(x, alpha=3.0, r0=0.5, center=c).ravel() for x in X])
    uD = np.concatenate([W.front_solution(x, alpha=3.0, r0=0.5, center=c).ravel() for x in X])
    b = top.rhs(f, uD=uD)
    u, hist = mx.solve(levels, np.zeros(top.n_dof()), b, sv.Options('scg', 3, 2, root_rtol=1e-12), max_cycles=30,
                       rtol=1e-12)
    assert hist[-1] <= 1e-12
    uex = np.linalg.solve(top.assemble(), b)
    assert np.abs(u - uex).max() <= 1e-9 * np.abs(uex).max()
    assert np.abs(u - uD).max() < 0.05            # the discrete solution approximates the front
