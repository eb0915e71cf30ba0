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


def _pou_mesh(name):
    if name == 'centre_jump':        # degree 4 in the centre of degree-3 elements: face jumps, and
        degs = np.full(27, 3)        # edge/vertex neighbours of the face neighbours on the other degree
        degs[13] = 4
    elif name == 'random_1to5':      # jumps across faces, edges and vertices in every combination
        degs = np.random.default_rng(3).integers(1, 6, 27)
    else:
        degs = np.full(27, 3)
    mm, *_ = mixed_mesh(3, degs, lambda Y: W.sine_bump_map(Y, 0.03))
    return mm, degs


@pytest.mark.parametrize('name', ['centre_jump', 'random_1to5', 'uniform'])
def test_mixed_schwarz_weights_are_a_partition_of_unity(name, monkeypatch):
    """With every local solve replaced by the identity, the combined correction of Sec. 4.3.1 is
    C^-1 sum_s R_s^T W_s R_s r, which must return r itself at every node: the weighted gather
    and scatter of the apply path form a partition of unity.  Without the normalisation the
    weight sums at degree jumps are 3/4 or 5/4, and on a uniform mesh they are 1 exactly.
    A subdomain reaches only elements of its own degree (zero fill, Sec. 4.3.1 item 5)."""
    mm, degs = _pou_mesh(name)
    sz = mx.MixedSchwarz(mm, 1)
    monkeypatch.setattr(mx.MixedSchwarz, 'local_solve', staticmethod(lambda sd, rs: rs))
    r = np.random.default_rng(1).standard_normal(mm.n_dof())
    assert np.abs(sz.apply(r) - r).max() <= 1e-14 * np.abs(r).max()
    defect = np.abs(sz.C - 1.0).max()
    if name == 'uniform':
        assert defect == 0.0
    else:
        assert 0.2 < defect < 0.3
    owner = np.repeat(np.arange(mm.E), (degs + 1) ** 3)
    for e, sd in enumerate(sz.sub):
        idx = sd['idx'][sd['idx'] >= 0]
        assert np.all(degs[owner[idx]] == degs[e])


def test_mixed_discretisation_converges_at_the_rate_of_its_lower_degree():
    """Manufactured solution u = sin(pi x) sin(pi y) sin(pi z) under the curved map, degree 2 on
    x < 1/2 and 3 beyond (the layout refines self-similarly, so the face between the degrees
    stays a plane).  The L2 error from 2^3 to 4^3 elements falls at about p_min + 1 = 3, the rate
    of the uniform degree-2 discretisation on the same meshes (3.19), with GLL quadrature and
    the mixed-face integration of the finer side; a dropped or mis-signed face term breaks the
    consistency and the rate."""
    errs = []
    for ne in (2, 4):
        ex = np.arange(ne ** 3) % ne
        degs = 2 + (ex >= ne // 2).astype(np.int64)
        nbr, bc = W.box_topology(ne, ne, ne)
        X = W.element_coords_mixed(W.box_vertices(ne, ne, ne), degs, lambda p: gll(p)[0],
                                   lambda Y: W.sine_bump_map(Y, 0.03))
        levels = mx.build_mixed_levels(degs, X, nbr, bc, m=1)
        top = levels[-1].mesh
        uex = np.concatenate([W.sine_solution(x[None])[0].ravel() for x in X])
        b = top.rhs(3 * np.pi ** 2 * uex)
        u, hist = mx.solve(levels, np.zeros_like(b), b, sv.Options('scg', 3, 2, root_rtol=1e-8), max_cycles=20,
                           rtol=1e-8)
        assert hist[-1] <= 1e-8
        e2 = sum(float(np.sum(top.el[e].w3 * top.el[e].detJ[0] * (top.block(u, e) - top.block(uex, e)) ** 2))
                 for e in range(top.E))
        errs.append(np.sqrt(e2))
    rate = np.log2(errs[0] / errs[1])
    assert 2.8 < rate < 3.6, (errs, rate)
