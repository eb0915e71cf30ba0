"""Pins of the h-coarsening oracle (Sec. 3.1 multilevel mesh by h-refinement, Sec. 3.2 transfers)."""
import numpy as np
import pytest

from oracle import hmg, operator as op, solvers as sv, dense as dn
from oracle.gll import gll
from oracle.mesh import Mesh
from paper_2608_14123_amd import workloads as W


@pytest.mark.parametrize('p', [1, 2, 3, 4, 7, 8])
def test_projection_inverts_interpolation_and_restriction_is_its_transpose(p):
    """P I = Id: a parent polynomial interpolated to its eight children and evaluated back at the
    parent's nodes (averaged where the children meet, even p) is returned exactly; R = I^T."""
    ht = hmg.HTransfer(p, (4, 2, 2))
    rng = np.random.default_rng(p)
    uc = rng.standard_normal((len(ht.children),) + (p + 1,) * 3)
    assert np.abs(ht.project(ht.prolong(uc)) - uc).max() < 1e-13
    I, R, P = hmg.dense_transfers(ht)
    assert np.array_equal(R, I.T)
    rf = rng.standard_normal(I.shape[0])
    assert np.abs(R @ rf - ht.restrict(rf).ravel()).max() < 1e-13


def test_projection_averages_the_children_at_shared_nodes():
    """Even p: the parent's midpoint nodes lie between children; a piecewise field that jumps there
    is averaged (Sec. 3.2), and a continuous one is reproduced."""
    p = 2
    ht = hmg.HTransfer(p, (2, 2, 2))
    uf = np.zeros((8, 3, 3, 3))
    uf[1] = 1.0                                     # the child bx = 1, by = bz = 0 is one, others zero
    up = ht.project(uf)[0]
    assert up[0, 0, 2] == 1.0 and up[0, 0, 0] == 0.0
    assert abs(up[0, 0, 1] - 0.5) < 1e-15           # on the plane x = 0 between children 0 and 1
    assert abs(up[1, 1, 1] - 0.125) < 1e-15         # the centre is shared by all eight


@pytest.mark.parametrize('periodic', [False, True])
def test_coarse_mesh_equals_the_directly_built_coarse_box(periodic):
    """An affine map: coarsening 4x4x4 elements gives the geometry and topology of the 2x2x2 box."""
    p = 3
    A = np.array([[1.0, 0.2, 0.1], [0.0, 0.9, 0.3], [0.1, 0.0, 1.1]])
    mp = lambda Y: Y @ A.T
    nbr, bc = W.box_topology(4, 4, 4, periodic=(periodic,) * 3)
    X = W.element_coords(W.box_vertices(4, 4, 4), gll(p)[0], mp)
    lv = hmg.build_hlevels(p, X, nbr, bc, (4, 4, 4), 1)
    nbrc, bcc = W.box_topology(2, 2, 2, periodic=(periodic,) * 3)
    Xc = W.element_coords(W.box_vertices(2, 2, 2), gll(p)[0], mp)
    assert np.abs(lv[0].mesh.X - Xc).max() < 1e-13
    assert np.array_equal(lv[0].mesh.nbr, nbrc)
    assert np.array_equal(lv[0].mesh.bc[nbrc < 0], bcc[nbrc < 0])


@pytest.mark.parametrize('p', [2, 3])
def test_h_vcycle_matches_dense_brute_force(p):
    """FAS V-cycle over an h-level (4^3 -> 2^3 at degree p), matrix-free against explicit matrices."""
    nbr, bc = W.box_topology(4, 4, 4)
    X = W.element_coords(W.box_vertices(4, 4, 4), gll(p)[0], lambda Y: W.sine_bump_map(Y, 0.03))
    levels = hmg.build_hlevels(p, X, nbr, bc, (4, 4, 4), 1)
    H = dn.DenseHierarchy(levels)
    b = op.rhs(levels[-1].mesh, W.uniform_nodal(X[:, 0].shape, 2))
    opts = sv.Options('was', 1, 1, root='direct')
    u = np.zeros_like(b)
    ud = u.ravel().copy()
    for _ in range(2):
        u = sv.fas_vcycle(levels, u, b, opts)
        ud = dn.fas_vcycle_dense(H, ud, b.ravel(), 1, 1)
        assert np.abs(u.ravel() - ud).max() <= 1e-12 * np.abs(ud).max()


def test_h_multigrid_converges_to_the_direct_solution():
    """h-FAS-MG-WAS(1,1) on C1 (4^3 unit cubes, p = 4, h-levels 4^3 -> 2^3 -> 1^3, SCG root at
    p = 4): every cycle contracts the residual (0.29 per cycle measured), FMG saves cycles, and
    the iterate reaches the solution of the fine system."""
    p = 4
    nbr, bc = W.box_topology(4, 4, 4)
    X = W.element_coords(W.box_vertices(4, 4, 4), gll(p)[0])
    levels = hmg.build_hlevels(p, X, nbr, bc, (4, 4, 4), 2)
    assert [lv.mesh.E for lv in levels] == [1, 8, 64]
    b = op.rhs(levels[-1].mesh, 3 * np.pi ** 2 * W.sine_solution(X))
    u, h = sv.solve(levels, np.zeros_like(b), b, sv.Options('was', 1, 1), max_cycles=20, rtol=1e-10)
    assert h[-1] <= 1e-10 and all(h[k + 1] < 0.35 * h[k] for k in range(len(h) - 1))
    uf, hf = sv.solve(levels, np.zeros_like(b), b, sv.Options('was', 1, 1, start='fmg'), max_cycles=20)
    assert len(hf) < len(h) and hf[1] < 0.01 * h[1]
    lp = sv.build_levels(p, X, nbr, bc)
    ue, _ = sv.solve(lp, np.zeros_like(b), b, sv.Options('scg', 3, 2), max_cycles=30, rtol=1e-12)
    assert np.abs(u - ue).max() <= 1e-9 * np.abs(ue).max()
