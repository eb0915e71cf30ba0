"""Pins of the local-refinement FAS oracle (Sec. 3.1 multilevel mesh, Sec. 3.2 transfers,
eq. helmholtz:fas, Alg. 2 with the frozen update).

* With every element refined there are no frozen elements and the cycle is the global h-MG
  cycle of the h-coarsening oracle (pinned on its own).
* The converged FAS state satisfies eq. helmholtz:fas:converged: it equals the dense solve of
  the composite equations (leaf rows of every level, twigs the projections of their children,
  frozen values interpolated from their leaf parents), built independently of the cycle.
* On a curved box with two nested refinement zones the cycle converges steadily."""
import numpy as np
import pytest

from oracle import hmg, localref as lr, operator as op, solvers as sv
from oracle.gll import gll
from paper_2608_14123_amd import workloads as W


def base_mesh(p, ne, map_fn=None):
    nbr, bc = W.box_topology(ne, ne, ne)
    X = W.element_coords(W.box_vertices(ne, ne, ne), gll(p)[0], map_fn)
    return X, nbr, bc


def near(c, rad):
    return lambda centres: np.linalg.norm(centres - np.asarray(c), axis=1) < rad


def level_b(levels, f_fn):
    """Discrete right-hand side of every level (f at the level's nodes, homogeneous Dirichlet)."""
    out = []
    for lv in levels:
        f = f_fn(lv.mesh.X)
        out.append(op.rhs(lv.mesh, f, uD=np.zeros_like(f)))
    return out


def test_refining_everything_is_global_h_multigrid():
    p, ne = 3, 2
    X, nbr, bc = base_mesh(p, ne)
    levels = lr.build_local_levels(p, (ne,) * 3, X, nbr, bc, [lambda c: np.ones(len(c), bool)], kappa=0.5)
    top = levels[-1]
    assert np.all(top.cls == lr.LEAF) and np.all(levels[0].cls == lr.TWIG)
    # the same fine mesh in box numbering, coarsened by the h-coarsening oracle
    data = lr.build_local_mesh(p, (ne,) * 3, X, nbr, bc, [lambda c: np.ones(len(c), bool)])
    cells = data[-1]['cells']
    nf = 2 * ne
    box_id = cells[:, 0] + nf * (cells[:, 1] + nf * cells[:, 2])
    nbr_f, bc_f = W.box_topology(nf, nf, nf)
    X_f = W.element_coords(W.box_vertices(nf, nf, nf), gll(p)[0])
    assert np.allclose(top.mesh.X, X_f[box_id], atol=1e-14)
    hl = hmg.build_hlevels(p, X_f, nbr_f, bc_f, (nf,) * 3, 1, kappa=0.5)
    rng = np.random.default_rng(4)
    b_box = rng.uniform(-1, 1, (nf ** 3, p + 1, p + 1, p + 1))
    opts = sv.Options('was', 2, 2)
    u_ref, h_ref = sv.solve(hl, np.zeros_like(b_box), b_box, opts, max_cycles=6, rtol=1e-14)
    b = [np.zeros((lv.mesh.E, p + 1, p + 1, p + 1)) for lv in levels]
    b[-1] = b_box[box_id]
    us, h = lr.solve(levels, b, opts, max_cycles=6, rtol=1e-14)
    assert np.allclose(h, h_ref, rtol=1e-9, atol=1e-15), (h, h_ref)
    assert np.abs(us[-1] - u_ref[box_id]).max() < 1e-10 * np.abs(u_ref).max()


def test_converged_state_is_the_composite_solution():
    """Base 3^3, p = 2, the centre element refined: 26 leaves on level 1, 8 leaves and 208
    frozen elements on level 2."""
    p, ne = 2, 3
    X, nbr, bc = base_mesh(p, ne, lambda Y: W.sine_bump_map(Y, 0.03))
    levels = lr.build_local_levels(p, (ne,) * 3, X, nbr, bc, [near((0.5, 0.5, 0.5), 0.2)], kappa=0.3)
    assert [int((lv.cls == k).sum()) for lv in levels for k in (lr.TWIG, lr.LEAF, lr.FROZEN)] == \
        [1, 26, 0, 0, 8, 208]
    b = level_b(levels, lambda Y: np.sin(3 * Y[:, 0]) * np.cos(2 * Y[:, 1]) + Y[:, 2])
    opts = sv.Options('scg', 3, 2)
    us, h = lr.solve(levels, b, opts, max_cycles=40, rtol=1e-13)
    assert h[-1] <= 1e-13, h
    ref = lr.composite_dense(levels, b)
    for u, r in zip(us, ref):
        assert np.abs(u - r).max() < 1e-9 * np.abs(ref[-1]).max()


def test_two_nested_zones_converge():
    p, ne = 3, 4
    X, nbr, bc = base_mesh(p, ne, lambda Y: W.sine_bump_map(Y, 0.05))
    c = (0.5, 0.5, 0.5)
    levels = lr.build_local_levels(p, (ne,) * 3, X, nbr, bc, [near(c, 0.3), near(c, 0.2)], p_coarsen=True)
    counts = [[int((lv.cls == k).sum()) for k in (lr.TWIG, lr.LEAF, lr.FROZEN)] for lv in levels]
    assert counts[-1][0] == 0 and counts[-1][1] > 0 and counts[-2][0] > 0, counts
    b = level_b(levels, lambda Y: np.exp(-20 * np.sum((Y - 0.5) ** 2, axis=1)))
    us, h = lr.solve(levels, b, sv.Options('was', 2, 2), max_cycles=8, rtol=1e-12)
    rates = np.array(h[1:]) / np.array(h[:-1])
    # measured 0.18, 0.31, 0.23, 0.27, 0.25, 0.26, 0.25
    assert rates.max() < 0.35 and h[-1] < 1e-4, h


def test_refine_list_generator_numbers_levels_like_the_builder():
    """workloads.local_refine_lists (the benchmark's input) marks and numbers the cells of each
    step as the oracle's builder does on a Cartesian box."""
    ne, p = 4, 2
    zones = [((0.5, 0.5, 0.5), 0.3), ((0.5, 0.5, 0.5), 0.2)]
    X, nbr, bc = base_mesh(p, ne)
    data = lr.build_local_mesh(p, (ne,) * 3, X, nbr, bc, [near(c, r) for c, r in zones])
    lists = W.local_refine_lists(ne, zones)
    assert [list(x) for x in lists] == [list(np.nonzero(d['cls'] == lr.TWIG)[0]) for d in data[:-1]]


def test_fmg_start_cuts_the_first_cycle():
    """FAS-FMG (Alg. 4) on the two-zone mesh with a smooth source: the start-up leaves a first
    cycle residual far below the plain first cycle's, and the cycles still converge."""
    p, ne = 3, 4
    X, nbr, bc = base_mesh(p, ne, lambda Y: W.sine_bump_map(Y, 0.05))
    c = (0.5, 0.5, 0.5)
    levels = lr.build_local_levels(p, (ne,) * 3, X, nbr, bc, [near(c, 0.3), near(c, 0.2)], p_coarsen=True)
    b = level_b(levels, lambda Y: np.exp(-20 * np.sum((Y - 0.5) ** 2, axis=1)))
    _, h0 = lr.solve(levels, b, sv.Options('was', 2, 2), max_cycles=3, rtol=1e-12)
    _, h1 = lr.solve(levels, b, sv.Options('was', 2, 2, start='fmg'), max_cycles=3, rtol=1e-12)
    # measured first cycles 0.18 plain, 0.0026 with FMG
    assert h1[1] < 0.05 * h0[1] and h1[-1] < h1[1], (h0, h1)
