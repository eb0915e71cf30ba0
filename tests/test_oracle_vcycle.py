"""Pins of the oracle's smoothers and cycles (Alg. 1, 2, 5, 6)."""
import csv
import os

import numpy as np
import pytest

from oracle import operator as op, solvers as sv, dense as dn
from oracle.cost import equivalent_vcycles, levels_p_mg
from oracle.gll import gll
from oracle.mesh import Mesh
from paper_2608_14123_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden')


def setup(p, ne, amp=0.0, seed=2):
    nbr, bc = W.box_topology(ne, ne, ne)
    x, _ = gll(p)
    X = W.element_coords(W.box_vertices(ne, ne, ne), x, (lambda Y: W.sine_bump_map(Y, amp)) if amp else None)
    levels = sv.build_levels(p, X, nbr, bc, m=1)
    f = W.uniform_nodal(X[:, 0].shape, seed)
    return levels, X, op.rhs(levels[-1].mesh, f)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_fas_matches_dense_brute_force(p):
    """Matrix-free FAS V-cycle == explicit-matrix V-cycle (B from dense surrogate inverses)."""
    levels, X, b = setup(p, 2, amp=0.03)
    H = dn.DenseHierarchy(levels)
    opts = sv.Options('was', 2, 2, root='direct')
    u = np.zeros_like(b)
    ud = u.ravel().copy()
    for _ in range(3):
        u = sv.fas_vcycle(levels, u, b, opts)
        ud = dn.fas_vcycle_dense(H, ud, b.ravel(), 2, 2)
        assert np.abs(u.ravel() - ud).max() <= 1e-12 * np.abs(ud).max()


def test_fas_equals_cs_for_linear_problem():
    """FAS and CS give the same iterates in exact arithmetic; in FP64 FAS loses digits to the
    cancellation in g - A u_bar, so the agreement is absolute in the relative residual."""
    levels, X, b = setup(4, 3)
    opts = sv.Options('was', 2, 2)
    _, h1 = sv.solve(levels, np.zeros_like(b), b, opts)
    _, h2 = sv.solve(levels, np.zeros_like(b), b, opts, cycle=sv.cs_vcycle)
    assert len(h1) == len(h2)
    for a, c in zip(h1, h2):
        assert abs(a - c) <= 1e-14 + 1e-9 * c


def test_converges_to_direct_solution_and_converged_state():
    levels, X, b = setup(3, 2, amp=0.03)
    A = op.assemble(levels[-1].mesh)
    uex = np.linalg.solve(A, b.ravel())
    u, hist = sv.solve(levels, np.zeros_like(b), b, sv.Options('was', 2, 2), rtol=1e-13, max_cycles=40)
    assert hist[-1] <= 1e-13
    assert np.abs(u.ravel() - uex).max() <= 1e-10 * np.abs(uex).max()
    # at convergence the coarse FAS equation is satisfied by u_bar = P u (eq. fas:converged)
    from oracle import transfer as tr
    lc, lv = levels[-2], levels[-1]
    ub = tr.project(lc.p, lv.p, u)
    g = lc.A(ub) + tr.restrict(lc.p, lv.p, b - lv.A(u))
    v = sv.scg(lc, ub.copy(), g, 200, 1e-14 * sv.norm(g))
    assert np.abs(v - ub).max() <= 1e-8 * np.abs(ub).max()


def test_scg_equals_textbook_pcg_with_symmetric_preconditioner():
    """With a fixed SPD preconditioner z^T r0 = 0, so the flexible beta equals Fletcher-Reeves."""
    levels, X, b = setup(3, 2, amp=0.03)
    lv = levels[-1]
    Dinv = 1.0 / np.diag(op.assemble(lv.mesh)).reshape(b.shape)
    prec = lambda r: Dinv * r
    u1 = sv.scg(lv, np.zeros_like(b), b, 25, 0.0, precond=prec)
    # textbook PCG
    x = np.zeros_like(b)
    r = b.copy()
    z = prec(r)
    p = z.copy()
    rz = np.sum(r * z)
    for _ in range(25):
        q = lv.A(p)
        a = rz / np.sum(p * q)
        x += a * p
        r -= a * q
        z = prec(r)
        rz_new = np.sum(r * z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    assert np.abs(u1 - x).max() <= 1e-10 * np.abs(x).max()


def test_scg_exit_rule():
    levels, X, b = setup(2, 2)
    st = {}
    sv.scg(levels[-1], np.zeros_like(b), b, 500, 1e-6 * sv.norm(b), stats=st)
    assert 1 < st['iters'] < 500


def test_cartesian_unit_cube_p4_history():
    """4^3 cubes, p = 4, sin sin sin: FAS-MG-WAS(2,2) reaches 1e-10, error at the DG level."""
    nbr, bc = W.box_topology(4, 4, 4)
    x, _ = gll(4)
    X = W.element_coords(W.box_vertices(4, 4, 4), x)
    levels = sv.build_levels(4, X, nbr, bc, m=1)
    ue = W.sine_solution(X)
    b = op.rhs(levels[-1].mesh, 3 * np.pi ** 2 * ue)
    u, hist = sv.solve(levels, np.zeros_like(b), b, sv.Options('was', 2, 2))
    assert hist[-1] <= 1e-10 and len(hist) - 1 <= 10
    assert all(hist[i + 1] < 0.1 * hist[i] for i in range(len(hist) - 1))
    assert op.l2_error(levels[-1].mesh, u, ue) < 1e-5


def test_cost_model_reproduces_printed_v10():
    """eq. cost:equivalent against the printed v10 column (Table cart-uni, Sec. 6.2.1)."""
    rows = [r for r in csv.reader(open(os.path.join(GOLDEN, 'cost_model_rows.csv'))) if r and not r[0].startswith('#')]
    checked = 0
    for meth, mg, p, s1, s2, sc, n10, v10 in rows:
        p, s1, s2, sc, n10, v10 = int(p), int(s1), int(s2), int(sc), int(n10), float(v10)
        sm = 'SCG' if meth.endswith('SCG') else 'WAS'
        if sm == 'SCG' and n10 == 1:
            continue
        a = 1 / 16 if mg == 'p' else 1 / 8
        L = levels_p_mg(p) if mg == 'p' else 4
        v = equivalent_vcycles(sm, meth.startswith('CS-CG'), s1, s2, sc, n10, a, L)
        assert abs(v - v10) <= 0.05 + 1e-9, (meth, p, v, v10)
        checked += 1
    assert checked >= 70


@pytest.mark.parametrize("p", [2, 4])
def test_fmg_cmg_and_crossover_match_dense_brute_force(p):
    """Alg. 4 (FMG) and Alg. 3 (CMG) start-ups and cycles with crossover smoothing, matrix-free
    against explicit matrices (dense surrogate inverses, Kronecker transfers, exact root solves)."""
    levels, X, b = setup(p, 2, amp=0.03)
    H = dn.DenseHierarchy(levels)
    f = b.ravel()
    opts = sv.Options('was', 2, 1, root='direct', ns0=3, nsc=2)
    u_f = sv.fmg_start(levels, np.zeros_like(b), b, opts).ravel()
    ud_f = dn.fmg_dense(H, f, 2, 1)
    assert np.abs(u_f - ud_f).max() <= 1e-12 * np.abs(ud_f).max()
    u_c = sv.cmg_start(levels, np.zeros_like(b), b, opts).ravel()
    ud_c = dn.cmg_dense(H, f, 3)
    assert np.abs(u_c - ud_c).max() <= 1e-12 * np.abs(ud_c).max()
    # three cycles with crossover after the FMG start: solve() against the dense sequence
    opts.start = 'fmg'
    u, hist = sv.solve(levels, np.zeros_like(b), b, opts, max_cycles=3, rtol=0.0)
    ud = dn.crossover_cycles_dense(H, ud_f, f, 2, 1, 2, 3)
    assert len(hist) == 4
    assert np.abs(u.ravel() - ud).max() <= 1e-12 * np.abs(ud).max()


def test_fmg_start_reaches_the_discretisation_error_in_one_cycle():
    """FMG's purpose (Sec. 3.3) on C1 (4^3, p = 4, the smooth manufactured solution, WAS(2,2)):
    after the start-up and one V-cycle the residual is two orders below that of the plain
    first cycle, CMG lies between the two, and 1e-10 takes fewer cycles with either start-up
    (the paper's cart-uni table: FAS-FMG needs no more cycles than FAS-CMG)."""
    ne, p = 4, 4
    nbr, bc = W.box_topology(ne, ne, ne)
    X = W.element_coords(W.box_vertices(ne, ne, ne), gll(p)[0])
    levels = sv.build_levels(p, X, nbr, bc, m=1)
    b = op.rhs(levels[-1].mesh, 3 * np.pi ** 2 * W.sine_solution(X))
    n10, first = {}, {}
    for start in (None, 'fmg', 'cmg'):
        _, h = sv.solve(levels, np.zeros_like(b), b, sv.Options('was', 2, 2, start=start), max_cycles=30)
        n10[start], first[start] = len(h) - 1, h[1]
    assert first['fmg'] < 0.02 * first[None]
    assert first['fmg'] < first['cmg'] < first[None]
    assert n10['fmg'] <= n10['cmg'] <= n10[None] and n10['fmg'] < n10[None]
