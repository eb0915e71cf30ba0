"""Semidefinite problems (kappa = 0 and no Dirichlet face: periodic or pure Neumann), where A has
the constants as its null space.  The remark on IPCG for semidefinite systems (Sec. 4.3.2) makes
the root SCG converge by projecting onto the range of A; the V-cycle then solves A u = f for a
zero-mean f.  Pins: A 1 = 0 and symmetry fix the null space and the range; the converged
solution equals the minimum-norm dense solution (pseudo-inverse) up to a constant."""
import numpy as np
import pytest

from oracle import operator as op, solvers as sv
from oracle.gll import gll
from paper_2608_14123_amd import workloads as W


def levels_and_rhs(p, ne, periodic, curved):
    bc_code = 1 if periodic else 2
    nbr, bc = W.box_topology(ne, ne, ne, periodic=(periodic,) * 3, bc_code=bc_code)
    if periodic:
        fn = (lambda X: X + 0.01 * np.sin(2 * np.pi * X)) if curved else None
    else:
        fn = (lambda X: W.sine_bump_map(X, 0.03)) if curved else None
    X = W.element_coords(W.box_vertices(ne, ne, ne), gll(p)[0], fn)
    levels = sv.build_levels(p, X, nbr, bc, kappa=0.0)
    n = p + 1
    b = np.random.default_rng(5).uniform(-1, 1, (ne ** 3, n, n, n))
    return levels, b - b.mean()


@pytest.mark.parametrize('periodic,curved', [(True, False), (True, True), (False, True)])
def test_cycle_reaches_the_pseudo_inverse_solution(periodic, curved):
    p, ne = 3, 2
    levels, b = levels_and_rhs(p, ne, periodic, curved)
    A = op.assemble(levels[-1].mesh)
    one = np.ones(A.shape[0])
    assert np.abs(A @ one).max() < 1e-11 * np.abs(A).max()
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    for sm, ns in (('was', (2, 2)), ('scg', (3, 2))):
        u, h = sv.solve(levels, np.zeros_like(b), b, sv.Options(sm, *ns, null_space=True), max_cycles=30,
                        rtol=1e-11)
        assert h[-1] <= 1e-11, (sm, h)
        ref = np.linalg.pinv(A) @ b.ravel()
        d = u.ravel() - u.mean()
        assert np.abs(d - (ref - ref.mean())).max() < 1e-8 * np.abs(ref).max(), sm
