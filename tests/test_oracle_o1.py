"""O1 (the C/OpenMP oracle) against the numpy oracle, element-wise, on small meshes: operator,
right-hand side, Schwarz application and transfers on every level, WAS and SCG smoothing, and
FAS V-cycle histories.  The numpy oracle is pinned by its own tests; O1 inherits those pins
here, which lets it stand for the oracle at the full sizes the numpy version cannot reach."""
import numpy as np
import pytest

from oracle import o1, operator as op, solvers as sv
from oracle.gll import gll
from paper_2608_14123_amd import workloads as W

CASES = [
    # name, p, ne, map amplitude, boundary code, kappa, mu_star, periodic
    ('cart_p4_3^3', 4, 3, 0.0, 1, 0.0, 2.0, False),
    ('curved_p7_2^3', 7, 2, 0.03, 1, 0.0, 5.0, False),
    ('curved_p3_3^3', 3, 3, 0.03, 1, 0.0, 2.0, False),
    ('neumann_kappa_p5_2^3', 5, 2, 0.03, 2, 0.7, 2.0, False),
    ('stretched_p8_2^3', 8, 2, 0.0, 1, 0.0, 5.0, False),
    ('periodic_kappa_p2_3^3', 2, 3, 0.0, 1, 1.0, 2.0, True),
]


def build(case):
    name, p, ne, amp, bcc, kappa, mu, per = case
    nbr, bc = W.box_topology(ne, ne, ne, periodic=(per,) * 3, bc_code=bcc)
    if name.startswith('stretched'):
        V, nbr, bc = W.stretched_perturbed(ne)
    else:
        V = W.box_vertices(ne, ne, ne)
    X = W.element_coords(V, gll(p)[0], (lambda Y: W.sine_bump_map(Y, amp)) if amp else None)
    levels = sv.build_levels(p, X, nbr, bc, m=1, kappa=kappa, mu_star=mu)
    fast = o1.O1(p, X, nbr, bc, m=1, kappa=kappa, mu_star=mu)
    return levels, fast, X


def rel(a, b):
    return np.abs(np.ravel(a) - np.ravel(b)).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize('case', CASES, ids=[c[0] for c in CASES])
def test_o1_matches_numpy_oracle_on_every_level(case):
    levels, fast, X = build(case)
    rng = np.random.default_rng(7)
    assert fast.n_levels == len(levels)
    for l in range(1, fast.n_levels + 1):
        lv = levels[l - 1]
        n = lv.mesh.n_dof()
        u, g = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        Au = lv.A(u).ravel()
        assert rel(fast.apply(l, u), Au) <= 1e-13, ('apply', l)
        assert rel(fast.residual(l, u, g), g - Au) <= 1e-13, ('residual', l)
        assert rel(fast.schwarz(l, g), lv.B(g)) <= 1e-12, ('schwarz', l)
        shp = (lv.mesh.E,) + (lv.p + 1,) * 3
        assert rel(fast.smooth(l, u, g, 2, 'was'), sv.was(lv, u.reshape(shp), g.reshape(shp), 2)) <= 1e-12
        assert rel(fast.smooth(l, u, g, 3, 'scg'), sv.scg(lv, u.reshape(shp), g.reshape(shp), 3)) <= 1e-11
        if l > 1:
            from oracle import transfer as tr
            pc, pf = levels[l - 2].p, lv.p
            shp = (lv.mesh.E,) + (pf + 1,) * 3
            assert rel(fast.project(l, u), tr.project(pc, pf, u.reshape(shp))) <= 1e-13
            assert rel(fast.restrict(l, g), tr.restrict(pc, pf, g.reshape(shp))) <= 1e-13
            uc = rng.uniform(-1, 1, levels[l - 2].mesh.n_dof())
            ref = u + tr.prolong(pc, pf, uc.reshape((lv.mesh.E,) + (pc + 1,) * 3)).ravel()
            assert rel(fast.prolong_add(l, uc, u), ref) <= 1e-13
    top = levels[-1].mesh
    f, uD = rng.uniform(-1, 1, top.n_dof()), rng.uniform(-1, 1, top.n_dof())
    assert rel(fast.rhs(f, uD), op.rhs(top, f.reshape(X[:, 0].shape), uD=uD.reshape(X[:, 0].shape))) <= 1e-13
    fast.close()


@pytest.mark.parametrize('smoother,ns', [('was', (2, 2)), ('scg', (3, 2))])
def test_o1_history_matches_numpy_oracle(smoother, ns):
    """Curved p = 4 on 3^3: the V-cycle histories (root SCG to 1e-12) agree per cycle to 1e-9,
    and the final iterates to 1e-10."""
    case = ('curved_p4_3^3', 4, 3, 0.03, 1, 0.0, 2.0, False)
    levels, fast, X = build(case)
    b = op.rhs(levels[-1].mesh, W.uniform_nodal(X[:, 0].shape, 2))
    u_ref, h_ref = sv.solve(levels, np.zeros_like(b), b, sv.Options(smoother, *ns), max_cycles=20, rtol=1e-10)
    u, h, its = fast.solve(b.ravel(), smoother=smoother, ns1=ns[0], ns2=ns[1], max_cycles=20, rtol=1e-10)
    assert len(h) == len(h_ref)
    for a, c in zip(h, h_ref):
        assert abs(a - c) <= 1e-9 * c + 1e-15
    assert rel(u, u_ref) <= 1e-10
    fast.close()
