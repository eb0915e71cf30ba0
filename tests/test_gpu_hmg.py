"""h-coarsening (Sec. 3.1 multilevel mesh by h-refinement, Sec. 3.2 transfers) against the
oracle: the operator and Schwarz application on every h-level, the parent/children transfers,
and FAS V-cycle / FMG histories with pure h-MG and with h- followed by p-coarsening."""
import numpy as np
import pytest

from oracle import hmg, operator as oop, solvers as osv, transfer as otr
from oracle.gll import gll as ogll
from paper_2608_14123_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


@pytest.fixture(scope='module')
def binding():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2608_14123_amd import binding as b
    return b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(np.ravel(a) - np.ravel(b)).max() / max(np.abs(b).max(), 1e-300)


class HCase:
    def __init__(self, name, p, ne, h_levels, h_only, amp=0.03, periodic=False, kappa=0.0):
        self.name, self.p, self.ne, self.hl, self.h_only = name, p, ne, h_levels, h_only
        self.kappa = kappa
        self.nbr, self.bc = W.box_topology(ne, ne, ne, periodic=(periodic,) * 3)
        self.V = W.box_vertices(ne, ne, ne)
        self.map = (lambda X: W.sine_bump_map(X, amp)) if amp else None

    def coords(self, xi):
        return W.element_coords(self.V, xi, self.map)

    def oracle_levels(self):
        return hmg.build_hlevels(self.p, self.coords(ogll(self.p)[0]), self.nbr, self.bc, (self.ne,) * 3, self.hl,
                                 kappa=self.kappa, p_coarsen=not self.h_only)

    def library(self, B, **opt):
        o = B.default_options(h_levels=self.hl, h_only=int(self.h_only), kappa=self.kappa, **opt)
        return B.Solver(np.full(self.ne ** 3, self.p, np.int32), self.coords(B.gll(self.p)[0]), self.nbr, self.bc, o,
                        box=(self.ne,) * 3)

    def __repr__(self):
        return self.name


CASES = [HCase('h2_only_p4_4^3', 4, 4, 2, True), HCase('h1_then_p_p4_4^3', 4, 4, 1, False),
         HCase('h1_only_p3_4^3', 3, 4, 1, True),
         HCase('h1_only_periodic_kappa_p2_4^3', 2, 4, 1, True, amp=0.0, periodic=True, kappa=1.0)]


@pytest.mark.parametrize('case', CASES, ids=repr)
def test_h_levels_operator_schwarz_and_transfers(binding, case):
    print('h-levels', case, flush=True)
    lv = case.oracle_levels()
    lib = case.library(binding)
    assert lib.n_levels == len(lv)
    rng = np.random.default_rng(3)
    for l in range(1, lib.n_levels + 1):
        o = lv[l - 1]
        n = o.mesh.n_dof()
        assert lib.level_info(l) == (o.p, n)
        u, g = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        out = torch.empty(n, dtype=torch.float64, device='cuda')
        lib.apply(l, dev(u), out)
        assert rel(host(out), o.A(u)) <= 1e-12, ('apply', l)
        lib.schwarz(l, dev(g), out)
        assert rel(host(out), o.B(g)) <= 1e-11, ('schwarz', l)
        if l > 1:
            c = lv[l - 2]
            nc = c.mesh.n_dof()
            oc = torch.empty(nc, dtype=torch.float64, device='cuda')
            lib.project(l, dev(u), oc)
            assert rel(host(oc), osv.t_project(c, o, u.reshape((o.mesh.E,) + (o.p + 1,) * 3))) <= 1e-13
            lib.restrict(l, dev(g), oc)
            assert rel(host(oc), osv.t_restrict(c, o, g.reshape((o.mesh.E,) + (o.p + 1,) * 3))) <= 1e-13
            uc = rng.uniform(-1, 1, nc)
            uf = dev(u)
            lib.prolong_add(l, dev(uc), uf)
            ref = u + osv.t_prolong(c, o, uc.reshape((c.mesh.E,) + (c.p + 1,) * 3)).ravel()
            assert rel(host(uf), ref) <= 1e-13
    lib.close()


@pytest.mark.parametrize('case,smoother,ns,start', [(CASES[0], 'was', (1, 1), None), (CASES[0], 'was', (1, 1), 'fmg'),
                                                    (CASES[1], 'scg', (3, 2), None), (CASES[2], 'was', (2, 2), 'fmg')],
                         ids=['h2_was11', 'h2_fmg_was11', 'h1p_scg32', 'h1_p3_fmg_was22'])
def test_h_multigrid_histories(binding, case, smoother, ns, start):
    print('h-MG history', case, smoother, ns, start, flush=True)
    lv = case.oracle_levels()
    top = lv[-1].mesh
    fo = 3 * np.pi ** 2 * W.sine_solution(case.coords(ogll(case.p)[0]))
    bo = oop.rhs(top, fo)
    uo, ho = osv.solve(lv, np.zeros_like(bo), bo, osv.Options(smoother, *ns, start=start), max_cycles=30)
    lib = case.library(binding, smoother=binding.SCG if smoother == 'scg' else binding.WAS, ns1=ns[0], ns2=ns[1],
                       start=binding.START_FMG if start == 'fmg' else binding.START_NONE)
    fg = dev(3 * np.pi ** 2 * W.sine_solution(case.coords(binding.gll(case.p)[0])))
    b = torch.empty_like(fg)
    lib.rhs(fg, b)
    u = torch.zeros_like(b)
    hg, ok = lib.solve(u, b, max_cycles=30, rtol=1e-10)
    assert ok
    assert len(hg) == len(ho), (list(hg), ho)
    for a, c in zip(hg, ho):
        assert abs(a - c) <= 1e-6 * c + 1e-14, (a, c)
    assert rel(host(u), uo) <= 1e-9
    lib.close()
