"""Local refinement (Sec. 3.1 multilevel mesh with twig, leaf and frozen elements; eq.
helmholtz:fas; Alg. 2 with the frozen update) through the library against the oracle: the
level structure and coordinates, the operator and the Schwarz smoother of the active elements
on every level, the per-level right-hand sides, V-cycle histories of the composite residual
and every level's solution.  The refinement marks are inputs; they are taken from the
oracle's builder (which applies the nesting rule to a distance criterion)."""
import numpy as np
import pytest

from oracle import localref as lr, operator as op, solvers as osv
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


def near(c, rad):
    return lambda centres: np.linalg.norm(centres - np.asarray(c), axis=1) < rad


def source(X):
    return np.sin(3 * X[:, 0]) * np.cos(2 * X[:, 1]) + X[:, 2]


class LCase:
    def __init__(self, name, p, ne, zones, amp=0.03, kappa=0.3):
        self.name, self.p, self.ne, self.zones, self.kappa = name, p, ne, zones, kappa
        self.nbr, self.bc = W.box_topology(ne, ne, ne)
        self.V = W.box_vertices(ne, ne, ne)
        self.map = lambda Y: W.sine_bump_map(Y, amp)

    def coords(self, xi):
        return W.element_coords(self.V, xi, self.map)

    def oracle(self):
        X = self.coords(ogll(self.p)[0])
        marks = [near(c, r) for c, r in self.zones]
        levels = lr.build_local_levels(self.p, (self.ne,) * 3, X, self.nbr, self.bc, marks, kappa=self.kappa,
                                       p_coarsen=True)
        data = lr.build_local_mesh(self.p, (self.ne,) * 3, X, self.nbr, self.bc, marks)
        refine = [np.nonzero(d['cls'] == lr.TWIG)[0] for d in data[:-1]]
        return levels, refine

    def library(self, B, refine, **opt):
        o = B.default_options(kappa=self.kappa, local_steps=len(refine), **opt)
        return B.Solver(np.full(self.ne ** 3, self.p, np.int32), self.coords(B.gll(self.p)[0]), self.nbr, self.bc, o,
                        refine=refine)

    def __repr__(self):
        return self.name


CASES = [LCase('centre_p2_3^3', 2, 3, [((0.5, 0.5, 0.5), 0.2)]),
         LCase('two_zones_p3_4^3', 3, 4, [((0.5, 0.5, 0.5), 0.3), ((0.5, 0.5, 0.5), 0.2)])]


@pytest.fixture(scope='module', params=CASES, ids=repr)
def pair(request, binding):
    case = request.param
    print('local refinement case', case.name, flush=True)
    levels, refine = case.oracle()
    lib = case.library(binding, refine)
    yield case, lib, levels, refine
    lib.close()


def test_levels_classes_and_coordinates(pair):
    case, lib, levels, _ = pair
    assert lib.n_levels == len(levels)
    for l, o in enumerate(levels, start=1):
        assert np.array_equal(lib.level_classes(l), o.cls), (case.name, l)
        assert rel(lib.level_coords(l), o.mesh.X) < 1e-13


def test_operator_and_schwarz_every_level(pair):
    case, lib, levels, _ = pair
    rng = np.random.default_rng(40)
    for l, o in enumerate(levels, start=1):
        u = rng.uniform(-1, 1, o.mesh.n_dof())
        out = torch.zeros(o.mesh.n_dof(), dtype=torch.float64, device='cuda')
        lib.apply(l, dev(u), out)
        assert rel(host(out), o.A(u)) < 1e-12, (case.name, l)
        out.zero_()
        lib.schwarz(l, dev(u * np.repeat(o.active, o.mesh.n ** 3)), out)
        ref = o.B(u * np.repeat(o.active, o.mesh.n ** 3))
        assert rel(host(out), ref) < 1e-11, (case.name, l)


@pytest.mark.parametrize('smoother,start', [('was', None), ('scg', None), ('was', 'fmg')])
def test_histories_and_solutions_match_oracle(pair, binding, smoother, start):
    case, lib0, levels, refine = pair
    ns = (2, 2) if smoother == 'was' else (3, 2)
    b = [op.rhs(lv.mesh, source(lv.mesh.X), uD=np.zeros((lv.mesh.E,) + (lv.mesh.n,) * 3)) for lv in levels]
    us, ho = lr.solve(levels, b, osv.Options(smoother, *ns, start=start), max_cycles=8, rtol=1e-13)
    lib = case.library(binding, refine, smoother=binding.SCG if smoother == 'scg' else binding.WAS, ns1=ns[0],
                       ns2=ns[1], start=binding.START_FMG if start == 'fmg' else binding.START_NONE)
    L = lib.n_levels
    bl = []
    for l in range(1, L + 1):
        Xl = lib.level_coords(l)
        t = torch.empty(Xl.size // 3, dtype=torch.float64, device='cuda')
        lib.level_rhs(l, dev(source(Xl)), t, uD=torch.zeros_like(t))
        assert rel(host(t), b[l - 1]) < 1e-12
        bl.append(t)
        if l < L:
            lib.set_level_rhs(l, t)
    u = torch.zeros_like(bl[-1])
    hist, _ = lib.solve(u, bl[-1], max_cycles=len(ho) - 1, rtol=1e-13)
    hist = list(hist)
    assert len(hist) == len(ho), (hist, ho)
    for a, c in zip(hist, ho):
        assert abs(a - c) <= 1e-6 * c + 1e-15, (case.name, hist, ho)
    assert rel(host(u), us[-1]) < 1e-9
    for l in range(1, L):
        t = torch.empty_like(bl[l - 1])
        lib.level_solution(l, t)
        assert rel(host(t), us[l - 1]) < 1e-9, (case.name, l)
    lib.close()
