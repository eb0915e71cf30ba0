"""A spatially varying diffusivity nu(x) (eq. helmholtz:pde) through the library against the
oracle: the operator, right-hand side and Schwarz surrogate (element-averaged nu, Sec. 4.3.1)
on every level of the p- and h-hierarchies (coarse levels evaluate the nodal field at their
own nodes), V-cycle histories, and the patch test across a jump of nu."""
import numpy as np
import pytest

from oracle import hmg, operator as oop, solvers as osv
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


class NuCase:
    """field: 'blade' (1 + cos cos cos, zero at isolated points), 'mild' (1 + cos cos cos / 2) or
    'jump' (a seeded constant per element, 0.5 to 4)."""

    def __init__(self, name, p, ne, field, amp=0.03, kappa=1.0, h_levels=0):
        self.name, self.p, self.ne, self.field, self.kappa, self.hl = name, p, ne, field, kappa, h_levels
        self.nbr, self.bc = W.box_topology(ne, ne, ne)
        self.V = W.box_vertices(ne, ne, ne)
        self.map = (lambda X: W.sine_bump_map(X, amp)) if amp else None

    def coords(self, xi):
        return W.element_coords(self.V, xi, self.map)

    def nu(self, X):
        if self.field == 'blade':
            return W.cosine_diffusivity(X)
        if self.field == 'mild':
            return 1.0 + 0.5 * (W.cosine_diffusivity(X) - 1.0)
        per = np.random.default_rng(9).uniform(0.5, 4.0, X.shape[0])
        return np.broadcast_to(per[:, None, None, None], X[:, 0].shape).copy()

    def oracle_levels(self):
        X = self.coords(ogll(self.p)[0])
        if self.hl:
            return hmg.build_hlevels(self.p, X, self.nbr, self.bc, (self.ne,) * 3, self.hl, nu=self.nu(X),
                                     kappa=self.kappa, p_coarsen=True)
        return osv.build_levels(self.p, X, self.nbr, self.bc, nu=self.nu(X), kappa=self.kappa)

    def library(self, B, **opt):
        X = self.coords(B.gll(self.p)[0])
        o = B.default_options(kappa=self.kappa, h_levels=self.hl, **opt)
        return B.Solver(np.full(self.ne ** 3, self.p, np.int32), X, self.nbr, self.bc, o,
                        box=(self.ne,) * 3 if self.hl else None, nu=self.nu(X))

    def __repr__(self):
        return self.name


# the element-averaged surrogate cannot follow a coefficient that jumps by up to 8 between
# neighbours: FAS-MG-WAS diverges there (in the oracle as well), so the jump case skips histories
CASES = [NuCase('blade_curved_p4_3^3', 4, 3, 'blade'), NuCase('mild_curved_p7_2^3', 7, 2, 'mild'),
         NuCase('blade_curved_p7_2^3', 7, 2, 'blade'), NuCase('jump_p3_4^3', 3, 4, 'jump', amp=0.0, kappa=0.0),
         NuCase('mild_h1_p3_4^3', 3, 4, 'mild', h_levels=1)]


@pytest.fixture(scope='module', params=CASES, ids=repr)
def pair(request, binding):
    case = request.param
    print('nu case', case.name, flush=True)
    lib = case.library(binding)
    lv = case.oracle_levels()
    yield case, lib, lv
    lib.close()


def test_operator_rhs_and_schwarz_every_level(pair):
    case, lib, lv = pair
    rng = np.random.default_rng(30)
    assert lib.n_levels == len(lv)
    for l in range(1, lib.n_levels + 1):
        o = lv[l - 1]
        u = rng.uniform(-1, 1, o.mesh.n_dof())
        out = torch.empty(o.mesh.n_dof(), dtype=torch.float64, device='cuda')
        lib.apply(l, dev(u), out)
        assert rel(host(out), o.A(u)) < 1e-12, (case.name, l)
        lib.schwarz(l, dev(u), out)
        assert rel(host(out), o.B(u)) < 1e-11, (case.name, l)
    top = lv[-1].mesh
    f, uD = rng.uniform(-1, 1, top.n_dof()), rng.uniform(-1, 1, top.n_dof())
    b = torch.empty(top.n_dof(), dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b, uD=dev(uD))
    assert rel(host(b), oop.rhs(top, f, uD=uD)) < 1e-12


def test_history_matches_oracle(pair):
    """FAS-MG-WAS(2,2) cycles from u = 0 on a seeded right-hand side: the library's residual
    history and solution follow the oracle's."""
    case, lib, lv = pair
    if case.field == 'jump' or (case.field == 'blade' and case.p == 7):
        pytest.skip('FAS-MG-WAS diverges on this coefficient (oracle too); operator parity covers it')
    top = lv[-1].mesh
    b = np.random.default_rng(31).uniform(-1, 1, (top.E, top.n, top.n, top.n))
    uo, ho = osv.solve(lv, np.zeros_like(b), b, osv.Options('was', 2, 2), max_cycles=5, rtol=1e-14)
    u = torch.zeros(top.n_dof(), dtype=torch.float64, device='cuda')
    hg, _ = lib.solve(u, dev(b), max_cycles=5, rtol=1e-14)
    hg = list(hg)
    assert len(hg) == len(ho)
    for a, c in zip(hg, ho):
        assert abs(a - c) <= 1e-6 * max(c, 1e-12), (case.name, hg, ho)
    assert rel(host(u), uo) < 1e-9


def test_patch_test_across_a_jump(binding):
    """nu1 = 1 for x < 1/2, nu2 = 6 beyond, u piecewise linear in x with a continuous flux: u lies
    in the discrete space and the library's residual b(f = 0, u_D = u) - A u vanishes."""
    p, ne = 3, 4
    V = W.box_vertices(ne, ne, ne)
    X = W.element_coords(V, binding.gll(p)[0])
    nbr, bc = W.box_topology(ne, ne, ne)
    ex = np.tile(np.arange(ne), ne * ne)
    left = (ex < ne // 2)[:, None, None, None]
    nu = np.where(left, 1.0, 6.0) * np.ones_like(X[:, 0])
    a1 = 1.7
    a2 = a1 / 6.0
    u = np.where(left, a1 * X[:, 0], a1 * 0.5 + a2 * (X[:, 0] - 0.5))
    lib = binding.Solver(np.full(ne ** 3, p, np.int32), X, nbr, bc, binding.default_options(), nu=nu)
    b = torch.empty(u.size, dtype=torch.float64, device='cuda')
    lib.rhs(dev(np.zeros_like(u)), b, uD=dev(u))
    r = torch.empty_like(b)
    lib.residual(lib.n_levels, dev(u), b, r)
    Au = torch.empty_like(b)
    lib.apply(lib.n_levels, dev(u), Au)
    assert np.abs(host(r)).max() < 1e-11 * np.abs(host(Au)).max()
    lib.close()
