"""FAS-CMG and FAS-FMG start-ups (Alg. 3, Alg. 4), crossover smoothing, plain additive
weighting and overlap derived from delta, against the oracle."""
import numpy as np
import pytest

from oracle import operator as oop, solvers as osv
from oracle.gll import gll as ogll
from paper_2608_14123_amd import workloads as W
from gpu_cases import Case

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


def histories_agree(hg, ho):
    assert len(hg) == len(ho), (hg, ho)
    for a, b in zip(hg, ho):
        assert abs(a - b) <= 1e-6 * b + 1e-14, (a, b)


def _problem(case, binding, smooth_rhs):
    lv = case.oracle_levels()
    top = lv[-1].mesh
    if smooth_rhs:
        fo = 3 * np.pi ** 2 * W.sine_solution(case.coords(ogll(case.p)[0]))
        fg = 3 * np.pi ** 2 * W.sine_solution(case.coords(binding.gll(case.p)[0]))
    else:
        fo = fg = W.uniform_nodal(top.n_dof(), 2)
    bo = oop.rhs(top, np.reshape(fo, (top.E,) + (case.p + 1,) * 3))
    return lv, bo, fg


STARTS = [('c1_cart_p4_4^3', Case('c1', 4, 4), True), ('curved_p4_3^3', Case('curved', 4, 3, amp=0.03), False)]


@pytest.mark.parametrize('name,case,smooth_rhs', STARTS, ids=[s[0] for s in STARTS])
@pytest.mark.parametrize('start', ['fmg', 'cmg'])
@pytest.mark.parametrize('smoother,ns', [('was', (2, 2)), ('scg', (3, 1))])
def test_startup_matches_oracle(binding, name, case, smooth_rhs, start, smoother, ns):
    print('startup', name, start, smoother, flush=True)
    lv, bo, fg = _problem(case, binding, smooth_rhs)
    opts = osv.Options(smoother, *ns, ns0=3)
    ref = (osv.fmg_start if start == 'fmg' else osv.cmg_start)(lv, np.zeros_like(bo), bo, opts)
    lib = case.library(binding, smoother=binding.SCG if smoother == 'scg' else binding.WAS, ns1=ns[0], ns2=ns[1],
                       ns0=3, start=binding.START_FMG if start == 'fmg' else binding.START_CMG)
    b = torch.empty(bo.size, dtype=torch.float64, device='cuda')
    lib.rhs(dev(fg), b)
    u = torch.zeros_like(b)
    lib.startup(u, b)
    assert rel(host(u), ref) <= 1e-10
    lib.close()


@pytest.mark.parametrize('start', ['fmg', 'cmg'])
def test_startup_and_crossover_histories_match_oracle(binding, start):
    """FAS-FMG-SCG(3,1,2) and FAS-CMG-WAS(2,1,2) on the curved p = 4 3^3 mesh: start-up, then
    cycles whose finest-level pre-smoothing after the first is nsc - ns2, to 1e-10."""
    case = Case('curved', 4, 3, amp=0.03)
    print('startup + crossover history', start, flush=True)
    lv, bo, fg = _problem(case, binding, False)
    sm, ns = (('scg', (3, 1)) if start == 'fmg' else ('was', (2, 1)))
    uo, ho = osv.solve(lv, np.zeros_like(bo), bo, osv.Options(sm, *ns, start=start, nsc=2), max_cycles=30)
    for graph in (0, 1):
        lib = case.library(binding, smoother=binding.SCG if sm == 'scg' else binding.WAS, ns1=ns[0], ns2=ns[1],
                           nsc=2, graph=graph, start=binding.START_FMG if start == 'fmg' else binding.START_CMG)
        b = torch.empty(bo.size, dtype=torch.float64, device='cuda')
        lib.rhs(dev(fg), b)
        u = torch.zeros_like(b)
        hg, ok = lib.solve(u, b, max_cycles=30, rtol=1e-10)
        assert ok
        histories_agree(list(hg), ho)
        assert rel(host(u), uo) <= 1e-9
        lib.close()


def test_fmg_reduces_the_first_cycle_on_c1(binding):
    """On C1 (smooth manufactured solution) the FMG start-up leaves a first-cycle residual two
    orders below the plain first cycle's, as in the oracle."""
    case = Case('c1', 4, 4)
    _, bo, fg = _problem(case, binding, True)
    first = {}
    for start in (binding.START_NONE, binding.START_FMG):
        lib = case.library(binding, start=start)
        b = torch.empty(bo.size, dtype=torch.float64, device='cuda')
        lib.rhs(dev(fg), b)
        u = torch.zeros_like(b)
        hg, ok = lib.solve(u, b, max_cycles=1, rtol=1e-10)
        first[start] = hg[1]
        lib.close()
    assert first[binding.START_FMG] < 0.02 * first[binding.START_NONE]


OPTION_CASES = [
    Case('plain_weighting_curved_p4_3^3', 4, 3, amp=0.03, weighting='plain'),
    # delta = 0.24: m = 3 at p = 8, 2 at p = 4, 1 at p = 2 and 1
    Case('delta0.24_curved_p8_2^3', 8, 2, amp=0.03, mu_star=5.0, delta=0.24),
    Case('delta0.24_stretched_p8_3^3', 8, 3, lengths=(1.0, 1.0, 100.0), perturb=(0.2, 4), mu_star=5.0, delta=0.24),
    Case('delta0.08_cart_p4_3^3', 4, 3, delta=0.08),
]


@pytest.mark.parametrize('case', OPTION_CASES, ids=repr)
def test_weighting_and_delta_schwarz_every_level(binding, case):
    print('options', case, flush=True)
    lv = case.oracle_levels()
    lib = case.library(binding)
    rng = np.random.default_rng(5)
    for l in range(1, lib.n_levels + 1):
        n = lv[l - 1].mesh.n_dof()
        g = rng.uniform(-1, 1, n)
        z = torch.empty(n, dtype=torch.float64, device='cuda')
        lib.schwarz(l, dev(g), z)
        assert rel(host(z), lv[l - 1].B(g)) <= 1e-11, l
    lib.close()


def test_delta_overlap_history_on_the_stretched_mesh(binding):
    """The stretched (1:100) perturbed p = 8 mesh with the paper's aspect-ratio overlap
    delta = 0.24 (m = 3 at p = 8, 2 at p = 4): FAS-MG-SCG(12,4) histories against the C/OpenMP
    oracle (pinned to the numpy oracle on these levels by the Schwarz check above)."""
    from oracle import o1
    case = OPTION_CASES[2]
    fast = o1.O1(8, case.coords(ogll(8)[0]), case.nbr, case.bc, mu_star=5.0, delta=0.24)
    f = W.uniform_nodal(fast.ndof[4], 4000)
    uo, ho, _ = fast.solve(fast.rhs(f), smoother='scg', ns1=12, ns2=4, max_cycles=6)
    fast.close()
    lib = case.library(binding, smoother=binding.SCG, ns1=12, ns2=4)
    b = torch.empty(f.size, dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b)
    u = torch.zeros_like(b)
    hg, ok = lib.solve(u, b, max_cycles=6, rtol=1e-10)
    assert ok
    histories_agree(list(hg), ho)
    assert rel(host(u), uo) <= 1e-9
    lib.close()


def test_l2_projection_transfers_and_history(binding):
    """projection = L2 (Sec. 3.2): dgfas_project on every level against the oracle's
    reference-element L2 projection, and the FAS-MG-WAS(2,2) history with it."""
    from oracle import transfer as otr
    case = Case('curved', 4, 3, amp=0.03)
    lv = case.oracle_levels()
    lib = case.library(binding, projection=binding.PROJECT_L2)
    rng = np.random.default_rng(9)
    for l in range(2, lib.n_levels + 1):
        pf, pc = lv[l - 1].p, lv[l - 2].p
        uf = rng.uniform(-1, 1, lv[l - 1].mesh.n_dof())
        out = torch.empty(lv[l - 2].mesh.n_dof(), dtype=torch.float64, device='cuda')
        lib.project(l, dev(uf), out)
        ref = otr.project(pc, pf, uf.reshape((case.E,) + (pf + 1,) * 3), 'l2')
        assert rel(host(out), ref) <= 1e-13, l
    top = lv[-1].mesh
    f = W.uniform_nodal(top.n_dof(), 2)
    bo = oop.rhs(top, f.reshape((top.E,) + (5,) * 3))
    uo, ho = osv.solve(lv, np.zeros_like(bo), bo, osv.Options('was', 2, 2, projection='l2'), max_cycles=30)
    b = torch.empty(bo.size, dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b)
    u = torch.zeros_like(b)
    hg, ok = lib.solve(u, b, max_cycles=30, rtol=1e-10)
    assert ok
    histories_agree(list(hg), ho)
    assert rel(host(u), uo) <= 1e-9
    lib.close()
