"""Addition (4): learned subdomain correction -- data pipeline, inference hook and fallback."""
import numpy as np
import pytest

from oracle import operator as oop, solvers as osv
from oracle.schwarz import Schwarz, local_pair, linear_jacobian
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


def embed(tile, shape, ns):
    out = np.zeros((ns, ns, ns))
    out[:shape[0], :shape[1], :shape[2]] = tile.reshape(shape)
    return out.ravel()


@pytest.mark.parametrize('centers', [[62], [0, 124], [31]])
def test_pairs_match_dense_local_solves(binding, centers):
    """5^3 perturbed elements, p = 2: X and T against the oracle's dense local Cholesky solves."""
    case = Case('pert_p2_5^3', 2, 5, perturb=(0.15, 7), mu_star=3.0)
    print('pairs', centers, flush=True)
    lv = case.oracle_levels()
    mesh = lv[-1].mesh
    A = oop.assemble(mesh)
    sz = Schwarz(mesh, 1)
    r = np.random.default_rng(40).uniform(-1, 1, mesh.n_dof())
    lib = case.library(binding)
    ns = 5
    n = len(centers)
    X = torch.empty((n, ns ** 3 + 9), dtype=torch.float32, device='cuda')
    T = torch.empty((n, ns ** 3), dtype=torch.float32, device='cuda')
    it = binding.learned_pairs(lib, dev(r), np.array(centers), X, T)
    print('pcg iterations', it)
    Xh, Th = host(X), host(T)
    J9 = linear_jacobian(mesh)
    for row, e in enumerate(centers):
        shape, rs, fd, exact = local_pair(mesh, sz, A, r, e)
        nrm = np.linalg.norm(rs)
        assert np.abs(Xh[row, :ns ** 3] - embed(rs / nrm, shape, ns)).max() < 1e-6
        assert np.abs(Xh[row, ns ** 3:] - J9[e].ravel()).max() < 1e-6
        t_ref = embed((exact - fd) / nrm, shape, ns)
        assert np.abs(Th[row] - t_ref).max() <= 1e-5 * max(np.abs(t_ref).max(), 1e-3)
    lib.close()


def test_pairs_vanish_on_cartesian_boxes(binding):
    """On undeformed Cartesian elements the FD solve is exact, so every target is zero."""
    case = Case('cart_p3_6^3', 3, 6)
    lib = case.library(binding)
    n3 = 6 ** 3 * 64
    r = dev(np.random.default_rng(41).uniform(-1, 1, n3))
    centers = np.array([0, 4 + 6 * (4 + 6 * 4), 0 + 6 * (5 + 6 * 0)])   # (0,0,0), (4,4,4), (0,5,0)
    X = torch.empty((3, 6 ** 3 + 9), dtype=torch.float32, device='cuda')
    T = torch.empty((3, 6 ** 3), dtype=torch.float32, device='cuda')
    binding.learned_pairs(lib, r, centers, X, T)
    assert np.abs(host(T)).max() < 1e-7
    with pytest.raises(binding.DgfasError):
        binding.learned_pairs(lib, r, np.array([0, 1]), X, T)      # patches overlap
    lib.close()


def test_zero_network_reproduces_plain_smoother(binding):
    case = Case('curved_p8_3^3', 8, 3, amp=0.03, mu_star=5.0)
    lib = case.library(binding, smoother=binding.SCG, ns1=2, ns2=2)
    net = binding.Mlp(11 ** 3 + 9, 64, 11 ** 3, seed=1)
    theta = net.get_params()
    theta[-(64 * 11 ** 3 + 11 ** 3):] = 0.0       # W3 = 0, b3 = 0: the network outputs zero
    net.set_params(theta)
    n = 27 * 729
    g = dev(np.random.default_rng(42).uniform(-1, 1, n))
    u0 = np.random.default_rng(43).uniform(-1, 1, n)
    ua, ub = dev(u0), dev(u0)
    lib.smooth(lib.n_levels, ua, g, 2)
    binding.set_learned(lib, net, True)
    lib.smooth(lib.n_levels, ub, g, 2)
    assert np.array_equal(host(ua), host(ub))
    binding.set_learned(lib, None, False)
    lib.close()
    net.close()


def test_fallback_rejects_a_harmful_network(binding):
    """A large random network makes the cycle worse: the solve undoes it, continues plain,
    converges and reports DGFAS_EFALLBACK; the solution equals the plain solve's."""
    case = Case('curved_p8_3^3', 8, 3, amp=0.03, mu_star=5.0)
    opts = dict(smoother=binding.SCG, ns1=3, ns2=2, root_rtol=1e-1)
    lib = case.library(binding, **opts)
    n = 27 * 729
    f = dev(W.uniform_nodal(n, 2))
    b = torch.empty_like(f)
    lib.rhs(f, b)
    u_plain = torch.zeros_like(b)
    hp, code_p = binding.solve_status(lib, u_plain, b, 40)
    net = binding.Mlp(11 ** 3 + 9, 64, 11 ** 3, seed=9)
    theta = net.get_params()
    theta[-11 ** 3:] = 5.0                          # b3 = 5: a large constant correction
    net.set_params(theta)
    binding.set_learned(lib, net, True)
    u = torch.zeros_like(b)
    hl, code = binding.solve_status(lib, u, b, 40)
    assert code_p == 0 and code == binding.DGFAS_EFALLBACK
    assert hl[-1] <= 1e-10
    assert np.abs(host(u) - host(u_plain)).max() <= 1e-8 * np.abs(host(u_plain)).max()
    lib.close()
    net.close()
