"""GPU parity of every hot-path step against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest

from oracle import operator as oop, solvers as osv, transfer as otr
from paper_2608_14123_amd import workloads as W
from gpu_cases import CASES

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


def relerr(a, b):
    return np.abs(np.ravel(a) - np.ravel(b)).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope='module', params=CASES, ids=repr)
def pair(request, binding):
    case = request.param
    print('case', case.name, flush=True)
    lib = case.library(binding)
    lv = case.oracle_levels()
    yield case, lib, lv
    lib.close()


def test_operator_every_level(pair):
    case, lib, lv = pair
    rng = np.random.default_rng(10)
    assert lib.n_levels == len(lv)
    for l in range(1, lib.n_levels + 1):
        o = lv[l - 1]
        u = rng.uniform(-1, 1, o.mesh.n_dof())
        g = rng.uniform(-1, 1, o.mesh.n_dof())
        ud, out = dev(u), torch.empty(o.mesh.n_dof(), dtype=torch.float64, device='cuda')
        lib.apply(l, ud, out)
        ref = o.A(u)
        assert relerr(host(out), ref) < 1e-12, (case.name, l)
        lib.residual(l, ud, dev(g), out)
        assert relerr(host(out), g - ref.ravel()) < 1e-12


def test_rhs(pair):
    case, lib, lv = pair
    top = lv[-1].mesh
    rng = np.random.default_rng(11)
    f = rng.uniform(-1, 1, top.n_dof())
    uD = rng.uniform(-1, 1, top.n_dof())
    qN = rng.uniform(-1, 1, top.n_dof())
    b = torch.empty(top.n_dof(), dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b, uD=dev(uD), qN=dev(qN))
    ref = oop.rhs(top, f, uD=uD, qN=qN)
    assert relerr(host(b), ref) < 1e-12


def test_schwarz_every_level(pair):
    case, lib, lv = pair
    rng = np.random.default_rng(12)
    for l in range(1, lib.n_levels + 1):
        o = lv[l - 1]
        r = rng.uniform(-1, 1, o.mesh.n_dof())
        z = torch.empty(o.mesh.n_dof(), dtype=torch.float64, device='cuda')
        lib.schwarz(l, dev(r), z)
        assert relerr(host(z), o.B(r)) < 1e-11, (case.name, l)


def test_transfers(pair):
    case, lib, lv = pair
    rng = np.random.default_rng(13)
    for l in range(2, lib.n_levels + 1):
        f, c = lv[l - 1], lv[l - 2]
        uf = rng.uniform(-1, 1, f.mesh.n_dof())
        uc = rng.uniform(-1, 1, c.mesh.n_dof())
        ub = rng.uniform(-1, 1, c.mesh.n_dof())
        out_c = torch.empty(c.mesh.n_dof(), dtype=torch.float64, device='cuda')
        lib.project(l, dev(uf), out_c)
        assert relerr(host(out_c), otr.project(c.p, f.p, uf.reshape(f.mesh.E, f.mesh.n, f.mesh.n, f.mesh.n))) < 1e-13
        lib.restrict(l, dev(uf), out_c)
        assert relerr(host(out_c), otr.restrict(c.p, f.p, uf.reshape(f.mesh.E, f.mesh.n, f.mesh.n, f.mesh.n))) < 1e-13
        fine = dev(uf)
        lib.prolong_add(l, dev(uc), fine, ubar=dev(ub))
        d = (uc - ub).reshape(c.mesh.E, c.mesh.n, c.mesh.n, c.mesh.n)
        assert relerr(host(fine), uf + otr.prolong(c.p, f.p, d).ravel()) < 1e-13


def test_was_steps(pair):
    case, lib, lv = pair
    rng = np.random.default_rng(14)
    top = lv[-1]
    u = rng.uniform(-1, 1, top.mesh.n_dof())
    g = rng.uniform(-1, 1, top.mesh.n_dof())
    ud = dev(u)
    lib.smooth(lib.n_levels, ud, dev(g), 2)
    ref = osv.was(top, u.reshape(top.mesh.E, top.mesh.n, top.mesh.n, top.mesh.n), g.reshape(-1).reshape(
        top.mesh.E, top.mesh.n, top.mesh.n, top.mesh.n), 2)
    assert relerr(host(ud), ref) < 1e-11


def test_root_solve(pair):
    case, lib, lv = pair
    if case.kappa == 0 and case.name.startswith('neumann'):
        pytest.skip('singular')
    root = lv[0]
    rng = np.random.default_rng(15)
    g = rng.uniform(-1, 1, root.mesh.n_dof())
    u = np.zeros(root.mesh.n_dof())
    ud = dev(u)
    it = lib.root_solve(ud, dev(g))
    st = {}
    ref = osv.scg(root, u.reshape(root.mesh.E, 2, 2, 2), g.reshape(root.mesh.E, 2, 2, 2), 500,
                  1e-12 * osv.norm(g), stats=st)
    assert it == st['iters']
    assert relerr(host(ud), ref) < 1e-9
