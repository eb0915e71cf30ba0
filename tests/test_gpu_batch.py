"""Multi-right-hand-side batches (vectors [n_rhs][n_dof]) against the oracle run per right-hand side."""
import numpy as np
import pytest

from oracle import operator as oop, solvers as osv
from paper_2608_14123_amd import workloads as W
from gpu_cases import Case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')

R = 3


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


@pytest.fixture(scope='module')
def stretched():
    # anisotropic perturbed elements (1:100 in z, 20% vertex perturbation), p = 8, mu_star = 5
    return Case('stretched_p8_3^3', 8, 3, lengths=(1.0, 1.0, 100.0), perturb=(0.2, 4), mu_star=5.0)


def test_batched_operator_and_schwarz(binding, stretched):
    print('batch kernels', flush=True)
    lv = stretched.oracle_levels()
    lib = stretched.library(binding, n_rhs=R)
    rng = np.random.default_rng(20)
    for l in range(1, lib.n_levels + 1):
        o = lv[l - 1]
        n = o.mesh.n_dof()
        u = rng.uniform(-1, 1, (R, n))
        out = torch.empty(R * n, dtype=torch.float64, device='cuda')
        lib.apply(l, dev(u), out)
        got = host(out).reshape(R, n)
        for k in range(R):
            ref = o.A(u[k]).ravel()
            assert np.abs(got[k] - ref).max() <= 1e-12 * np.abs(ref).max()
        lib.schwarz(l, dev(u), out)
        got = host(out).reshape(R, n)
        for k in range(R):
            ref = o.B(u[k]).ravel()
            assert np.abs(got[k] - ref).max() <= 1e-11 * np.abs(ref).max()
        nrm = lib.norm(l, dev(u))
        assert np.allclose(nrm, np.linalg.norm(u, axis=1), rtol=1e-13)
    lib.close()


def test_batched_scg_vcycles(binding, stretched):
    """FAS-MG-SCG(3,2) on three right-hand sides at once: every right-hand side follows its
    own oracle iterates (per-rhs SCG scalars); the reported history is the worst one."""
    print('batch vcycle', flush=True)
    lv = stretched.oracle_levels()
    top = lv[-1].mesh
    n = top.n_dof()
    f = np.stack([W.uniform_nodal(n, 4000 + k) for k in range(R)])
    cycles = 4
    opts = osv.Options('scg', 3, 2, root_rtol=1e-1)
    hists, sols = [], []
    for k in range(R):
        bo = oop.rhs(top, f[k])
        u, h = osv.solve(lv, np.zeros_like(bo), bo, opts, max_cycles=cycles, rtol=0.0)
        hists.append(h)
        sols.append(u.ravel())
    ref_hist = np.max(np.array(hists), axis=0)
    lib = stretched.library(binding, n_rhs=R, smoother=binding.SCG, ns1=3, ns2=2, root_rtol=1e-1)
    b = torch.empty(R * n, dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b)
    u = torch.zeros_like(b)
    hg, ok = lib.solve(u, b, max_cycles=cycles, rtol=0.0)
    assert len(hg) == len(ref_hist)
    for a, c in zip(hg, ref_hist):
        assert abs(a - c) <= 1e-6 * c + 1e-14, (hg, ref_hist)
    got = host(u).reshape(R, n)
    for k in range(R):
        assert np.abs(got[k] - sols[k]).max() <= 1e-9 * np.abs(sols[k]).max()
    lib.close()


@pytest.mark.parametrize('precision', ['fp32', 'bf16'])
def test_batched_rhs_match_single_solves(binding, stretched, precision):
    """A batch of right-hand sides with the reduced-precision smoother and the whole cycle as
    one graph (fixed-iteration root): each right-hand side's iterate is bitwise the one of its
    own single solve, and the history is the worst of theirs."""
    print('batch single', precision, flush=True)
    prec = binding.FP32 if precision == 'fp32' else binding.BF16
    n = stretched.oracle_levels()[-1].mesh.n_dof()
    f = np.stack([W.uniform_nodal(n, 4100 + k) for k in range(R)])
    kw = dict(smoother=binding.SCG, ns1=3, ns2=2, root_rtol=0.0, root_max_iter=6, graph=1, precision=prec)
    cycles = 3
    singles, hists = [], []
    for k in range(R):
        lib = stretched.library(binding, **kw)
        b = torch.empty(n, dtype=torch.float64, device='cuda')
        lib.rhs(dev(f[k]), b)
        u = torch.zeros_like(b)
        h, _ = lib.solve(u, b, max_cycles=cycles, rtol=0.0)
        singles.append(host(u).copy())
        hists.append(h)
        lib.close()
    lib = stretched.library(binding, n_rhs=R, **kw)
    b = torch.empty(R * n, dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b)
    u = torch.zeros_like(b)
    hg, _ = lib.solve(u, b, max_cycles=cycles, rtol=0.0)
    got = host(u).reshape(R, n)
    for k in range(R):
        assert np.array_equal(got[k], singles[k]), k
    assert np.array_equal(hg, np.max(np.array(hists), axis=0))
    lib.close()
