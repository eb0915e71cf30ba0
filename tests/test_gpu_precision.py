"""Addition (1): correction-form FP32 smoothing with FP64 residual, tau-correction and root.

The error is stated against the FP64 oracle for the same input: per smoothing call the
relative error of the update du = u_new - u, per solve the final solution."""
import numpy as np
import pytest

from oracle import operator as oop, solvers as osv
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


@pytest.mark.parametrize('smoother,steps,mfma', [('was', 2, False), ('scg', 3, False), ('was', 2, True),
                                                 ('scg', 3, True)])
def test_fp32_smoothing_update_error(binding, smoother, steps, mfma):
    """FP32 smoothing on the vector unit or with the FD contractions on FP32 matrix cores."""
    case = Case('curved_p7', 7, 3, amp=0.03, mu_star=5.0)
    print('fp32 smooth', smoother, 'mfma' if mfma else 'valu', flush=True)
    lv = case.oracle_levels()
    top = lv[-1]
    n = top.mesh.n_dof()
    rng = np.random.default_rng(30)
    u = rng.uniform(-1, 1, n)
    g = rng.uniform(-1, 1, n)
    shape = (top.mesh.E, top.mesh.n, top.mesh.n, top.mesh.n)
    ref = osv.smooth(top, u.reshape(shape), g.reshape(shape), steps, osv.Options(smoother, steps, steps)).ravel()
    lib = case.library(binding, precision=binding.FP32_MFMA if mfma else binding.FP32,
                       smoother=binding.SCG if smoother == 'scg' else binding.WAS)
    ud = dev(u)
    lib.smooth(lib.n_levels, ud, dev(g), steps)
    du_gpu, du_ref = host(ud) - u, ref - u
    err = np.linalg.norm(du_gpu - du_ref) / np.linalg.norm(du_ref)
    print('relative update error %.2e' % err)
    assert err < 1e-5
    lib.close()


@pytest.mark.parametrize('mfma', [False, True])
def test_fp32_solve_reaches_fp64_solution(binding, mfma):
    case = Case('curved_p4', 4, 3, amp=0.03, mu_star=5.0)
    print('fp32 solve', 'mfma' if mfma else 'valu', flush=True)
    lv = case.oracle_levels()
    top = lv[-1].mesh
    f = W.uniform_nodal(top.n_dof(), 2)
    bo = oop.rhs(top, f)
    opts = osv.Options('scg', 3, 2, root_rtol=1e-1)
    uo, ho = osv.solve(lv, np.zeros_like(bo), bo, opts, max_cycles=30)
    lib = case.library(binding, precision=binding.FP32_MFMA if mfma else binding.FP32, smoother=binding.SCG,
                       ns1=3, ns2=2, root_rtol=1e-1)
    b = torch.empty(top.n_dof(), dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b)
    u = torch.zeros_like(b)
    hg, ok = lib.solve(u, b, max_cycles=30, rtol=1e-10)
    assert ok and abs((len(hg) - 1) - (len(ho) - 1)) <= 1
    # early cycles agree to FP32 accuracy
    for a, c in zip(hg[1:4], ho[1:4]):
        assert abs(a - c) <= 1e-4 * c
    err = np.abs(host(u) - uo.ravel()).max() / np.abs(uo).max()
    print('fp32-smoothed solution vs FP64 oracle: %.2e' % err)
    assert err < 1e-9
    lib.close()


@pytest.mark.parametrize('steps', [1, 2])
def test_bf16_matrix_core_smoothing_update_error(binding, steps):
    """FD contractions on BF16 matrix cores (operands rounded to 8 significant bits, FP32
    accumulation): the WAS update stays within a few percent of the FP64 oracle's."""
    case = Case('curved_p7', 7, 3, amp=0.03, mu_star=5.0)
    print('bf16 smooth', steps, flush=True)
    lv = case.oracle_levels()
    top = lv[-1]
    n = top.mesh.n_dof()
    rng = np.random.default_rng(31)
    u = rng.uniform(-1, 1, n)
    g = rng.uniform(-1, 1, n)
    shape = (top.mesh.E, top.mesh.n, top.mesh.n, top.mesh.n)
    ref = osv.smooth(top, u.reshape(shape), g.reshape(shape), steps, osv.Options('was', steps, steps)).ravel()
    lib = case.library(binding, precision=binding.BF16, smoother=binding.WAS)
    ud = dev(u)
    lib.smooth(lib.n_levels, ud, dev(g), steps)
    du_gpu, du_ref = host(ud) - u, ref - u
    err = np.linalg.norm(du_gpu - du_ref) / np.linalg.norm(du_ref)
    print('bf16 relative update error %.2e' % err)
    assert err < 3e-2
    lib.close()


def test_bf16_solve_reaches_fp64_solution(binding):
    """The FP64 residual and tau-correction keep the BF16-smoothed cycle converging to the
    FP64 solution; the cycle count is stated against FP64."""
    case = Case('curved_p4', 4, 3, amp=0.03, mu_star=5.0)
    print('bf16 solve', flush=True)
    lv = case.oracle_levels()
    top = lv[-1].mesh
    f = W.uniform_nodal(top.n_dof(), 2)
    bo = oop.rhs(top, f)
    opts = osv.Options('scg', 3, 2, root_rtol=1e-1)
    uo, ho = osv.solve(lv, np.zeros_like(bo), bo, opts, max_cycles=30)
    lib = case.library(binding, precision=binding.BF16, smoother=binding.SCG, ns1=3, ns2=2, root_rtol=1e-1)
    b = torch.empty(top.n_dof(), dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b)
    u = torch.zeros_like(b)
    hg, ok = lib.solve(u, b, max_cycles=60, rtol=1e-10)
    print('cycles to 1e-10: bf16 %d, fp64 oracle %d' % (len(hg) - 1, len(ho) - 1))
    assert ok and len(hg) - 1 <= 2 * (len(ho) - 1)
    err = np.abs(host(u) - uo.ravel()).max() / np.abs(uo).max()
    print('bf16-smoothed solution vs FP64 oracle: %.2e' % err)
    assert err < 1e-9
    lib.close()
