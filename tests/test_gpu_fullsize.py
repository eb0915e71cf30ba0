"""Full-size history parity on the curved 32^3, p = 7 workload (16,777,216 DOF), the
configuration the benchmark times: FAS-MG-SCG(3,2), mu_star = 5, root SCG to 1e-1.

The expected history and sampled element blocks of the final iterate are the oracle's
(tests/golden/c2_curved_p7_history.json, written by tests/golden/make_c2_history.py with the
C/OpenMP oracle only).  Criterion: every cycle's relative residual within 1e-6 of the
oracle's (while above 1e-12), the same cycle count to 1e-10, and the final iterate within
1e-9 of the oracle's, relative to its largest value.  The FP32 and BF16 smoothers (FP64
residual, tau-correction and root solve) must reach 1e-10 and the FP64 oracle's solution."""
import json
import os

import numpy as np
import pytest

from paper_2608_14123_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')
GOLDEN = os.path.join(os.path.dirname(__file__), 'golden', 'c2_curved_p7_history.json')


@pytest.fixture(scope='module')
def binding():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2608_14123_amd import binding as b
    return b


@pytest.fixture(scope='module')
def workload(binding):
    ne, p = 32, 7
    V, nbr, bc, mp = W.curved_cube(ne)
    X = W.element_coords(V, binding.gll(p)[0], mp)
    f = W.uniform_nodal(ne ** 3 * (p + 1) ** 3, 2)
    with open(GOLDEN) as fh:
        ref = json.load(fh)
    return ne, p, X, nbr, bc, f, ref


def _solve(binding, workload, **kw):
    ne, p, X, nbr, bc, f, ref = workload
    o = binding.default_options(smoother=binding.SCG, ns1=3, ns2=2, mu_star=5.0, root_rtol=0.1, **kw)
    lib = binding.Solver(np.full(ne ** 3, p, np.int32), X, nbr, bc, o)
    fd = torch.from_numpy(f).cuda()
    b = torch.empty_like(fd)
    lib.rhs(fd, b)
    u = torch.zeros_like(b)
    hist, ok = lib.solve(u, b, max_cycles=30, rtol=1e-10)
    torch.cuda.synchronize()
    uh = u.cpu().numpy()
    lib.close()
    n3 = (p + 1) ** 3
    blocks = np.array([uh[e * n3:(e + 1) * n3] for e in ref['sample_elements']])
    err = np.abs(blocks - np.array(ref['u_blocks'])).max() / ref['u_max_abs']
    return hist, ok, err


def test_curved_32_p7_fp64_history_matches_the_oracle(binding, workload):
    print('full size: curved 32^3 p=7 FP64 FAS-MG-SCG(3,2)', flush=True)
    ref = workload[-1]
    hist, ok, err = _solve(binding, workload)
    assert ok
    assert len(hist) == len(ref['history']), (len(hist), len(ref['history']))
    for k, (a, c) in enumerate(zip(hist, ref['history'])):
        if c > 1e-12:
            assert abs(a - c) <= 1e-6 * c, (k, a, c)
    assert err <= 1e-9, err


@pytest.mark.parametrize('prec', ['FP32', 'BF16'])
def test_curved_32_p7_reduced_precision_smoother_reaches_the_oracle_solution(binding, workload, prec):
    print('full size: curved 32^3 p=7 %s smoother' % prec, flush=True)
    ref = workload[-1]
    hist, ok, err = _solve(binding, workload, precision=getattr(binding, prec))
    assert ok and len(hist) - 1 <= ref['n10'] + 1, (len(hist) - 1, ref['n10'])
    assert err <= 1e-9, err
