"""The Morton element order of the sweep kernels changes only the order in which workgroups
take elements: operator and Schwarz outputs are bitwise those of the natural order; the fused
SCG dot products sum their per-tile partials in another order, so cycles agree to rounding."""
import numpy as np
import pytest

from paper_2608_14123_amd import workloads as W
from gpu_cases import Case, MixedCase

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


@pytest.fixture(scope='module')
def binding():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2608_14123_amd import binding as b
    return b


def run(lib, n, levels):
    rng = np.random.default_rng(21)
    out = []
    for l in range(1, levels + 1):
        nl = lib.level_info(l)[1]
        u = torch.from_numpy(rng.uniform(-1, 1, nl)).cuda()
        y = torch.empty_like(u)
        lib.apply(l, u, y)
        out.append(y.cpu().numpy())
        lib.schwarz(l, u, y)
        out.append(y.cpu().numpy())
    f = torch.from_numpy(W.uniform_nodal(n, 2)).cuda()
    b = torch.empty_like(f)
    lib.rhs(f, b)
    u = torch.zeros_like(b)
    hist, _ = lib.solve(u, b, max_cycles=3, rtol=0.0)
    out += [hist, u.cpu().numpy()]
    return out


@pytest.mark.parametrize('case', [Case('curved_p4_4^3', 4, 4, amp=0.03),
                                  MixedCase('mixed_2to4_4^3', 4, np.random.default_rng(5).integers(2, 5, 64),
                                            amp=0.03)], ids=repr)
def test_morton_order_is_bitwise_natural(binding, case):
    print('order', case, flush=True)
    res = []
    for order in (binding.ORDER_NATURAL, binding.ORDER_MORTON):
        lib = case.library(binding, smoother=binding.SCG, ns1=3, ns2=2, root_rtol=1e-1, order=order)
        n = lib.level_info(lib.n_levels)[1]
        res.append(run(lib, n, lib.n_levels))
        lib.close()
    for a, b in zip(res[0][:-2], res[1][:-2]):
        assert np.array_equal(a, b)
    for a, b in zip(res[0][-2:], res[1][-2:]):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
