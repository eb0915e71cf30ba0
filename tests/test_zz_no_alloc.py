"""The allocation-free Schwarz application (dgfas_schwarz_noalloc, overlap inbox in the
library's static device array) against dgfas_schwarz: bitwise the same result on two calls
in a row, the second with a smaller input, also across solvers and on a mixed-degree level
whose inbox regions toward other degrees must read zero; levels whose inbox exceeds the
array are refused."""
import numpy as np
import pytest

from gpu_cases import Case, MixedCase

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


@pytest.fixture(scope='module')
def binding():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2608_14123_amd import binding as b
    return b


def _compare(lib, level, rng):
    n = lib._n(level)
    r = torch.from_numpy(rng.uniform(-1, 1, n)).cuda()
    ref = torch.empty_like(r)
    out = torch.full_like(r, float('nan'))
    lib.schwarz(level, r, ref)
    lib.schwarz_noalloc(level, r, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref), (level, (out - ref).abs().max().item())


def test_noalloc_schwarz_equals_schwarz_on_consecutive_calls(binding):
    rng = np.random.default_rng(21)
    print('noalloc: curved p=4 4^3, finest level then the next coarser one', flush=True)
    big = Case('curved_p4_4^3', 4, 4, amp=0.03).library(binding)
    _compare(big, big.n_levels, rng)
    _compare(big, big.n_levels - 1, rng)
    print('noalloc: mixed degrees 1..5 on 3^3 after the larger call', flush=True)
    mixed = MixedCase('mixed_1to5_3^3', 3, np.random.default_rng(3).integers(1, 6, 27), amp=0.03).library(binding)
    for level in range(mixed.n_levels, 0, -1):
        _compare(mixed, level, rng)
    mixed.close()
    big.close()


def test_noalloc_schwarz_refuses_an_inbox_beyond_the_array(binding):
    print('noalloc: 7^3 elements at p = 8 with 64 right-hand sides (13.2M inbox doubles)', flush=True)
    lib = Case('cart_p8_7^3', 8, 7).library(binding, n_rhs=64)
    n = lib._n(lib.n_levels)
    r = torch.zeros(n, dtype=torch.float64, device='cuda')
    z = torch.zeros_like(r)
    with pytest.raises(binding.DgfasError) as err:
        lib.schwarz_noalloc(lib.n_levels, r, z)
    assert 'static scratch array' in str(err.value)
    lib.close()
