"""Caller-owned workspace (dgfas_workspace_size / dgfas_set_workspace): the configured cycle
runs in a torch tensor's memory with bitwise the results of the library-owned block, also
after switching back and forth; short or misaligned buffers are refused."""
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


def _solve(lib, f, cycles):
    n = lib._n(lib.n_levels)
    b = torch.empty(n, dtype=torch.float64, device='cuda')
    lib.rhs(f, b)
    u = torch.zeros_like(b)
    hist, _ = lib.solve(u, b, max_cycles=cycles, rtol=1e-10)
    torch.cuda.synchronize()
    return np.array(hist), u.cpu().numpy()


CASES = [('curved_p4_3^3_scg_fp64', lambda B: Case('curved', 4, 3, amp=0.03).library(
             B, smoother=B.SCG, ns1=3, ns2=2, start=B.START_FMG, nsc=3, graph=1)),
         ('mixed_1to5_3^3_scg_fp32', lambda B: MixedCase('mixed', 3, np.random.default_rng(3).integers(1, 6, 27),
                                                            amp=0.03).library(B, precision=B.FP32, smoother=B.SCG))]


@pytest.mark.parametrize('name,make', CASES, ids=[c[0] for c in CASES])
def test_caller_workspace_gives_the_same_solve(binding, name, make):
    print('workspace', name, flush=True)
    ref_lib = make(binding)
    n = ref_lib._n(ref_lib.n_levels)
    f = torch.from_numpy(W.uniform_nodal(n, 2)).cuda()
    h_ref, u_ref = _solve(ref_lib, f, 8)
    ref_lib.close()
    lib = make(binding)
    size = lib.workspace_size()
    assert size >= 8 * n          # at least the finest residual vector
    buf = torch.empty(size, dtype=torch.uint8, device='cuda')
    lib.set_workspace(buf)
    h, u = _solve(lib, f, 8)
    assert np.array_equal(h, h_ref) and np.array_equal(u, u_ref)
    lib.set_workspace(None)
    h, u = _solve(lib, f, 8)
    assert np.array_equal(h, h_ref) and np.array_equal(u, u_ref)
    buf2 = torch.empty(size + 512, dtype=torch.uint8, device='cuda')
    lib.set_workspace(buf2)
    h, u = _solve(lib, f, 8)
    assert np.array_equal(h, h_ref) and np.array_equal(u, u_ref)
    with pytest.raises(ValueError):                      # the binding refuses a short tensor
        lib.set_workspace(buf[:size - 8])
    # and so does the library itself, for a short size or a misaligned pointer
    assert binding._lib.dgfas_set_workspace(lib._h, buf.data_ptr(), size - 8) == binding.DGFAS_EINVAL
    with pytest.raises(binding.DgfasError):
        lib.set_workspace(buf2[1:])
    h, u = _solve(lib, f, 8)                            # the refusals left the workspace in place
    assert np.array_equal(h, h_ref) and np.array_equal(u, u_ref)
    lib.close()
