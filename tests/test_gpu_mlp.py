"""GPU network kernels (BF16 MFMA GEMMs, FP32 accumulation) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


@pytest.fixture(scope='module')
def binding():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2608_14123_amd import binding as b
    return b


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), as float64."""
    a = np.asarray(a, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def blocks(n_in, h, n_out):
    """(name, slice) of the parameter blocks W1 b1 W2 b2 W3 b3."""
    out, o = [], 0
    for name, n in (('W1', n_in * h), ('b1', h), ('W2', h * h), ('b2', h), ('W3', h * n_out), ('b3', n_out)):
        out.append((name, slice(o, o + n)))
        o += n
    return out


# rows >= 512 take the split-K weight gradients (K = rows cut into slices, the last one ragged)
# and several chunks of the bias column sums
@pytest.mark.parametrize('n_in,h,n_out,rows', [(37, 64, 29, 50), (1340, 256, 1331, 96), (64, 64, 40, 1500),
                                               (1340, 256, 1331, 1100)])
def test_forward_and_gradient(binding, n_in, h, n_out, rows):
    print('mlp', n_in, h, n_out, rows, flush=True)
    net = binding.Mlp(n_in, h, n_out, seed=5)
    rng = np.random.default_rng(1)
    theta = net.get_params().astype(np.float64)
    theta[-n_out:] = rng.standard_normal(n_out) * 0.1
    theta = bf16_round(theta)                  # weights exactly representable in BF16
    net.set_params(theta.astype(np.float32))
    X = bf16_round(rng.standard_normal((rows, n_in)))
    T = rng.standard_normal((rows, n_out))
    Y = torch.empty((rows, n_out), dtype=torch.float32, device='cuda')
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    net.forward(Xd, Y)
    torch.cuda.synchronize()
    Yo, _ = omlp.forward(theta, X, n_in, h, n_out)
    ferr = np.linalg.norm(Y.cpu().numpy() - Yo) / np.linalg.norm(Yo)
    grad = torch.empty(net.n_params, dtype=torch.float32, device='cuda')
    loss = net.gradient(Xd, torch.from_numpy(T.astype(np.float32)).cuda(), grad)
    lo, go = omlp.loss_and_grad(theta, X, T, n_in, h, n_out)
    gerr = np.linalg.norm(grad.cpu().numpy() - go) / np.linalg.norm(go)
    print('forward rel err %.2e, loss rel err %.2e, gradient rel err %.2e' % (ferr, abs(loss - lo) / lo, gerr))
    # BF16 rounding of the hidden activations and of the back-propagated signals bounds the error
    assert ferr < 2e-2 and abs(loss - lo) / lo < 2e-2 and gerr < 5e-2
    g = grad.cpu().numpy()
    for name, sl in blocks(n_in, h, n_out):
        berr = np.linalg.norm(g[sl] - go[sl]) / np.linalg.norm(go[sl])
        assert berr < 5e-2, (name, berr)
    net.close()


def test_training_reduces_loss_on_a_linear_map(binding):
    n_in, h, n_out, n = 64, 128, 48, 4096
    rng = np.random.default_rng(2)
    A = rng.standard_normal((n_in, n_out)) / np.sqrt(n_in)
    X = rng.standard_normal((n, n_in)).astype(np.float32)
    T = (X @ A).astype(np.float32)
    net = binding.Mlp(n_in, h, n_out, seed=3)
    losses = net.train(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), batch=256, steps=400,
                       lr0=3e-3, lr_min=1e-4)
    print('loss %.3e -> %.3e' % (losses[0], losses[-1]))
    assert losses[-1] < 0.05 * losses[0]
    net.close()
