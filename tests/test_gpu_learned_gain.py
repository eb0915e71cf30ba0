"""What the trained network gains: the whole learned pipeline at reduced size.

Pairs from plain FAS-MG-SCG(3,2) cycles on two seeded curved 8^3, p = 8 meshes, GPU training,
then plain vs learned (with the fallback judge) on a held-out mesh of the same family.  The
test records the gain (plain minus learned n10 and t10) and requires that both solves reach
1e-10.  A learned solve that needs more cycles or more time than the plain one, or whose
network the judge switched off, is a loss and is reported as an expected failure with the
numbers, not as a pass."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


def test_learned_vs_plain(capsys):
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2608_14123_amd import learned as LR
    ne = 8
    X, T, st = LR.generate_pairs(torch, ne, [40, 41], [4100, 4101], [0, 2])
    assert st['pairs'] == 2 * 2 * 2 * ne ** 3 and np.isfinite(X.cpu().numpy()).all()
    net, tr = LR.train(torch, X, T, epochs=40, batch=1024)
    assert tr['loss_last'] < tr['loss_first']
    ev = LR.evaluate(torch, net, ne, 47, 4000, max_cycles=40)
    plain, learned = ev['plain'], ev['learned']
    print(json.dumps({'pairs': st, 'training': tr,
                      'plain': {k: plain[k] for k in ('n10', 't10_s', 'status')},
                      'learned': {k: learned[k] for k in ('n10', 't10_s', 'status')},
                      'learned_without_judge': {k: ev['learned_unjudged'][k] for k in ('n10', 'final_rho')}}))
    net.close()
    assert plain['status'] == 0 and plain['final_rho'] <= 1e-10
    assert learned['status'] in (0, 2) and learned['final_rho'] <= 1e-10
    gain = {'n10': plain['n10'] - learned['n10'], 't10_s': round(plain['t10_s'] - learned['t10_s'], 4),
            'fallback': learned['status'] == 2}
    print(json.dumps({'gain': gain}))
    if gain['fallback'] or gain['n10'] < 0 or gain['t10_s'] < 0:
        pytest.xfail('the learned correction loses to the plain smoother: %s' % json.dumps(gain))
