"""Local refinement at the benchmark's size (curved 16^3, p = 7, zones of radius 0.3 and 0.15:
10.2M active DOF on 5 levels), checked through properties the converged FAS state has at any
size (eq. helmholtz:fas:converged).  After FAS-FMG-SCG(3,2) to a composite residual of 1e-10,
every twig equals the projection P of its active children and every frozen element the
interpolation I of its leaf parent, up to the solve's tolerance.  A level built by refinement
lists 8 children per refined parent in parent order; each block's parent is found from the
geometry (the element whose mean node is nearest to the block's)."""
import numpy as np
import pytest

from oracle import hmg
from paper_2608_14123_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


def _t3(Tz, Ty, Tx, u):
    return np.einsum('ck,bj,ai,...kji->...cba', Tz, Ty, Tx, u)


def test_converged_state_satisfies_the_composite_equations():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2608_14123_amd import binding as B
    ne, p = 16, 7
    n = p + 1
    refine = W.local_refine_lists(ne, [((0.5, 0.5, 0.5), 0.3), ((0.5, 0.5, 0.5), 0.15)])
    V, nbr, bc, mp = W.curved_cube(ne)
    X = W.element_coords(V, B.gll(p)[0], mp)
    print('local refinement full size', [len(r) for r in refine], flush=True)
    lib = B.Solver(np.full(ne ** 3, p, np.int32), X, nbr, bc,
                   B.default_options(local_steps=2, mu_star=5.0, root_rtol=0.1, smoother=B.SCG, ns1=3, ns2=2,
                                     start=B.START_FMG), refine=refine)
    L = lib.n_levels
    bl, coords = [], []
    for l in range(1, L + 1):
        Xl = lib.level_coords(l)
        coords.append(Xl)
        t = torch.empty(Xl.size // 3, dtype=torch.float64, device='cuda')
        lib.level_rhs(l, torch.from_numpy(W.gaussian_source(Xl).ravel()).cuda(), t, uD=torch.zeros_like(t))
        bl.append(t)
        if l < L:
            lib.set_level_rhs(l, t)
    u = torch.zeros_like(bl[-1])
    hist, ok = lib.solve(u, bl[-1], max_cycles=40, rtol=1e-10)
    hist = list(hist)
    print('history', ['%.2e' % h for h in hist], flush=True)
    assert ok and len(hist) - 1 <= 25, hist
    us = []
    for l in range(1, L):
        t = torch.empty_like(bl[l - 1])
        lib.level_solution(l, t)
        us.append(t.cpu().numpy().reshape(-1, n, n, n))
    us.append(u.cpu().numpy().reshape(-1, n, n, n))
    scale = np.abs(us[-1]).max()
    I, P = hmg.child_matrices(p)
    for l in (L - 1, L):                       # the two levels built by refinement (1-based)
        cls_c, cls_f = lib.level_classes(l - 1), lib.level_classes(l)
        uc, uf = us[l - 2], us[l - 1]
        cen_c = coords[l - 2].mean(axis=(2, 3, 4))
        blocks = coords[l - 1].reshape(-1, 8, 3, n, n, n).mean(axis=(3, 4, 5)).mean(axis=1)
        d = np.linalg.norm(cen_c[None, :, :] - blocks[:, None, :], axis=2)
        parent = d.argmin(axis=1)
        h = 1.0 / (ne * 2 ** (l - (L - 2)))          # element size of the coarse level
        assert np.all(d[np.arange(len(parent)), parent] < 0.1 * h) and len(set(parent.tolist())) == len(parent)
        tw_err = fr_err = 0.0
        for q, e in enumerate(parent):
            kids = uf[8 * q:8 * q + 8]
            kc = cls_f[8 * q:8 * q + 8]
            if cls_c[e] == 0:                  # twig: u^t = P u^a of its active children
                assert np.all(kc != 2)
                proj = sum(_t3(P[c >> 2], P[(c >> 1) & 1], P[c & 1], kids[c]) for c in range(8))
                tw_err = max(tw_err, np.abs(uc[e] - proj).max())
            else:                              # leaf with frozen children: u^f = I u^l
                assert cls_c[e] == 1 and np.all(kc == 2)
                for c in range(8):
                    fr_err = max(fr_err, np.abs(kids[c] - _t3(I[c >> 2], I[(c >> 1) & 1], I[c & 1], uc[e])).max())
        print('level', l, 'twig defect %.2e, frozen defect %.2e, scale %.2e' % (tw_err, fr_err, scale), flush=True)
        # the frozen update is exact after the last cycle; twigs follow their children up to the
        # solve's tolerance (measured 8e-14 and 3e-15 of the scale)
        assert fr_err <= 1e-12 * scale and tw_err <= 1e-8 * scale
    lib.close()
