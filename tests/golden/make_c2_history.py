"""Writes c2_curved_p7_history.json: the oracle's FAS-MG-SCG(3,2) history on the curved
32^3, p = 7 workload (16,777,216 DOF) and sampled element blocks of its final iterate.

Runs only the oracle (O1, the C/OpenMP version, which the numpy oracle pins element-wise on
small meshes) on the seeded synthetic input: 32^3 elements of [0,1]^3 under
x' = x + 0.1 sin(2 pi x) sin(2 pi y) sin(2 pi z) (every component), nodal f ~ U[-1,1] with
seed 2, u_D = 0, u_0 = 0, mu_star = 5, overlap 1, SCG smoothing with 3 + 2 steps, root SCG
to 1e-1 of its initial residual (at most 500 iterations), cycles until 1e-10.

    python tests/golden/make_c2_history.py [ne]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import o1                                    # noqa: E402
from oracle.gll import gll                               # noqa: E402
from paper_2608_14123_amd import workloads as W          # noqa: E402

SAMPLE_SEED = 12


def sample_elements(ne):
    E = ne ** 3
    fixed = [0, E - 1, (ne // 2) + ne * ((ne // 2) + ne * (ne // 2))]
    rnd = np.random.default_rng(SAMPLE_SEED).choice(E, 5, replace=False).tolist()
    return sorted(set(fixed + rnd))


def main(ne=32, p=7):
    V, nbr, bc, mp = W.curved_cube(ne)
    X = W.element_coords(V, gll(p)[0], mp)
    E, n3 = ne ** 3, (p + 1) ** 3
    t0 = time.time()
    fast = o1.O1(p, X, nbr, bc, m=1, mu_star=5.0)
    f = W.uniform_nodal(E * n3, 2)
    b = fast.rhs(f)
    t1 = time.time()
    u, hist, its = fast.solve(b, smoother='scg', ns1=3, ns2=2, root_maxit=500, root_rtol=0.1, max_cycles=30,
                              rtol=1e-10)
    t2 = time.time()
    els = sample_elements(ne)
    out = {
        'workload': 'curved_cube_%d^3_p%d_sine_bump_0.1' % (ne, p),
        'cycle': 'FAS-MG-SCG(3,2), overlap 1, mu_star 5, root SCG to 1e-1 (max 500), rtol 1e-10',
        'rhs': 'nodal f ~ U[-1,1] seed 2, u_D = 0, u_0 = 0',
        'oracle': 'O1 (C/OpenMP, FP64) with %d threads; set-up %.1f s, solve %.1f s' % (o1.threads(), t1 - t0,
                                                                                      t2 - t1),
        'n10': len(hist) - 1,
        'history': [float(h) for h in hist],
        'root_iterations': [int(i) for i in its],
        'sample_elements': els,
        'u_blocks': [[float(x) for x in u[e * n3:(e + 1) * n3]] for e in els],
        'u_max_abs': float(np.abs(u).max()),
    }
    name = 'c2_curved_p7_history.json' if ne == 32 else 'curved_%d_p%d_history.json' % (ne, p)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), name), 'w') as fh:
        json.dump(out, fh, indent=1)
    print(name, out['n10'], 'cycles', out['oracle'])


if __name__ == '__main__':
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 32)
