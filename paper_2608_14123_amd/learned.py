"""Training pipeline of the learned subdomain correction (drives the C ABI; no arithmetic here).

Pairs come from the method itself: plain FAS V-cycles run on seeded perturbed stretched
meshes; after selected cycles the finest-level residual r = b - A u is cut into subdomain
problems whose exact local solves are computed by `dgfas_learned_pairs`.  The network is
trained with `dgfas_mlp_train` (Adam, cosine learning-rate decay) and then judged against
the plain smoother on a held-out mesh by `dgfas_solve` with the fallback rule.
"""
import time

import numpy as np

from . import binding as B
from . import workloads as W


def center_classes(ne):
    """64 classes of centre elements of an ne^3 grid: (ex, ey, ez) = (ox, oy, oz) mod 4."""
    ex, ey, ez = np.meshgrid(np.arange(ne), np.arange(ne), np.arange(ne), indexing='ij')
    idx = ex + ne * (ey + ne * ez)
    out = []
    for oz in range(4):
        for oy in range(4):
            for ox in range(4):
                sel = (ex % 4 == ox) & (ey % 4 == oy) & (ez % 4 == oz)
                out.append(np.sort(idx[sel].ravel()).astype(np.int32))
    return out


def build_mesh(ne, seed, p=8, family='curved'):
    """family 'curved': unit cube under a seeded sine-bump map (seed None: the reference map);
    'stretched': [0,1]^2 x [0,100] with perturbed vertices."""
    if family == 'stretched':
        V, nbr, bc = W.stretched_perturbed(ne, seed=seed)
        X = W.element_coords(V, B.gll(p)[0])
    else:
        nbr, bc = W.box_topology(ne, ne, ne)
        mp = W.sine_bump_map if seed is None else W.seeded_bump_map(seed)
        X = W.element_coords(W.box_vertices(ne, ne, ne), B.gll(p)[0], mp)
    return X, nbr, bc


def solver_for(ne, seed, p=8, family='curved', **opts):
    X, nbr, bc = build_mesh(ne, seed, p, family)
    o = B.default_options(**opts)
    return B.Solver(np.full(ne ** 3, p, np.int32), X, nbr, bc, o)


def generate_pairs(torch, ne, mesh_seeds, rhs_seeds, stages, p=8, opts=None, family='curved', log=print):
    """Returns device tensors (X [n][ns^3+9], T [n][ns^3]) and statistics."""
    opts = dict(smoother=B.SCG, ns1=3, ns2=2, mu_star=5.0, root_rtol=1e-1) if opts is None else opts
    classes = center_classes(ne)
    ns = p + 3
    nt = ns ** 3
    Xs, Ts = [], []
    iters = []
    t0 = time.perf_counter()
    for ms in mesh_seeds:
        lib = solver_for(ne, ms, p, family, **opts)
        n = lib.level_info(lib.n_levels)[1]
        L = lib.n_levels
        for rs in rhs_seeds:
            f = torch.from_numpy(W.uniform_nodal(n, rs)).cuda()
            b = torch.empty_like(f)
            lib.rhs(f, b)
            u = torch.zeros_like(b)
            r = torch.empty_like(b)
            done = 0
            for stage in sorted(stages):
                while done < stage:
                    lib.vcycle(u, b)
                    done += 1
                lib.residual(L, u, b, r)
                for cls in classes:
                    X = torch.empty((len(cls), nt + 9), dtype=torch.float32, device='cuda')
                    T = torch.empty((len(cls), nt), dtype=torch.float32, device='cuda')
                    iters.append(B.learned_pairs(lib, r, cls, X, T))
                    Xs.append(X)
                    Ts.append(T)
        lib.close()
        log('mesh seed %d done: %d pairs, %.1fs' % (ms, sum(x.shape[0] for x in Xs), time.perf_counter() - t0))
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    return X, T, {'pairs': int(X.shape[0]), 'pcg_iters_mean': float(np.mean(iters)),
                  'seconds': time.perf_counter() - t0}


def train(torch, X, T, hidden=256, batch=4096, epochs=4, lr0=1e-3, lr_min=1e-5, seed=5, log=print):
    n = X.shape[0]
    g = torch.Generator(device='cuda')
    g.manual_seed(seed)
    perm = torch.randperm(n, device='cuda', generator=g)
    Xp = X[perm].contiguous()
    Tp = T[perm].contiguous()
    net = B.Mlp(X.shape[1], hidden, T.shape[1], seed=seed)
    steps = max(1, epochs * n // batch)
    t0 = time.perf_counter()
    losses = net.train(Xp, Tp, batch=batch, steps=steps, lr0=lr0, lr_min=lr_min, total_steps=steps)
    torch.cuda.synchronize()
    log('trained %d steps in %.1fs: loss %.3e -> %.3e' % (steps, time.perf_counter() - t0, losses[0], losses[-1]))
    return net, {'steps': steps, 'loss_first': float(losses[0]), 'loss_last': float(losses[-1]),
                 'seconds': time.perf_counter() - t0, 'target_mean_square': float((T.double() ** 2).mean())}


def evaluate(torch, net, ne, mesh_seed, rhs_seed, p=8, opts=None, max_cycles=60, rtol=1e-10, family='curved'):
    """n10 / t10 of the plain and the learned smoother on one held-out mesh."""
    opts = dict(smoother=B.SCG, ns1=3, ns2=2, mu_star=5.0, root_rtol=1e-1) if opts is None else opts
    lib = solver_for(ne, mesh_seed, p, family, **opts)
    n = lib.level_info(lib.n_levels)[1]
    f = torch.from_numpy(W.uniform_nodal(n, rhs_seed)).cuda()
    b = torch.empty_like(f)
    lib.rhs(f, b)
    out = {}
    for name, on, judge in (('plain', False, True), ('learned', True, True), ('learned_unjudged', True, False)):
        B.set_learned(lib, net if on else None, on, judge)
        u = torch.zeros_like(b)
        B.solve_status(lib, u, b, 2, rtol)          # warm-up (and the plain reference factor)
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            hist, code = B.solve_status(lib, u, b, max_cycles, rtol)
        except B.DgfasError as e:            # the plain smoother itself may diverge
            hist, code = np.array([1.0, np.inf]), e.code
        torch.cuda.synchronize()
        out[name] = {'n10': len(hist) - 1, 't10_s': time.perf_counter() - t0, 'final_rho': float(hist[-1]),
                     'status': int(code), 'hist': [float(h) for h in hist]}
    B.set_learned(lib, None, False)
    lib.close()
    return out


def main(argv=None):
    """The learned-correction experiment on seeded meshes of one family: pairs from plain
    FAS-MG-SCG cycles on the training meshes (the initial residual of one right-hand side),
    training, then plain vs learned on the held-out mesh.  Prints one JSON line per stage."""
    import argparse, json
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument('--ne', type=int, default=48)
    ap.add_argument('--family', default='stretched', choices=['stretched', 'curved'])
    ap.add_argument('--train-seeds', default='40-47', help='mesh seeds of the training pairs, a-b')
    ap.add_argument('--eval-seed', type=int, default=4, help='held-out mesh seed')
    ap.add_argument('--ns1', type=int, default=12)
    ap.add_argument('--ns2', type=int, default=4)
    ap.add_argument('--epochs', type=int, default=8)
    ap.add_argument('--max-cycles', type=int, default=40)
    args = ap.parse_args(argv)
    import torch
    a, b = (int(x) for x in args.train_seeds.split('-'))
    opts = dict(smoother=B.SCG, ns1=args.ns1, ns2=args.ns2, mu_star=5.0, root_rtol=1e-1)
    log = lambda s: print(s, flush=True)
    X, T, st = generate_pairs(torch, args.ne, list(range(a, b + 1)), [4100], [0], opts=opts, family=args.family,
                              log=log)
    print(json.dumps({'pairs': st}), flush=True)
    net, tr = train(torch, X, T, epochs=args.epochs, batch=4096, log=log)
    print(json.dumps({'training': tr}), flush=True)
    del X, T
    torch.cuda.empty_cache()
    ev = evaluate(torch, net, args.ne, args.eval_seed, 4000, opts=opts, max_cycles=args.max_cycles,
                  family=args.family)
    for k, v in ev.items():
        print(json.dumps({k: v}), flush=True)
    net.close()


if __name__ == '__main__':
    main()
