"""Benchmark: the Schwarz sweep and FAS V-cycles on the curved 32^3, p = 7 workload.

One step = one FAS-MG-SCG(3,2) V-cycle (Alg. 2 with Alg. 6 smoothing, p-levels
7 -> 3 -> 1, SCG root solve) over the 16.8M-DOF curvilinear mesh (sine-bump
map, mu_star = 5), FP64, inputs resident in HBM.  Prints one JSON line.
`value` is the FP64 WAS sweep throughput on the finest level (residual r = g - A u,
Schwarz application and update u += B r; Alg. 5), median of per-call event timings:
DOF / sweep time.  Beside it: the same sweep in FP32 and BF16, the Schwarz application and
one SCG iteration, the time to 1e-10 of the plain, reduced-precision, graph and FMG
forms with their HBM-roofline time, and the C/OpenMP oracle on the host's cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0     # dense BF16 matrix-core peak
# HBM bytes of one residual launch of the operator kernel at 32^3, p = 7 from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs, scaled by a 1 GiB copy (profiles/c2_curved_p7_hbm_traffic_pmc.md);
# valid only for the kernel source it was measured on.
OPERATOR_TRAFFIC = {'sha256_prefix': '61deb11c012bf61b', 'bytes': 1.670e9, 'ne': 32, 'p': 7}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=10)
    ap.add_argument('--warmup', type=int, default=2)
    ap.add_argument('--ne', type=int, default=32)
    ap.add_argument('--p', type=int, default=7)
    ap.add_argument('--reps', type=int, default=20, help='repetitions of the isolated kernel timings')
    ap.add_argument('--no-cpu', action='store_true', help='skip the oracle cpu_baseline leg')
    ap.add_argument('--no-t10', action='store_true', help='skip the time-to-tolerance solves')
    ap.add_argument('--calib-copy', action='store_true', help='also run a plain copy kernel (PMC calibration)')
    ap.add_argument('--order', default='natural', choices=['natural', 'morton'],
                    help='curved workload: element order of the sweep kernels (the h-coarsening solves keep '
                         'the natural order, the only one the library takes with h-levels)')
    ap.add_argument('--workload', default='curved', choices=['curved', 'front', 'stretched', 'mlp', 'local',
                                                              'diamond'],
                    help='curved: the 32^3 p = 7 headline workload; front: the hp front (27^3, degrees 2..8); '
                         'stretched: 48^3, p = 8, aspect 1:100, 16 right-hand sides; mlp: the learned '
                         'correction network at its p = 8 size; local: local refinement, 16^3 p = 7 with two '
                         'nested zones; diamond: the periodic cube of extruded diamond cells (irregular edges '
                         'and vertices) at p = 4 and 8')
    ap.add_argument('--cycles', type=int, default=40, help='stretched workload: largest V-cycle count of a solve')
    return ap.parse_args()


def build_workload(ne, p, xi):
    from paper_2608_14123_amd import workloads as W
    V, nbr, bc, mp = W.curved_cube(ne)
    X = W.element_coords(V, xi, mp)
    return X, nbr, bc


def host_info():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = 'unknown'
    try:
        with open('/proc/cpuinfo') as fh:
            for line in fh:
                if line.startswith('model name'):
                    model = line.split(':', 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count()
    return {'cpu_model': model, 'nproc': os.cpu_count(), 'allowed_cpus': allowed}


def cpu_baseline(ne, p, n10_c2, reps=5):
    """The C/OpenMP FP64 oracle (O1) on this host's cores: medians of `reps` timed runs after a
    warm-up of one WAS sweep (residual, Schwarz, update), one Schwarz application and one
    operator application on the full curved 32^3, p = 7 mesh, one FAS-MG-SCG(3,2) cycle (whose
    time times the GPU's cycle count estimates the oracle's t10 there), and the full solve of
    the 4^3, p = 4 unit-cube case."""
    info = host_info()          # before the OpenMP runtime binds this thread to one CPU
    os.environ.setdefault('OMP_PROC_BIND', 'close')
    from oracle import o1
    from oracle.gll import gll as ogll
    from paper_2608_14123_amd import workloads as W

    def med(fn):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    V, nbr, bc, mp = W.curved_cube(ne)
    X = W.element_coords(V, ogll(p)[0], mp)
    t0 = time.perf_counter()
    fast = o1.O1(p, X, nbr, bc, m=1, mu_star=5.0)
    setup = time.perf_counter() - t0
    L = fast.n_levels
    nd = fast.ndof[L]
    g = fast.rhs(W.uniform_nodal(nd, 2))
    u = W.uniform_nodal(nd, 4)
    s_sweep = med(lambda: fast.smooth(L, u, g, 1, 'was'))
    s_sz = med(lambda: fast.schwarz(L, g))
    s_op = med(lambda: fast.apply(L, u))
    t0 = time.perf_counter()
    fast.solve(g, smoother='scg', ns1=3, ns2=2, root_rtol=0.1, max_cycles=1, rtol=0.0)
    s_cycle = time.perf_counter() - t0
    fast.close()
    # C1: 4^3 unit cubes, p = 4, f = 3 pi^2 sin sin sin, FAS-MG-WAS(2,2) to 1e-10
    Vc, nbrc, bcc = W.cartesian_unit_cube(4)
    Xc = W.element_coords(Vc, ogll(4)[0])
    c1 = o1.O1(4, Xc, nbrc, bcc)
    bc1 = c1.rhs((3 * np.pi ** 2 * W.sine_solution(Xc)).ravel())
    t0 = time.perf_counter()
    _, h1, _ = c1.solve(bc1, smoother='was', ns1=2, ns2=2, max_cycles=30, rtol=1e-10)
    t10_c1 = time.perf_counter() - t0
    c1.close()
    out = {'value': round(nd / s_sweep / 1e9, 4), 'unit': 'GDOF/s', 'cores': o1.threads(), 'kind': 'oracle',
           'sample': 'O1 (C/OpenMP, FP64) on the full %d^3, p = %d curved mesh (%d DOF): median of %d WAS sweeps '
                     '(residual + Schwarz + update) after one warm-up; set-up %.1f s' % (ne, p, nd, reps, setup),
           'schwarz_gdofs': round(nd / s_sz / 1e9, 4), 'operator_gdofs': round(nd / s_op / 1e9, 4),
           'c2_cycle_s': round(s_cycle, 3),
           'c2_t10_estimate_s': round(s_cycle * n10_c2, 2),
           'c2_t10_estimate_basis': 'one FAS-MG-SCG(3,2) cycle timed, times the %d cycles to 1e-10' % n10_c2,
           'c1_t10_s': round(t10_c1, 4), 'c1_n10': len(h1) - 1, 'omp_proc_bind': os.environ.get('OMP_PROC_BIND')}
    out.update(info)
    return out


def front_bench(args, torch, B):
    """The hp front workload (27^3 unit cubes, degrees 2..8 from the front distance, 3,217,284
    DOF, alpha = 50): per-degree launches, one-launch batches (a workgroup per tile, or a
    persistent grid striding through the tiles), and autotuned launches with the cycle legs
    replayed from HIP graphs.  Prints one JSON line."""
    from paper_2608_14123_amd import workloads as W
    ne = 27
    degs, X, nbr, bc, f_host, uD_host = W.front_workload(ne, lambda p: B.gll(p)[0])
    flat = np.concatenate([x.ravel() for x in X])
    ndof = int(((degs.astype(np.int64) + 1) ** 3).sum())
    stream = torch.cuda.current_stream()
    cyc = dict(smoother=B.SCG, ns1=3, ns2=2, root_rtol=0.1)
    f = torch.from_numpy(f_host).cuda()
    uD = torch.from_numpy(uD_host).cuda()
    modes = [('per_degree', dict(batch=B.BATCH_PER_DEGREE)), ('one_launch', dict(batch=B.BATCH_ONE_LAUNCH)),
             ('persistent', dict(batch=B.BATCH_PERSISTENT)),
             ('tuned_graph', dict(batch=B.BATCH_TUNED, graph=1)),
             # a fixed 16-iteration root solve: every cycle is one captured graph
             ('tuned_whole_cycle_graph_fixed_root16', dict(batch=B.BATCH_TUNED, graph=1, root_max_iter=16))]
    out_modes = {}
    tune = None

    def timed(fn, reps):
        fn()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / reps

    for name, extra in modes:
        for prec in ('fp64', 'fp32'):
            if prec == 'fp32' and name != 'tuned_graph':
                continue
            kw = dict(cyc, **extra)
            if name.endswith('fixed_root16'):
                kw['root_rtol'] = 0.0
            o = B.default_options(precision=B.FP64 if prec == 'fp64' else B.FP32, **kw)
            lib = B.Solver(degs, flat, nbr, bc, o, stream=stream.cuda_stream)
            L = lib.n_levels
            if name.startswith('tuned') and tune is None:
                tune = lib.autotune(None, reps=10)
            elif name.startswith('tuned'):
                lib.autotune(None, reps=10)
            b = torch.empty_like(f)
            lib.rhs(f, b, uD=uD)
            u = torch.zeros_like(b)
            rec = {}
            if prec == 'fp64':
                g = torch.from_numpy(W.uniform_nodal(ndof, 3)).cuda()
                r = torch.empty_like(g)
                uu = torch.from_numpy(W.uniform_nodal(ndof, 4)).cuda()
                rec['residual_ms'] = round(timed(lambda: lib.residual(L, uu, g, r), args.reps), 4)
                rec['schwarz_ms'] = round(timed(lambda: lib.schwarz(L, g, r), args.reps), 4)
                ms_sweep = timed(lambda: lib.smooth(L, uu, g, 1), args.reps)
                rec['residual_plus_scg_iteration_ms'] = round(ms_sweep, 4)
                rec['sweep_gdofs'] = round(ndof / (ms_sweep * 1e-3) / 1e9, 3)
                lib.solve(u.zero_(), b, max_cycles=args.warmup, rtol=0.0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lib.solve(u.zero_(), b, max_cycles=args.steps, rtol=0.0)
                torch.cuda.synchronize()
                rec['ms_per_cycle'] = round((time.perf_counter() - t0) * 1e3 / args.steps, 4)
            hist, ok = lib.solve(u.zero_(), b, max_cycles=40, rtol=1e-10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hist, ok = lib.solve(u.zero_(), b, max_cycles=40, rtol=1e-10)
            torch.cuda.synchronize()
            rec['t10_s'] = round(time.perf_counter() - t0, 4)
            rec['n10'] = len(hist) - 1
            rec['converged'] = bool(ok)
            lib.close()
            out_modes[name if prec == 'fp64' else name + '_fp32_smoother'] = rec
            print(name, prec, rec, file=sys.stderr, flush=True)
    best = out_modes['tuned_graph']
    sweeps = cyc['ns1'] + cyc['ns2']
    bytes_res = 48.0 * ndof
    ach = bytes_res / (best['residual_ms'] * 1e-3) / 1e9
    levels = ['%d' % int(x) for x in np.unique(degs)]
    out = {
        'metric': 'GDOF/s per Schwarz sweep; time-to-1e-10 residual, plain FP64 vs mixed/learned',
        'value': round(ndof * sweeps / (best['ms_per_cycle'] * 1e-3) / 1e9, 3), 'unit': 'GDOF/s', 'n_gpus': 1,
        'steps': args.steps, 'warmup': args.warmup, 'ms_per_step': best['ms_per_cycle'], 'higher_is_better': True,
        'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f64', 'data': 'synthetic',
        'config': {'workload': 'hp_front_27^3_degrees_2to8_alpha50', 'n_dof': ndof,
                   'degrees': dict(zip(levels, np.unique(degs, return_counts=True)[1].tolist())),
                   'cycle': 'FAS-MG-SCG(3,2), per-element p-coarsening, root SCG to 1e-1', 'overlap': 1,
                   'mu_star': 2.0},
        'roofline': {'kernel': 'operator stage (residual), tuned launches', 'bound': 'hbm', 'achieved': round(ach, 1),
                     'peak': HBM_PEAK_GBS, 'unit': 'GB/s', 'frac': round(ach / HBM_PEAK_GBS, 4), 'traffic': None},
        'modes': out_modes,
        'autotune_ms': {'level%d' % (l + 1): {st: tune[l][k].round(4).tolist()
                                              for k, st in enumerate(('operator', 'solve', 'add'))}
                        for l in range(tune.shape[0]) if tune[l].any()},
    }
    print(json.dumps(out))


def local_bench(args, torch, B):
    """Local refinement (Sec. 3.1, 3.3): the curved 16^3, p = 7 cube with two nested zones refined
    around its centre (radii 0.3 and 0.15 of the unit cube), a Gaussian source there, solved to a
    composite residual of 1e-10: FAS-MG-SCG(3,2) on the headline's sine-bump map (amplitude 0.1,
    mu_star = 5; WAS(2,2) diverges there, as without refinement), and FAS-MG-WAS(2,2) on a milder
    map (amplitude 0.03, mu_star = 2), each without and with the FMG start-up.  Reports the active DOF per level, n10, t10, the V-cycle time
    and the finest level's operator over its active elements."""
    from paper_2608_14123_amd import workloads as W
    ne, p = 16, 7
    zones = [((0.5, 0.5, 0.5), 0.3), ((0.5, 0.5, 0.5), 0.15)]
    refine = W.local_refine_lists(ne, zones)
    xi = B.gll(p)[0]
    V, nbr, bc, mp = W.curved_cube(ne)
    stream = torch.cuda.current_stream()
    modes = {}
    structure = None
    for name, amp, mu, kw in (('bump0.1_scg32', 0.1, 5.0, dict(smoother=B.SCG, ns1=3, ns2=2)),
                              ('bump0.1_scg32_fmg', 0.1, 5.0, dict(smoother=B.SCG, ns1=3, ns2=2, start=B.START_FMG)),
                              ('bump0.03_was22', 0.03, 2.0, dict(smoother=B.WAS, ns1=2, ns2=2)),
                              ('bump0.03_was22_fmg', 0.03, 2.0, dict(smoother=B.WAS, ns1=2, ns2=2,
                                                                   start=B.START_FMG))):
        X = W.element_coords(V, xi, lambda Y: mp(Y, amp))
        t0 = time.perf_counter()
        lib = B.Solver(np.full(ne ** 3, p, np.int32), X, nbr, bc,
                       B.default_options(local_steps=len(refine), mu_star=mu, root_rtol=0.1, **kw),
                       stream=stream.cuda_stream, refine=refine)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        L = lib.n_levels
        n3 = (p + 1) ** 3
        bl = []
        levels = []
        for l in range(1, L + 1):
            cls = lib.level_classes(l)
            Xl = lib.level_coords(l)
            t = torch.empty(Xl.size // 3, dtype=torch.float64, device='cuda')
            lib.level_rhs(l, torch.from_numpy(W.gaussian_source(Xl).ravel()).cuda(), t, uD=torch.zeros_like(t))
            bl.append(t)
            if l < L:
                lib.set_level_rhs(l, t)
            levels.append({'elements': int(len(cls)), 'twig': int((cls == 0).sum()), 'leaf': int((cls == 1).sum()),
                           'frozen': int((cls == 2).sum()), 'active_dof': int((cls != 2).sum()) * n3})
        structure = levels
        u = torch.zeros_like(bl[-1])
        lib.solve(u, bl[-1], max_cycles=args.warmup, rtol=0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lib.solve(u.zero_(), bl[-1], max_cycles=args.steps, rtol=0.0)
        torch.cuda.synchronize()
        ms_cycle = (time.perf_counter() - t0) * 1e3 / args.steps
        t0 = time.perf_counter()
        try:
            hist, ok = lib.solve(u.zero_(), bl[-1], max_cycles=40, rtol=1e-10)
        except B.DgfasError as ex:          # a diverging cycle is recorded, not fatal
            hist, ok = [float('nan')], False
            print(name, 'solve failed:', ex, file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t10 = time.perf_counter() - t0
        # the finest level's operator over its active elements
        g = torch.from_numpy(W.uniform_nodal(bl[-1].numel(), 3)).cuda()
        r = torch.zeros_like(g)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        lib.residual(L, u, g, r)
        ev0.record(stream)
        for _ in range(args.reps):
            lib.residual(L, u, g, r)
        ev1.record(stream)
        ev1.synchronize()
        op_ms = ev0.elapsed_time(ev1) / args.reps
        modes[name] = {'setup_s': round(setup_s, 3), 'ms_per_cycle': round(ms_cycle, 3), 'n10': len(hist) - 1,
                       't10_s': round(t10, 4), 'converged': bool(ok), 'hist': ['%.3e' % h for h in hist],
                       'finest_operator_ms': round(op_ms, 4)}
        print(name, modes[name], file=sys.stderr, flush=True)
        lib.close()
    active = sum(lv['active_dof'] for lv in structure)
    fin = structure[-1]['active_dof']
    best = modes['bump0.1_scg32']
    sweeps = 5
    ach = 48.0 * fin / (best['finest_operator_ms'] * 1e-3) / 1e9
    out = {
        'metric': 'GDOF/s per Schwarz sweep; time-to-1e-10 residual, plain FP64 vs mixed/learned',
        'value': round(active * sweeps / (best['ms_per_cycle'] * 1e-3) / 1e9, 3), 'unit': 'GDOF/s', 'n_gpus': 1,
        'steps': args.steps, 'warmup': args.warmup, 'ms_per_step': best['ms_per_cycle'], 'higher_is_better': True,
        'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f64', 'data': 'synthetic',
        'config': {'workload': 'local_refinement_curved_16^3_p7_zones_0.3_0.15', 'active_dof': active,
                   'uniform_equivalent_dof': (4 * ne) ** 3 * (p + 1) ** 3, 'levels': structure,
                   'value': 'active DOF of all levels x 5 sweeps over the FAS-MG-SCG(3,2) cycle time',
                   'rhs': 'exp(-50 |x - c|^2), u_D = 0', 'mu_star': 5.0, 'root': 'SCG to 1e-1'},
        'roofline': {'kernel': 'sipg_apply_kernel<8,double> over the finest level\'s active elements', 'bound': 'hbm',
                     'achieved': round(ach, 1), 'peak': HBM_PEAK_GBS, 'unit': 'GB/s',
                     'frac': round(ach / HBM_PEAK_GBS, 4), 'traffic': None},
        'modes': modes,
    }
    print(json.dumps(out))


def diamond_bench(args, torch, B):
    """The irregular mesh of Sec. 6.2.4: the periodic cube [0, 2 pi)^3 of the Cartesian study
    (kappa = 0, semidefinite, null-space projection in the root SCG) built from nc x nc diamond
    cells (a central quadrilateral and four trapezoids; cell corners shared by 8 elements, the
    diamond's corners by 3) extruded into layers, every element's local axes turned at random.
    About 32^3 elements' worth of DOF at p = 4 (nc = 16, 24 layers) and 16^3 at p = 8 (nc = 8,
    12 layers), as the Cartesian study sizes its meshes.  Per mode: set-up, V-cycle time, n10 and
    t10 from u = 0 on random zero-mean data; per degree the unstructured operator and Schwarz
    application (medians of per-call HIP-event timings) and the WAS sweep they make."""
    from paper_2608_14123_amd import workloads as W
    stream = torch.cuda.current_stream()
    sizes = {4: (16, 24), 8: (8, 12)}
    modes, kernels, struct = {}, {}, {}
    for p, (nc, layers) in sizes.items():
        t0 = time.perf_counter()
        X = W.diamond_coords(nc, layers, B.gll(p)[0], length=2 * np.pi, height=2 * np.pi, shift_seed=1, rot_seed=2)
        nbr, nf, no, bc = W.face_connectivity(X, period=2 * np.pi)
        mesh_s = time.perf_counter() - t0
        E, n3 = len(X), (p + 1) ** 3
        ndof = E * n3
        b = W.uniform_nodal(ndof, 11)
        b -= b.mean()
        bd = torch.from_numpy(b).cuda()
        for name, kw in (('scg84', dict(smoother=B.SCG, ns1=8, ns2=4)),
                         ('scg84_fmg', dict(smoother=B.SCG, ns1=8, ns2=4, start=B.START_FMG)),
                         ('was22', dict(smoother=B.WAS, ns1=2, ns2=2))):
            t0 = time.perf_counter()
            lib = B.Solver(np.full(E, p, np.int32), X, nbr, bc,
                           B.default_options(kappa=0.0, null_space=1, mu_star=5.0, root_rtol=0.1, **kw),
                           stream=stream.cuda_stream, nbr_face=nf, nbr_orient=no)
            torch.cuda.synchronize()
            setup_s = time.perf_counter() - t0
            L = lib.n_levels
            if p not in struct:
                struct[p] = {'cells': nc, 'layers': layers, 'elements': E, 'dof': ndof, 'mesh_build_s': round(mesh_s, 2),
                             'blocks_finest': dict(zip(('own', 'face', 'mapped', 'zero_filled', 'merged'),
                                                       lib.level_blocks(L).tolist()))}
            u = torch.zeros_like(bd)
            cycles = 40
            if name != 'was22':
                lib.solve(u, bd, max_cycles=args.warmup, rtol=0.0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lib.solve(u.zero_(), bd, max_cycles=args.steps, rtol=0.0)
                torch.cuda.synchronize()
                ms_cycle = (time.perf_counter() - t0) * 1e3 / args.steps
            else:
                ms_cycle, cycles = None, 4
            t0 = time.perf_counter()
            try:
                hist, ok = lib.solve(u.zero_(), bd, max_cycles=cycles, rtol=1e-10)
            except B.DgfasError as ex:          # a diverging cycle is recorded, not fatal
                hist, ok = [float('nan')], False
                print(name, 'solve failed:', ex, file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            t10 = time.perf_counter() - t0
            modes['p%d_%s' % (p, name)] = {'setup_s': round(setup_s, 3), 'ms_per_cycle': None if ms_cycle is None else
                                           round(ms_cycle, 3), 'n10': len(hist) - 1 if ok else None,
                                           't10_s': round(t10, 4) if ok else None, 'converged': bool(ok),
                                           'hist': ['%.3e' % h for h in hist]}
            print(p, name, modes['p%d_%s' % (p, name)], file=sys.stderr, flush=True)
            if name == 'scg84':
                # the finest level's operator and Schwarz application, medians of per-call timings
                g = torch.from_numpy(W.uniform_nodal(ndof, 3)).cuda()
                r, z = torch.zeros_like(g), torch.zeros_like(g)
                ts = {'operator': [], 'schwarz': []}
                for _ in range(2):
                    lib.residual(L, u, g, r)
                    lib.schwarz(L, r, z)
                for _ in range(args.reps):
                    for key, fn in (('operator', lambda: lib.residual(L, u, g, r)), ('schwarz', lambda: lib.schwarz(L, r, z))):
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                        fn()
                        e1.record(stream)
                        e1.synchronize()
                        ts[key].append(e0.elapsed_time(e1))
                op_ms, sz_ms = float(np.median(ts['operator'])), float(np.median(ts['schwarz']))
                kernels[p] = {'operator_ms': round(op_ms, 4), 'operator_gdofs': round(ndof / op_ms / 1e6, 2),
                              'operator_frac_48B': round(48.0 * ndof / (op_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                              'schwarz_ms': round(sz_ms, 4), 'schwarz_gdofs': round(ndof / sz_ms / 1e6, 2),
                              'was_sweep_gdofs': round(ndof / (op_ms + sz_ms) / 1e6, 2)}
                print(p, kernels[p], file=sys.stderr, flush=True)
            lib.close()
    k4 = kernels[4]
    out = {
        'metric': 'GDOF/s per Schwarz sweep; time-to-1e-10 residual, plain FP64 vs mixed/learned',
        'value': k4['was_sweep_gdofs'], 'unit': 'GDOF/s', 'n_gpus': 1, 'steps': args.steps, 'warmup': args.warmup,
        'ms_per_step': modes['p4_scg84']['ms_per_cycle'], 'higher_is_better': True, 'scaling': 'weak',
        'vs_baseline': None, 'dtype': 'f64', 'data': 'synthetic',
        'config': {'workload': 'diamond_periodic_2pi^3', 'sizes': {'p%d' % k: v for k, v in struct.items()},
                   'value': 'p = 4 WAS sweep (unstructured residual + Schwarz application), DOF / median time',
                   'rhs': 'uniform random, zero mean', 'kappa': 0.0, 'mu_star': 5.0, 'root': 'SCG to 1e-1'},
        'roofline': {'kernel': 'sipg_apply_kernel<5,double,orient> (residual, p = 4)', 'bound': 'hbm',
                     'achieved': round(k4['operator_frac_48B'] * HBM_PEAK_GBS, 1), 'peak': HBM_PEAK_GBS, 'unit': 'GB/s',
                     'frac': k4['operator_frac_48B'], 'traffic': None},
        'kernels': {'p%d' % k: v for k, v in kernels.items()},
        'modes': modes,
    }
    print(json.dumps(out))


def mlp_bench(args, torch, B):
    """The learned correction's network at the size of the p = 8, m = 1 subdomain tile: 1340 -> 256
    -> 256 -> 1331, batch 4096 (BF16 weights, FP32 accumulation on the matrix cores).  Times the
    forward pass (three GEMMs with bias and ReLU epilogues) and one forward + backward pass
    (eight GEMMs, the MSE gradient, ReLU derivatives and column sums) as medians of per-call
    event timings, and reports the GEMM flops over them against the BF16 MFMA peak."""
    n_in, h, n_out, rows = 1340, 256, 1331, 4096
    stream = torch.cuda.current_stream()
    net = B.Mlp(n_in, h, n_out, seed=5, stream=stream.cuda_stream)
    g = torch.Generator(device='cpu').manual_seed(7)
    X = torch.rand(rows, n_in, generator=g).cuda() - 0.5
    T = (torch.rand(rows, n_out, generator=g).cuda() - 0.5) * 0.1
    Y = torch.empty(rows, n_out, device='cuda')
    grad = torch.empty(net.n_params, device='cuda')

    def med_ms(fn, reps):
        fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in evs:
            e0.record(stream)
            fn()
            e1.record(stream)
        evs[-1][1].synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))

    ms_fwd = med_ms(lambda: net.forward(X, Y), args.reps)
    ms_grad = med_ms(lambda: net.gradient(X, T, grad), args.reps)
    flops_fwd = 2.0 * rows * (n_in * h + h * h + h * n_out)
    # backward: dW3 and dH2 (h out), dW2 and dH1 (h h), dW1 (n_in h); no gradient of the input
    flops_bwd = 2.0 * rows * (2 * h * n_out + 2 * h * h + n_in * h)
    tf_fwd = flops_fwd / (ms_fwd * 1e-3) / 1e12
    tf_grad = (flops_fwd + flops_bwd) / (ms_grad * 1e-3) / 1e12
    net.close()
    peak = BF16_PEAK_TFLOPS
    out = {
        'metric': 'GDOF/s per Schwarz sweep; time-to-1e-10 residual, plain FP64 vs mixed/learned',
        'value': round(tf_grad, 3), 'unit': 'TFLOP/s', 'n_gpus': 1, 'steps': args.reps, 'warmup': 1,
        'ms_per_step': round(ms_grad, 4), 'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None,
        'dtype': 'bf16', 'data': 'synthetic',
        'config': {'workload': 'learned_correction_mlp_1340_256_256_1331_batch4096',
                   'value': 'GEMM flops of one forward + backward pass over its median time'},
        'roofline': {'kernel': 'gemm_bf16_kernel (forward + backward)', 'bound': 'mfma', 'achieved': round(tf_grad, 3),
                     'peak': peak, 'unit': 'TFLOP/s', 'frac': round(tf_grad / peak, 5), 'traffic': None},
        'forward_ms': round(ms_fwd, 4), 'forward_tflops': round(tf_fwd, 3),
        'forward_backward_ms': round(ms_grad, 4),
    }
    print(json.dumps(out))


def stretched_bench(args, torch, B):
    """The anisotropic stress workload: 48^3 elements on [0,1]^2 x [0,100] (aspect 1:100),
    interior vertices perturbed by U[-0.2, 0.2] h_min (seed 4), p = 8 (80,621,568 DOF), 16
    right-hand sides (nodal U[-1,1], seeds 4000..4015) in one batch, FAS-MG-SCG(12,4) with the
    overlap of delta = 0.24.  Reports the Schwarz application and one SCG iteration over all 16
    right-hand sides, and the time to 1e-10 (every right-hand side) with FP64 and FP32
    smoothers, and with the FP32 smoother after the FMG start-up (t10 includes it).  Prints one
    JSON line."""
    from paper_2608_14123_amd import workloads as W
    ne, p, R = 48, 8, 16
    E = ne ** 3
    V, nbr, bc = W.stretched_perturbed(ne, seed=4)
    X = W.element_coords(V, B.gll(p)[0])
    ndof = E * (p + 1) ** 3
    stream = torch.cuda.current_stream()
    f = torch.empty(R * ndof, dtype=torch.float64, device='cuda')
    for k in range(R):
        f[k * ndof:(k + 1) * ndof].copy_(torch.from_numpy(W.uniform_nodal(ndof, 4000 + k)))
    # the paper's overlap for its aspect-ratio tests, delta = 0.24: m = 3 at p = 8, 2 at p = 4
    cyc = dict(smoother=B.SCG, ns1=12, ns2=4, mu_star=5.0, root_rtol=0.1, n_rhs=R, overlap=-1, delta=0.24)

    def timed(fn, reps):
        fn()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / reps

    modes = {}
    # (the matrix-core FD tile takes overlap 1 only; at m = 3 the FP32 solves run on the vector unit)
    for prec in ('fp64', 'fp32', 'fp32_fmg'):
        o = B.default_options(precision=B.FP64 if prec == 'fp64' else B.FP32,
                              start=B.START_FMG if prec.endswith('fmg') else B.START_NONE, **cyc)
        t0 = time.perf_counter()
        lib = B.Solver(np.full(E, p, np.int32), X, nbr, bc, o, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        rec = {'setup_s': round(time.perf_counter() - t0, 3)}
        L = lib.n_levels
        b = torch.empty_like(f)
        lib.rhs(f, b)
        if prec == 'fp64':
            z = torch.empty_like(f)
            ms_sz = timed(lambda: lib.schwarz(L, b, z), max(2, args.reps // 4))
            del z
            u = torch.zeros_like(f)
            ms1 = timed(lambda: lib.smooth(L, u, b, 1), 2)
            ms3 = timed(lambda: lib.smooth(L, u, b, 3), 2)
            rec['schwarz_gdofs_all_rhs'] = round(R * ndof / (ms_sz * 1e-3) / 1e9, 3)
            rec['scg_iteration_ms'] = round((ms3 - ms1) / 2, 3)
            rec['scg_iteration_gdofs_all_rhs'] = round(R * ndof / ((ms3 - ms1) / 2 * 1e-3) / 1e9, 3)
            del u
        u = torch.zeros_like(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist, ok = lib.solve(u, b, max_cycles=args.cycles, rtol=1e-10)
        torch.cuda.synchronize()
        rec['t10_s'] = round(time.perf_counter() - t0, 3)
        rec['n10'] = len(hist) - 1
        rec['s_per_cycle'] = round(rec['t10_s'] / max(1, len(hist) - 1), 4)
        rec['converged_1e-10'] = bool(ok)
        rec['hist'] = ['%.3e' % h for h in hist]
        print(prec, rec, file=sys.stderr, flush=True)
        modes[prec] = rec
        del u, b
        lib.close()
    out = {
        'metric': 'GDOF/s per Schwarz sweep; time-to-1e-10 residual, plain FP64 vs mixed/learned',
        'value': modes['fp64']['schwarz_gdofs_all_rhs'], 'unit': 'GDOF/s', 'n_gpus': 1, 'steps': args.cycles,
        'warmup': 1, 'ms_per_step': round(modes['fp64']['s_per_cycle'] * 1e3, 2), 'higher_is_better': True,
        'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f64', 'data': 'synthetic',
        'config': {'workload': 'stretched_perturbed_48^3_p8_aspect100_16rhs', 'n_dof_per_rhs': ndof, 'n_rhs': R,
                   'cycle': 'FAS-MG-SCG(12,4), p-levels 8->4->2->1, root SCG to 1e-1', 'mu_star': 5.0,
                   'overlap': 'delta 0.24: m = 3 at p = 8, 2 at p = 4, 1 below'},
        'modes': modes,
    }
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print('bench.py runs on one GPU only: the library has no multi-GPU path.',
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2608_14123_amd import binding as B
    assert torch.cuda.is_available(), 'needs a GPU'
    if args.workload == 'front':
        front_bench(args, torch, B)
        return
    if args.workload == 'stretched':
        stretched_bench(args, torch, B)
        return
    if args.workload == 'local':
        return local_bench(args, torch, B)
    if args.workload == 'diamond':
        return diamond_bench(args, torch, B)
    if args.workload == 'mlp':
        mlp_bench(args, torch, B)
        return
    ne, p = args.ne, args.p
    E = ne ** 3
    n3 = (p + 1) ** 3
    ndof = E * n3
    X, nbr, bc = build_workload(ne, p, B.gll(p)[0])
    from paper_2608_14123_amd import workloads as W
    f_host = W.uniform_nodal(ndof, 2)
    stream = torch.cuda.current_stream()
    cyc = dict(smoother=B.SCG, ns1=3, ns2=2, mu_star=5.0, root_rtol=0.1)
    degs = np.full(E, p, np.int32)

    order = B.ORDER_MORTON if args.order == 'morton' else B.ORDER_NATURAL

    def solver(**kw):
        o = dict(cyc, **kw)
        if 'h_levels' not in o:
            o['order'] = order
        return B.Solver(degs, X, nbr, bc, B.default_options(**o), stream=stream.cuda_stream, box=(ne, ne, ne))

    t_setup = time.perf_counter()
    lib = solver()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    L = lib.n_levels
    level_dofs = [lib.level_info(l)[1] for l in range(1, L + 1)]
    levels_str = '->'.join(str(lib.level_info(l)[0]) for l in range(L, 0, -1))
    f = torch.from_numpy(f_host).cuda()
    b = torch.empty_like(f)
    lib.rhs(f, b)
    u = torch.zeros_like(b)
    print('setup %.2fs, %d levels, %d DOF' % (t_setup, L, ndof), file=sys.stderr, flush=True)

    # timed steps: FAS-MG-SCG(3,2) V-cycles
    for _ in range(args.warmup):
        lib.vcycle(u, b)
    torch.cuda.synchronize()
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lib.vcycle(u, b)
    torch.cuda.synchronize()
    ms_cycle = (time.perf_counter() - t0) * 1e3 / args.steps
    print('V-cycle %.3f ms' % ms_cycle, file=sys.stderr, flush=True)

    g = torch.from_numpy(W.uniform_nodal(ndof, 3)).cuda()
    r = torch.empty_like(g)
    uu = torch.from_numpy(W.uniform_nodal(ndof, 4)).cuda()

    def med_ms(fn, reps=None):
        """median of per-call event timings on the library's stream, after one warm-up call"""
        reps = reps or args.reps
        fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in evs:
            e0.record(stream)
            fn()
            e1.record(stream)
        evs[-1][1].synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))

    def mean_ms(fn, reps=None):
        """mean over back-to-back calls between two events (the launch duration of one kernel)"""
        reps = reps or args.reps
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    # kernels and sweeps of the FP64 SCG solver on the finest level
    ms_res = mean_ms(lambda: lib.residual(L, uu, g, r))          # one operator launch
    ms_sz = med_ms(lambda: lib.schwarz(L, g, r))                # FD solve + overlap add
    ms_scg1 = med_ms(lambda: lib.smooth(L, uu, g, 1))
    ms_scg3 = med_ms(lambda: lib.smooth(L, uu, g, 3))
    ms_scg_it = (ms_scg3 - ms_scg1) / 2                          # one SCG iteration
    lib_sweeps = {}
    # WAS sweeps (r = g - A u; u += B r) in each precision: FP64 one call of one step; the
    # reduced-precision forms time one inner correction sweep as smooth(2) - smooth(1)
    for key, kw in (('fp64', {}), ('fp32', dict(precision=B.FP32)), ('bf16', dict(precision=B.BF16)),
                    ('fp32_matrix_cores', dict(precision=B.FP32_MFMA))):
        w = solver(smoother=B.WAS, **kw)
        t1 = med_ms(lambda: w.smooth(L, uu, g, 1))
        if key == 'fp64':
            ms = t1
        else:
            ms = med_ms(lambda: w.smooth(L, uu, g, 2)) - t1
        w.close()
        bal = 72.0 if key == 'fp64' else 36.0
        gd = ndof / (ms * 1e-3) / 1e9
        lib_sweeps[key] = {'ms': round(ms, 4), 'gdofs': round(gd, 3), 'algorithmic_bytes_per_dof': bal,
                           'roofline_gdofs': round(HBM_PEAK_GBS / bal, 1), 'frac': round(gd / (HBM_PEAK_GBS / bal), 4)}
        print('WAS sweep', key, lib_sweeps[key], file=sys.stderr, flush=True)
    value = lib_sweeps['fp64']['gdofs']

    # algorithmic work: the operator's minimum bytes (u, g, r and the geometry as coordinates,
    # 3 x 8 B) and the FD solve's exact flops, each over its measured launch time
    bytes_res = 48.0 * ndof
    ach_res = bytes_res / (ms_res * 1e-3) / 1e9
    ns = p + 3
    n_int = ne - 2
    sizes = [ns] * n_int + [ns - 1] * 2
    flops_fd = 0.0
    for a in sizes:
        for b_ in sizes:
            for c in sizes:
                flops_fd += (4.0 * (a + b_ + c) + 1.0) * a * b_ * c
    ach_fd = flops_fd / (ms_sz * 1e-3) / 1e12
    import hashlib
    src = os.path.join(ROOT, 'paper_2608_14123_amd', 'csrc', 'k_operator.hip')
    sha = hashlib.sha256(open(src, 'rb').read()).hexdigest()[:16]
    traffic = (OPERATOR_TRAFFIC['bytes'] if sha == OPERATOR_TRAFFIC['sha256_prefix'] and ne == OPERATOR_TRAFFIC['ne']
               and p == OPERATOR_TRAFFIC['p'] else None)
    roof_res = {'kernel': 'sipg_apply_kernel<8,double> (residual)', 'bound': 'hbm', 'achieved': round(ach_res, 1),
                'peak': HBM_PEAK_GBS, 'unit': 'GB/s', 'frac': round(ach_res / HBM_PEAK_GBS, 4),
                'traffic': traffic, 'traffic_unit': 'bytes per launch', 'algorithmic_bytes': bytes_res,
                'launch_ms': round(ms_res, 4)}
    roof_fd = {'kernel': 'schwarz_solve_kernel<8,1,double> + overlap add', 'bound': 'alu',
               'achieved': round(ach_fd, 2), 'peak': FP64_PEAK_TFLOPS, 'unit': 'TFLOP/s',
               'frac': round(ach_fd / FP64_PEAK_TFLOPS, 4), 'traffic': None, 'median_ms': round(ms_sz, 4)}
    dominant, other = (roof_res, roof_fd) if ms_res >= ms_sz else (roof_fd, roof_res)

    def t10_roof_s(n10, ns1, ns2, nsc, lowp):
        """Algorithmic time of the n10 cycles at the HBM roof: per cycle the finest level's
        smoothing iterations (each an operator and a Schwarz application: 72 B/DOF in FP64,
        36 B/DOF in FP32) plus two FP64 residuals (48 B/DOF), scaled by the coarser levels'
        share of the DOF; start-ups are not counted."""
        pre = ns1 if (nsc is None or n10 <= 1) else (ns1 + (n10 - 1) * (nsc - ns2)) / n10
        per_dof = (pre + ns2) * (36.0 if lowp else 72.0) + 2 * 48.0
        return n10 * per_dof * sum(level_dofs) / (HBM_PEAK_GBS * 1e9)

    t10 = {}
    if not args.no_t10:
        def time_to_tol(solver_, key, ns=(3, 2), nsc=None, lowp=False):
            hist, ok = solver_.solve(u.zero_(), b, max_cycles=30, rtol=1e-10)
            torch.cuda.synchronize()
            t_a = time.perf_counter()
            hist, ok = solver_.solve(u.zero_(), b, max_cycles=30, rtol=1e-10)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t_a
            n10 = len(hist) - 1
            roof = t10_roof_s(n10, ns[0], ns[1], nsc, lowp)
            t10[key] = {'t10_s': round(ts, 4), 'n10': n10, 'converged': bool(ok), 'final_rho': float(hist[-1]),
                        't10_roof_s': round(roof, 5), 't10_over_roof': round(ts / roof, 2)}
            print('t10', key, t10[key], file=sys.stderr, flush=True)
            solver_.close()

        time_to_tol(lib, 'fp64')
        # the other forms of the same cycle: FP32 / BF16 smoothing of the correction system, a
        # fixed 16-iteration root solve with every cycle one captured HIP graph, and the paper's
        # start-ups: FAS-FMG-SCG(3,2) and FAS-FMG-SCG(3,2,3) with crossover smoothing (the
        # paper's best p = 8 method on its Cartesian meshes)
        fixed = dict(root_rtol=0.0, root_max_iter=16, graph=1)
        fmg = dict(start=B.START_FMG)
        for key, kw, nsc, lowp in (
                ('fp32_smoother', dict(precision=B.FP32), None, True),
                ('bf16_matrix_core_smoother', dict(precision=B.BF16), None, True),
                ('fp32_matrix_core_smoother', dict(precision=B.FP32_MFMA), None, True),
                ('fp64_fixed_root16_whole_cycle_graph', fixed, None, False),
                ('fp32_smoother_fixed_root16_whole_cycle_graph', dict(fixed, precision=B.FP32), None, True),
                ('fp64_fmg', fmg, None, False),
                ('fp32_smoother_fmg_fixed_root16_graph', dict(fmg, precision=B.FP32, **fixed), None, True),
                ('fp64_fmg_crossover3', dict(fmg, nsc=3), 3, False),
                # h-coarsening (Sec. 3.1): 32^3 -> 16^3 -> 8^3 elements at p = 7, then the p-levels of
                # the 8^3 mesh (a third h-step would leave 4^3 elements whose p = 1 maps fold); and
                # pure h-MG to a 4^3, p = 7 root
                ('fp64_h2_then_p', dict(h_levels=2), None, False),
                ('fp64_h2_then_p_fmg', dict(h_levels=2, **fmg), None, False),
                ('fp64_h3_only', dict(h_levels=3, h_only=1), None, False),
                # h-coarsening with the FP32 smoother (a fixed-count root is not used there: the 8^3,
                # p = 1 root level is indefinite at mu_star = 5, and only the tolerance-driven root stops
                # at the breakdown)
                ('fp32_smoother_h2_then_p', dict(h_levels=2, precision=B.FP32), None, True)):
            try:
                time_to_tol(solver(**kw), key, nsc=nsc, lowp=lowp)
            except B.DgfasError as ex:     # a form the library refuses for this mesh is recorded
                t10[key] = {'error': str(ex)}
                print('t10', key, t10[key], file=sys.stderr, flush=True)
    else:
        lib.close()

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device='cuda')   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    out = {
        'metric': 'GDOF/s per Schwarz sweep; time-to-1e-10 residual, plain FP64 vs mixed/learned',
        'value': round(value, 3), 'unit': 'GDOF/s', 'n_gpus': 1, 'steps': args.steps, 'warmup': args.warmup,
        'ms_per_step': round(ms_cycle, 4), 'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None,
        'dtype': 'f64', 'data': 'synthetic',
        'config': {'workload': 'curved_cube_%d^3_p%d_sine_bump_0.1' % (ne, p), 'n_dof': ndof,
                   'value': 'FP64 WAS sweep (residual + Schwarz + update) on the finest level, median of %d'
                            % args.reps,
                   'step': 'one FAS-MG-SCG(3,2) V-cycle, p-levels %s, root SCG to 1e-1' % levels_str,
                   'overlap': 1, 'mu_star': 5.0, 'rhs': 'U[-1,1] seed 2', 'element_order': args.order},
        'roofline': dominant,
        'roofline_other': other,
        'was_sweep': lib_sweeps,
        'kernel_ms': {'operator_launch': round(ms_res, 4), 'schwarz_application': round(ms_sz, 4),
                      'scg_iteration': round(ms_scg_it, 4)},
        'schwarz_gdofs': round(ndof / (ms_sz * 1e-3) / 1e9, 3),
        'scg_iteration_gdofs': round(ndof / (ms_scg_it * 1e-3) / 1e9, 3),
        'cycle_gdofs_5_sweeps': round(ndof * 5 / (ms_cycle * 1e-3) / 1e9, 3),
        't10': t10,
        'setup_s': round(t_setup, 3),
    }
    if not args.no_cpu:
        n10 = t10.get('fp64', {}).get('n10', 22)
        out['cpu_baseline'] = cpu_baseline(ne, p, n10)
    print(json.dumps(out))


if __name__ == '__main__':
    main()
