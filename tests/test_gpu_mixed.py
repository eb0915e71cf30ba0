"""Mixed-degree levels (a degree per element) against the oracle's mixed-degree reading:
operator, right-hand side, Schwarz smoother and transfers on every level, the V-cycle,
multi-right-hand-side batches and, at the size of the hp front workload (27^3 elements,
degrees 2..8), sampled elements against oracle blocks."""
import numpy as np
import pytest

from oracle import mixed as mx, solvers as osv
from paper_2608_14123_amd import workloads as W
from gpu_cases import MixedCase, mixed_block

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


@pytest.fixture(scope='module')
def binding():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2608_14123_amd import binding as b
    return b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = [
    # every degree pair 1..5 in a seeded layout, curved map (degree-1 elements stay on all levels)
    MixedCase('mixed_1to5_3^3', 3, np.random.default_rng(3).integers(1, 6, 27), amp=0.03),
    # a front-like layout with degrees 2..8 and Neumann faces with kappa > 0
    MixedCase('front_2to8_3^3', 3, W.front_degrees(3, center=(0.1, 0.1, 0.1), r0=0.55), amp=0.02, bc_code=2,
              kappa=0.5),
    MixedCase('mixed_2to4_4^3', 4, np.random.default_rng(5).integers(2, 5, 64), amp=0.03, mu_star=5.0),
]


@pytest.mark.parametrize('case', CASES, ids=repr)
def test_mixed_operator_rhs_schwarz_every_level(binding, case):
    print('mixed kernels', case, flush=True)
    lv = case.oracle_levels()
    lib = case.library(binding)
    assert lib.n_levels == len(lv)
    rng = np.random.default_rng(11)
    for l in range(1, lib.n_levels + 1):
        o = lv[l - 1]
        n = o.mesh.n_dof()
        assert lib.level_info(l) == (int(o.mesh.p.max()), n)
        u = rng.uniform(-1, 1, n)
        g = rng.uniform(-1, 1, n)
        out = torch.empty(n, dtype=torch.float64, device='cuda')
        lib.apply(l, dev(u), out)
        ref = o.A(u)
        assert rel(host(out), ref) <= 1e-12, ('apply', l)
        lib.residual(l, dev(u), dev(g), out)
        assert rel(host(out), g - ref) <= 1e-12, ('residual', l)
        lib.schwarz(l, dev(g), out)
        assert rel(host(out), o.B(g)) <= 1e-11, ('schwarz', l)
    top = lv[-1].mesh
    n = top.n_dof()
    f = rng.uniform(-1, 1, n)
    uD = rng.uniform(-1, 1, n)
    b = torch.empty(n, dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b, uD=dev(uD))
    assert rel(host(b), top.rhs(f, uD=uD)) <= 1e-12
    lib.close()


@pytest.mark.parametrize('case', CASES[:2], ids=repr)
def test_mixed_transfers(binding, case):
    print('mixed transfers', case, flush=True)
    lv = case.oracle_levels()
    lib = case.library(binding)
    rng = np.random.default_rng(12)
    for l in range(2, lib.n_levels + 1):
        F, C = lv[l - 1].mesh, lv[l - 2].mesh
        uf = rng.uniform(-1, 1, F.n_dof())
        uc = rng.uniform(-1, 1, C.n_dof())
        ub = rng.uniform(-1, 1, C.n_dof())
        out_c = torch.empty(C.n_dof(), dtype=torch.float64, device='cuda')
        lib.restrict(l, dev(uf), out_c)
        assert rel(host(out_c), mx.restrict(F, C, uf)) <= 1e-13
        lib.project(l, dev(uf), out_c)
        assert rel(host(out_c), mx.project(F, C, uf)) <= 1e-13
        out_f = dev(uf)
        lib.prolong_add(l, dev(uc), out_f, ubar=dev(ub))
        assert rel(host(out_f), uf + mx.prolong(C, F, uc - ub)) <= 1e-13
    lib.close()


def front_problem(case, lib_side, binding=None):
    """f and u_D of the spherical front (centre outside the domain) at the nodes of either side."""
    from oracle.gll import gll as ogll
    xi = (lambda p: binding.gll(p)[0]) if lib_side else (lambda p: ogll(p)[0])
    X = case.coords(xi)
    c = (-0.05, -0.05, -0.05)
    f = np.concatenate([W.front_source(x, alpha=3.0, r0=0.5, center=c).ravel() for x in X])
    uD = np.concatenate([W.front_solution(x, alpha=3.0, r0=0.5, center=c).ravel() for x in X])
    return f, uD


@pytest.mark.parametrize('precision', ['fp64', 'fp32', 'bf16', 'fp32mfma'])
def test_mixed_vcycle_history_and_solution(binding, precision):
    """FAS-MG-SCG(3,2) on a mixed 2^3 mesh: FP64 follows the oracle's history cycle by cycle;
    every precision (BF16 and FP32 matrix cores: subdomain solves per degree bucket) reaches
    the direct solution of the mixed system."""
    print('mixed vcycle', precision, flush=True)
    case = MixedCase('mixed_vc_2^3', 2, [4, 3, 3, 2, 3, 2, 2, 2])
    lv = case.oracle_levels()
    top = lv[-1].mesh
    fo, uDo = front_problem(case, False)
    bo = top.rhs(fo, uD=uDo)
    opts = osv.Options('scg', 3, 2, root_rtol=1e-1)
    cycles = 6
    uo, ho = mx.solve(lv, np.zeros_like(bo), bo, opts, max_cycles=cycles, rtol=0.0)
    prec = {'fp64': binding.FP64, 'fp32': binding.FP32, 'bf16': binding.BF16, 'fp32mfma': binding.FP32_MFMA}[precision]
    lib = case.library(binding, smoother=binding.SCG, ns1=3, ns2=2, root_rtol=1e-1, precision=prec)
    f, uD = front_problem(case, True, binding)
    b = torch.empty(top.n_dof(), dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b, uD=dev(uD))
    u = torch.zeros_like(b)
    if precision == 'fp64':
        hg, _ = lib.solve(u, b, max_cycles=cycles, rtol=0.0)
        for a, c in zip(hg, ho):
            assert abs(a - c) <= 1e-6 * c + 1e-14, (hg, ho)
        assert rel(host(u), uo) <= 1e-8
        u.zero_()
    hg, ok = lib.solve(u, b, max_cycles=60, rtol=1e-11)
    assert ok and hg[-1] <= 1e-11, hg
    uex = np.linalg.solve(top.assemble(), bo)
    assert rel(host(u), uex) <= 1e-8
    lib.close()


def test_mixed_batched_rhs(binding):
    print('mixed batch', flush=True)
    case = CASES[0]
    R = 3
    lv = case.oracle_levels()
    lib = case.library(binding, n_rhs=R)
    rng = np.random.default_rng(13)
    for l in range(1, lib.n_levels + 1):
        o = lv[l - 1]
        n = o.mesh.n_dof()
        u = rng.uniform(-1, 1, (R, n))
        out = torch.empty(R * n, dtype=torch.float64, device='cuda')
        lib.apply(l, dev(u), out)
        got = host(out).reshape(R, n)
        for k in range(R):
            assert rel(got[k], o.A(u[k])) <= 1e-12
        lib.schwarz(l, dev(u), out)
        got = host(out).reshape(R, n)
        for k in range(R):
            assert rel(got[k], o.B(u[k])) <= 1e-11
        if l > 1:
            C = lv[l - 2].mesh
            oc = torch.empty(R * C.n_dof(), dtype=torch.float64, device='cuda')
            lib.restrict(l, dev(u), oc)
            got = host(oc).reshape(R, C.n_dof())
            for k in range(R):
                assert rel(got[k], mx.restrict(o.mesh, C, u[k])) <= 1e-13
    lib.close()


@pytest.fixture(scope='module')
def front27(binding):
    """The hp front workload: 27^3 unit cubes, p_e = max(2, 8 - floor(d_e / h)), 3,217,284 DOF."""
    degs = W.front_degrees(27)
    case = MixedCase('front_27^3', 27, degs)
    lib = case.library(binding, smoother=binding.SCG, ns1=3, ns2=2, root_rtol=1e-1)
    yield case, lib
    lib.close()


def test_front_workload_sampled_elements(binding, front27):
    """Finest level at full size: operator and Schwarz outputs of sampled elements against
    oracle blocks (radius 1 for the operator, 2 for the Schwarz smoother)."""
    print('front 27^3 sampled', flush=True)
    case, lib = front27
    n = int(case.off[-1])
    assert lib.level_info(lib.n_levels) == (8, n) and n == 3217284
    rng = np.random.default_rng(14)
    u = rng.uniform(-1, 1, n)
    Au = torch.empty(n, dtype=torch.float64, device='cuda')
    z = torch.empty(n, dtype=torch.float64, device='cuda')
    lib.apply(lib.n_levels, dev(u), Au)
    lib.schwarz(lib.n_levels, dev(u), z)
    Au, z = host(Au), host(z)
    degs = case.degrees
    nbr = case.nbr
    mortar = [e for e in range(case.E) if any(nbr[e, f] >= 0 and degs[nbr[e, f]] != degs[e] for f in range(6))]
    picks = [mortar[0], mortar[len(mortar) // 2], int(np.argmax(degs == 8)), int(np.argmax(degs == 2)),
             int(np.argmax(degs == 5))]
    for e in picks:
        for radius, kind in ((1, 'A'), (2, 'B')):
            mesh, ids, c = mixed_block(case, e, radius)
            ub = np.concatenate([u[case.off[g]:case.off[g + 1]] for g in ids])
            ref = mesh.apply(ub) if kind == 'A' else mx.MixedSchwarz(mesh, 1).apply(ub)
            got = (Au if kind == 'A' else z)[case.off[e]:case.off[e + 1]]
            assert rel(got, ref[mesh.off[c]:mesh.off[c + 1]]) <= 1e-11, (e, kind, degs[e])


def test_front_workload_converges(binding, front27):
    """Full-size FAS-MG-SCG(3,2) V-cycles on the front (alpha = 50): the residual falls by at
    least 5x per cycle.  (Plain WAS diverges on mixed-degree meshes under the no-overlap
    reading at degree jumps; the oracle shows the same on small front meshes.)"""
    print('front 27^3 cycles', flush=True)
    case, lib = front27
    n = int(case.off[-1])
    X = case.coords(lambda p: binding.gll(p)[0])
    f = np.concatenate([W.front_source(x).ravel() for x in X])
    uD = np.concatenate([W.front_solution(x).ravel() for x in X])
    b = torch.empty(n, dtype=torch.float64, device='cuda')
    lib.rhs(dev(f), b, uD=dev(uD))
    u = torch.zeros_like(b)
    hist, _ = lib.solve(u, b, max_cycles=4, rtol=0.0)
    assert all(np.isfinite(hist)) and all(hist[k + 1] < 0.2 * hist[k] for k in range(len(hist) - 1)), hist


@pytest.mark.parametrize('case', CASES, ids=repr)
def test_one_launch_batches_match_per_degree_launches(binding, case):
    """The one-launch batch (and its persistent form) of every sweep stage computes every
    element as its degree's own launch does: bitwise equal results on every level."""
    print('one-launch batches', case, flush=True)
    lv = case.oracle_levels()
    per = case.library(binding)
    one = case.library(binding, batch=binding.BATCH_ONE_LAUNCH)
    pst = case.library(binding, batch=binding.BATCH_PERSISTENT)
    rng = np.random.default_rng(15)
    for l in range(1, per.n_levels + 1):
        n = lv[l - 1].mesh.n_dof()
        u, g = dev(rng.uniform(-1, 1, n)), dev(rng.uniform(-1, 1, n))
        outs = []
        for lib in (per, one, pst):
            a = torch.empty(n, dtype=torch.float64, device='cuda')
            r = torch.empty_like(a)
            z = torch.empty_like(a)
            lib.apply(l, u, a)
            lib.residual(l, u, g, r)
            lib.schwarz(l, g, z)
            outs.append([host(a), host(r), host(z)])
        for other in outs[1:]:
            for x, y in zip(outs[0], other):
                assert np.array_equal(x, y), (l, np.abs(x - y).max())
        assert rel(outs[1][2], lv[l - 1].B(host(g))) <= 1e-11
    per.close()
    one.close()
    pst.close()


def test_persistent_batches_at_front_size(binding, front27):
    """On the 27^3 front the stages have far more tiles than the persistent grid, so its
    workgroups stride through the tile list: operator, residual and Schwarz results on the
    finest level are bitwise those of per-degree launches."""
    print('front 27^3 persistent', flush=True)
    case, _ = front27
    n = int(case.off[-1])
    rng = np.random.default_rng(18)
    u, g = dev(rng.uniform(-1, 1, n)), dev(rng.uniform(-1, 1, n))
    outs = []
    for batch in (binding.BATCH_PER_DEGREE, binding.BATCH_PERSISTENT):
        lib = case.library(binding, smoother=binding.SCG, ns1=3, ns2=2, root_rtol=0.1, batch=batch)
        L = lib.n_levels
        a = torch.empty(n, dtype=torch.float64, device='cuda')
        r, z = torch.empty_like(a), torch.empty_like(a)
        lib.apply(L, u, a)
        lib.residual(L, u, g, r)
        lib.schwarz(L, g, z)
        outs.append([host(a), host(r), host(z)])
        lib.close()
    for x, y in zip(*outs):
        assert np.array_equal(x, y), np.abs(x - y).max()


@pytest.mark.parametrize('batch,precision', [(0, 'fp64'), (1, 'fp64'), (1, 'fp32')])
def test_graph_replayed_cycles_are_bitwise_eager(binding, batch, precision):
    """dgfas_solve with the captured legs replays them once per cycle, with the eager root
    solve and residual norms between replays: histories and iterates are bitwise those of
    the eager cycles."""
    print('graph replay', batch, precision, flush=True)
    case = CASES[2]
    prec = binding.FP64 if precision == 'fp64' else binding.FP32
    n = int(case.off[-1])
    f = np.random.default_rng(16).uniform(-1, 1, n)
    res = []
    for graph in (0, 1):
        lib = case.library(binding, smoother=binding.SCG, ns1=3, ns2=2, root_rtol=1e-1, precision=prec,
                           batch=batch, graph=graph)
        b = torch.empty(n, dtype=torch.float64, device='cuda')
        lib.rhs(dev(f), b)
        u = torch.zeros_like(b)
        h1, _ = lib.solve(u, b, max_cycles=4, rtol=0.0)
        u1 = host(u).copy()
        h2, _ = lib.solve(u, b, max_cycles=3, rtol=0.0)     # replays continue from the current iterate
        res.append((h1, u1, h2, host(u)))
        lib.close()
    for x, y in zip(*res):
        assert np.array_equal(x, y)
    assert res[0][0][-1] < 1e-2


def test_autotuner_times_choices_and_reuses_its_cache(binding, tmp_path):
    print('autotune', flush=True)
    case = CASES[1]
    lv = case.oracle_levels()
    cache = tmp_path / 'tune.json'
    lib = case.library(binding)
    rep = lib.autotune(cache, reps=3)
    mixed = [l for l in range(lib.n_levels) if len(np.unique(lv[l].mesh.p)) > 1]
    assert mixed and all((rep[l] > 0).all() for l in mixed)
    assert all((rep[l] == 0).all() for l in range(lib.n_levels) if l not in mixed)
    text = cache.read_text()
    assert text.count('operator') == len(mixed) and text.count('solve') == len(mixed)
    # tuned launches give the oracle's results
    rng = np.random.default_rng(17)
    for l in range(1, lib.n_levels + 1):
        nl = lv[l - 1].mesh.n_dof()
        u = rng.uniform(-1, 1, nl)
        out = torch.empty(nl, dtype=torch.float64, device='cuda')
        lib.apply(l, dev(u), out)
        assert rel(host(out), lv[l - 1].A(u)) <= 1e-12
        lib.schwarz(l, dev(u), out)
        assert rel(host(out), lv[l - 1].B(u)) <= 1e-11
    lib.close()
    # a second solver finds every choice in the cache and times nothing
    lib2 = case.library(binding)
    rep2 = lib2.autotune(cache, reps=3)
    assert (rep2 == 0).all()
    assert cache.read_text() == text
    lib2.close()
