"""CPU checks of the HIP library: symbols, host tables against the oracle (values only)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, 'paper_2608_14123_amd', 'libdgfas.so')


def declared_functions():
    src = open(os.path.join(ROOT, 'include', 'dgfas.h')).read()
    src = re.sub(r'/\*.*?\*/', '', src, flags=re.S)
    return sorted(set(re.findall(r'\b(dgfas_[a-z0-9_]+)\s*\(', src)))


@pytest.fixture(scope='module')
def lib():
    if not os.path.exists(LIB):
        pytest.fail('libdgfas.so is not built (run __graft_entry__.build())')
    from paper_2608_14123_amd import binding
    return binding


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    so = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(so, n), n
    assert set(names) <= set(lib.EXPORTED) | {'dgfas_default_options'}


@pytest.mark.parametrize('p', [1, 2, 3, 4, 7, 8, 12, 16])
def test_gll_matches_oracle(lib, p):
    from oracle.gll import gll
    x, w = lib.gll(p)
    xo, wo = gll(p)
    assert np.abs(x - xo).max() < 1e-15 and np.abs(w - wo).max() < 1e-15


@pytest.mark.parametrize('p,m', [(1, 1), (3, 1), (4, 1), (4, 2), (7, 1), (8, 1), (8, 2)])
@pytest.mark.parametrize('lr', [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (0, 2), (1, 2)])
def test_schwarz_tables_match_oracle(lib, p, m, lr):
    from oracle.schwarz import variant_1d
    code = 'idn'
    v = variant_1d(p, m, code[lr[0]], code[lr[1]], 2.0)
    S, lam, W = lib.schwarz_tables_1d(p, m, lr[0], lr[1], 2.0)
    assert np.allclose(W, v['W'], atol=1e-15)
    # eigenpairs up to order and sign: compare the reconstructed operators
    M = np.diag(v['M'])
    Linv_lib = S @ np.diag(1 / lam) @ S.T
    Linv_or = v['S'] @ np.diag(1 / v['lam']) @ v['S'].T
    assert np.abs(Linv_lib - Linv_or).max() < 1e-11 * np.abs(Linv_or).max()
    assert np.abs(S.T @ M @ S - np.eye(len(lam))).max() < 1e-13
    assert np.abs(np.sort(lam) - np.sort(v['lam'])).max() < 1e-11 * np.abs(lam).max()


@pytest.mark.parametrize('p,m', [(2, 1), (3, 1), (8, 1)])
@pytest.mark.parametrize('lr', [(3, 3), (3, 0), (0, 3), (3, 1), (2, 3)])
def test_no_overlap_interior_side_matches_oracle(lib, p, m, lr):
    """Side code 3: interior face toward another degree, no overlap (mixed-degree levels)."""
    from oracle.mixed import variant_1d_sides
    code = {0: 'i', 1: 'd', 2: 'n', 3: 'i'}
    ms = [0 if c == 3 else (m if c == 0 else 0) for c in lr]
    v = variant_1d_sides(p, ms[0], ms[1], code[lr[0]], code[lr[1]], 2.0)
    S, lam, W = lib.schwarz_tables_1d(p, m, lr[0], lr[1], 2.0)
    assert len(lam) == len(v['nodes'])
    assert np.allclose(W, v['W'], atol=1e-15)
    Linv_lib = S @ np.diag(1 / lam) @ S.T
    Linv_or = v['S'] @ np.diag(1 / v['lam']) @ v['S'].T
    assert np.abs(Linv_lib - Linv_or).max() < 1e-11 * np.abs(Linv_or).max()


def test_argument_errors_are_reported_without_gpu(lib):
    with pytest.raises(lib.DgfasError) as ei:
        lib.gll(0)
    assert ei.value.code == lib.DGFAS_EINVAL
    with pytest.raises(lib.DgfasError):
        lib.schwarz_tables_1d(4, 5, 0, 0, 2.0)


def test_binding_refuses_host_and_non_tensor_vectors(lib):
    """Vector arguments go to the kernels as raw device pointers: a host tensor or a
    non-tensor is refused in the binding before any call."""
    torch = pytest.importorskip('torch')
    with pytest.raises(ValueError):
        lib._dev(torch.zeros(8, dtype=torch.float64), 8, 'u')
    with pytest.raises(TypeError):
        lib._dev(np.zeros(8), 8, 'u')
    assert lib._dev(None, 8, 'u') is None


@pytest.mark.parametrize('bad', [dict(root_rtol=-1.0), dict(root_rtol=float('nan')), dict(precision=7),
                                 dict(n_rhs=0), dict(batch=5), dict(root_max_iter=0), dict(graph=2)])
def test_bad_options_are_refused_before_any_device_work(lib, bad):
    """Options are validated on the host before the solver touches the device, so the
    refusal is seen without a GPU."""
    from paper_2608_14123_amd import workloads as W
    ne, p = 2, 2
    nbr, bc = W.box_topology(ne, ne, ne)
    X = W.element_coords(W.box_vertices(ne, ne, ne), lib.gll(p)[0], lambda x: x)
    o = lib.default_options(**bad)
    with pytest.raises(lib.DgfasError) as ei:
        lib.Solver(np.full(ne ** 3, p, np.int32), X, nbr, bc, o)
    assert ei.value.code == lib.DGFAS_EINVAL


@pytest.mark.parametrize('bad', [dict(start=3), dict(weighting=2), dict(ns2=3, nsc=2),
                                 dict(overlap=-1, delta=1.0), dict(overlap=-1, delta=-0.1)])
def test_bad_start_crossover_weighting_and_delta_are_refused(lib, bad):
    from paper_2608_14123_amd import workloads as W
    ne, p = 2, 4
    nbr, bc = W.box_topology(ne, ne, ne)
    X = W.element_coords(W.box_vertices(ne, ne, ne), lib.gll(p)[0])
    with pytest.raises(lib.DgfasError) as ei:
        lib.Solver(np.full(ne ** 3, p, np.int32), X, nbr, bc, lib.default_options(**bad))
    assert ei.value.code == lib.DGFAS_EINVAL


@pytest.mark.parametrize('p,kw', [(8, dict(overlap=-1, delta=0.5)), (7, dict(overlap=2)), (5, dict(overlap=3))])
def test_overlap_without_a_kernel_is_unsupported(lib, p, kw):
    """delta = 0.5 at p = 8 covers the neighbour's GLL nodes up to its centre: m = 5, for which no
    Schwarz kernel exists; m = 2 exists only at p = 4 and 8, m = 3 only at p = 8."""
    from oracle.schwarz import overlap_layers
    from paper_2608_14123_amd import workloads as W
    if 'delta' in kw:
        assert overlap_layers(p, kw['delta']) == 5
    ne = 2
    nbr, bc = W.box_topology(ne, ne, ne)
    X = W.element_coords(W.box_vertices(ne, ne, ne), lib.gll(p)[0])
    with pytest.raises(lib.DgfasError) as ei:
        lib.Solver(np.full(ne ** 3, p, np.int32), X, nbr, bc, lib.default_options(**kw))
    assert ei.value.code == lib.DGFAS_EUNSUPPORTED


@pytest.mark.parametrize('case', ['negative', 'nan', 'mixed_degrees'])
def test_bad_nodal_nu_is_refused(lib, case):
    """A nodal diffusivity must be finite and >= 0 and needs one degree on the mesh; both are
    checked on the host before any device work."""
    from paper_2608_14123_amd import workloads as W
    ne, p = 2, 3
    nbr, bc = W.box_topology(ne, ne, ne)
    deg = np.full(ne ** 3, p, np.int32)
    if case == 'mixed_degrees':
        deg[0] = 2
    xs = {q: lib.gll(q)[0] for q in set(deg.tolist())}
    X = np.concatenate([x.ravel() for x in W.element_coords_mixed(W.box_vertices(ne, ne, ne), deg,
                                                                  lambda q: xs[q])])
    nu = np.ones(X.size // 3)
    if case == 'negative':
        nu[5] = -0.1
    elif case == 'nan':
        nu[7] = np.nan
    with pytest.raises(lib.DgfasError) as ei:
        lib.Solver(deg, X, nbr, bc, lib.default_options(), nu=nu)
    assert ei.value.code == (lib.DGFAS_EUNSUPPORTED if case == 'mixed_degrees' else lib.DGFAS_EINVAL)


@pytest.mark.parametrize('bad', [dict(null_space=2), dict(null_space=1, kappa=0.5)])
def test_bad_null_space_option_is_refused(lib, bad):
    from paper_2608_14123_amd import workloads as W
    ne, p = 2, 2
    nbr, bc = W.box_topology(ne, ne, ne, periodic=(True,) * 3)
    X = W.element_coords(W.box_vertices(ne, ne, ne), lib.gll(p)[0])
    with pytest.raises(lib.DgfasError) as ei:
        lib.Solver(np.full(ne ** 3, p, np.int32), X, nbr, bc, lib.default_options(**bad))
    assert ei.value.code == lib.DGFAS_EINVAL
