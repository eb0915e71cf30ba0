"""The library's host-side subdomain tables for unstructured meshes (csrc/topology.cpp, built
here with g++ through tests/topology_shim.cpp; no GPU) against the oracle's Schwarz method of
oracle.unstructured: the block counts, every slot's nodes and merge shares, and every per-node
weight (share x tensor weight / weight sum, Sec. 4.3.1)."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle.gll import gll
from oracle.mesh import Mesh
from oracle.schwarz import side_codes
from oracle.unstructured import TopoSchwarz
from paper_2608_14123_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def bump_mesh(p, ne=3):
    nbr, bc = W.box_topology(ne, ne, ne)
    X = W.element_coords(W.box_vertices(ne, ne, ne), gll(p)[0], lambda Y: W.sine_bump_map(Y, 0.03))
    return X, nbr, bc


def turned(X, seed):
    rot = np.random.default_rng(seed).integers(0, len(W.ROTATIONS), size=len(X))
    return W.rotate_local_axes(X, rot)


def diamond(p, nc=2, layers=2, periodic=False):
    X = W.diamond_coords(nc, layers, gll(p)[0], shift_seed=1, rot_seed=2)
    nbr, nf, no, bc = W.face_connectivity(X, period=1.0 if periodic else None)
    return X, nbr, nf, no, bc


@pytest.fixture(scope='module')
def shim():
    src = [os.path.join(ROOT, 'paper_2608_14123_amd', 'csrc', 'topology.cpp'), os.path.join(ROOT, 'tests', 'topology_shim.cpp')]
    d = tempfile.mkdtemp()
    so = os.path.join(d, 'topo_shim.so')
    subprocess.run(['g++', '-std=c++17', '-O1', '-shared', '-fPIC', '-o', so] + src, check=True)
    lib = ctypes.CDLL(so)
    lib.shim_topo_tables.restype = ctypes.c_int
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def host_tables(lib, mesh, m):
    """Run topology.cpp on the oracle's variants: (blocks, gather, merged lists, per-node lists)."""
    from oracle.schwarz import variant_1d
    n, E = mesh.n, mesh.E
    ns = n + 2 * m
    keys, var = {}, np.zeros((E, 3), np.int8)
    for e in range(E):
        sc = side_codes(mesh, e)
        for d in range(3):
            var[e, d] = keys.setdefault(sc[d], len(keys))
    nv = len(keys)
    map1d = np.full((nv, ns), -1, np.int32)
    Wt = np.zeros((nv, ns))
    for lr, v in keys.items():
        vt = variant_1d(mesh.p, m, lr[0], lr[1], mesh.mu_star)
        for s, (dl, l) in enumerate(vt['nodes']):
            map1d[v, s] = ((dl + 1) << 6) | l
            Wt[v, s] = vt['W'][s]
    nt = ns ** 3
    cap = E * nt * 8
    blocks = np.zeros(5, np.int64)
    gather = np.zeros(E * nt, np.int32)
    nmerge = ctypes.c_int()
    mptr = np.zeros(E * nt + 1, np.int32)
    midx = np.zeros(cap, np.int32)
    sptr = np.zeros(mesh.n_dof() + 1, np.int64)
    sslot = np.zeros(cap, np.int32)
    scoef = np.zeros(cap)
    rc = lib.shim_topo_tables(E, n, _ptr(np.ascontiguousarray(mesh.nbr, np.int32)),
                              _ptr(np.ascontiguousarray(np.where(mesh.nbr >= 0, mesh.nbr_face, 0), np.int8)),
                              _ptr(np.ascontiguousarray(mesh.nbr_orient, np.int8)), ns, _ptr(var), _ptr(map1d),
                              _ptr(Wt), 1, _ptr(blocks), _ptr(gather), ctypes.byref(nmerge), _ptr(mptr), len(mptr),
                              _ptr(midx), len(midx), _ptr(sptr), _ptr(sslot), _ptr(scoef), ctypes.c_int64(cap))
    assert rc == 0, rc
    nnz = int(sptr[-1])
    return blocks, gather.reshape(E, nt), mptr[:nmerge.value + 1], midx, sptr, sslot[:nnz], scoef[:nnz], ns


@pytest.mark.parametrize('case', ['diamond', 'diamond_periodic', 'turned'])
def test_library_host_tables_match_the_oracle(shim, case):
    p = 2
    if case == 'turned':
        X0, _, _ = bump_mesh(p)
        X = turned(X0, 9)
        nbr, nf, no, bc = W.face_connectivity(X)
    else:
        X, nbr, nf, no, bc = diamond(p, nc=2, layers=3, periodic=case.endswith('periodic'))
    mesh = Mesh(p, X, nbr, bc, nbr_face=nf, nbr_orient=no)
    T = TopoSchwarz(mesh, 1)
    blocks, gather, mptr, midx, sptr, sslot, scoef, ns = host_tables(shim, mesh, 1)
    kinds = ('own', 'face', 'map', 'zero', 'merge')
    want = [sum(list(sd['kinds'].values()).count(k) for sd in T.sub) for k in kinds]
    assert blocks.tolist() == want
    nt = ns ** 3
    lib_entries, ora_entries = [], []
    for sd in T.sub:
        e = sd['e']
        n3, n2, n1 = sd['shape']
        for s, g, c in zip(sd['slot'], sd['gidx'], sd['coef']):
            s1, s2, s3 = s % n1, (s // n1) % n2, s // (n1 * n2)
            ora_entries.append((e, (s3 * ns + s2) * ns + s1, int(g), round(float(c), 12)))
        for ls in range(nt):
            gi = int(gather[e, ls])
            if gi >= 0:
                lib_entries.append((e, ls, gi, 1.0))
            elif gi <= -2:
                j = -2 - gi
                nodes = midx[mptr[j]:mptr[j + 1]]
                lib_entries += [(e, ls, int(x), round(1.0 / len(nodes), 12)) for x in nodes]
    assert sorted(lib_entries) == sorted(ora_entries)
    # per-node lists: every normalised weight is the oracle's share x tensor weight / weight sum
    ora = {}
    for sd in T.sub:
        e = sd['e']
        n3, n2, n1 = sd['shape']
        Wf = sd['W'].ravel()
        for s, g, c in zip(sd['slot'], sd['gidx'], sd['coef']):
            s1, s2, s3 = s % n1, (s // n1) % n2, s // (n1 * n2)
            ora[(int(g), e * nt + (s3 * ns + s2) * ns + s1)] = c * Wf[s] / T.C[g]
    got = {}
    for g in range(mesh.n_dof()):
        for k in range(sptr[g], sptr[g + 1]):
            got[(g, int(sslot[k]))] = scoef[k]
    assert set(got) == set(ora)
    assert max(abs(got[k] - ora[k]) for k in ora) < 1e-14
