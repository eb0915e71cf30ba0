"""Unstructured meshes in the oracle (oriented faces, Sec. 5.1; zero fill and merging of the
Schwarz subdomains at irregular edges and vertices, Sec. 4.3.1), pinned against facts that do
not come from the oracle itself:
* turning every element's local axes leaves the operator and the Schwarz method unchanged up to
  the renumbering of the nodes (a dropped flip, transposition or sign breaks this);
* on a regular mesh the topology-walking Schwarz method is the structured one, node for node;
* the elements around every edge and vertex of the diamond mesh, found by brute force from the
  coordinates, decide which blocks are mapped, zero-filled or merged, and which elements merge;
* every node placed in a subdomain slot next to the element is the same physical point as the
  element's own boundary node there;
* the operator on the diamond mesh is symmetric and its discrete solutions converge spectrally
  to a smooth exact solution.
"""
import numpy as np
import pytest

from oracle import operator as oop, solvers as osv
from oracle.gll import gll
from oracle.mesh import Mesh
from oracle.schwarz import Schwarz
from oracle.unstructured import TopoSchwarz
from paper_2608_14123_amd import workloads as W

OPP = np.array([1, 0, 3, 2, 5, 4])


def bump_mesh(p, ne=3):
    nbr, bc = W.box_topology(ne, ne, ne)
    X = W.element_coords(W.box_vertices(ne, ne, ne), gll(p)[0], lambda Y: W.sine_bump_map(Y, 0.03))
    return X, nbr, bc


def turned(X, seed):
    rot = np.random.default_rng(seed).integers(0, len(W.ROTATIONS), size=len(X))
    return W.rotate_local_axes(X, rot)


def node_perm(X0, X1):
    """perm[e * n^3 + k] = the node of X0 at the position of node k of the turned element e."""
    E = len(X0)
    a = X0.reshape(E, 3, -1).transpose(0, 2, 1)
    b = X1.reshape(E, 3, -1).transpose(0, 2, 1)
    P = np.argmin(((b[:, :, None, :] - a[:, None, :, :]) ** 2).sum(-1), axis=2)
    return (np.arange(E)[:, None] * a.shape[1] + P).ravel()


def diamond(p, nc=2, layers=2, periodic=False):
    X = W.diamond_coords(nc, layers, gll(p)[0], shift_seed=1, rot_seed=2)
    nbr, nf, no, bc = W.face_connectivity(X, period=1.0 if periodic else None)
    return X, nbr, nf, no, bc


def test_face_connectivity_of_a_box_is_aligned():
    X, nbr, bc = bump_mesh(2)
    nb, nf, no, bc2 = W.face_connectivity(X)
    assert np.array_equal(nb, nbr) and np.array_equal(bc2, bc)
    inter = nb >= 0
    assert np.all(nf[inter] == np.broadcast_to(OPP, nb.shape)[inter]) and np.all(no[inter] == 0)


def test_operator_is_unchanged_by_turning_local_axes():
    p = 3
    X0, nbr0, bc0 = bump_mesh(p)
    X1 = turned(X0, 5)
    nbr, nf, no, bc = W.face_connectivity(X1)
    m0 = Mesh(p, X0, nbr0, bc0, kappa=1.0, mu_star=3.0)
    m1 = Mesh(p, X1, nbr, bc, kappa=1.0, mu_star=3.0, nbr_face=nf, nbr_orient=no)
    assert m1.oriented and set(np.unique(no[nbr >= 0])) == set(range(8))
    perm = node_perm(X0, X1)
    u = np.random.default_rng(1).standard_normal(m0.n_dof())
    A0 = oop.apply(m0, u).ravel()
    A1 = oop.apply(m1, u[perm]).ravel()
    assert np.abs(A1 - A0[perm]).max() < 1e-12 * np.abs(A0).max()
    assert np.isclose(np.sort(m1.mu.ravel()), np.sort(m0.mu.ravel()), rtol=1e-12).all()


def test_topology_schwarz_is_the_structured_one_on_a_regular_mesh():
    p = 3
    X, nbr, bc = bump_mesh(p)
    m = Mesh(p, X, nbr, bc, kappa=1.0)
    r = np.random.default_rng(2).standard_normal(m.n_dof())
    for weighting in ('quintic', 'plain'):
        zs = Schwarz(m, 1, weighting).apply(r)
        T = TopoSchwarz(m, 1, weighting)
        assert np.array_equal(T.apply(r), zs)
        assert all(set(sd['kinds'].values()) <= {'own', 'face', 'map'} for sd in T.sub)
    assert np.all(T.C is None or T.C == 1.0)


def test_topology_schwarz_is_unchanged_by_turning_local_axes():
    p = 2
    X0, nbr0, bc0 = bump_mesh(p)
    X1 = turned(X0, 7)
    nbr, nf, no, bc = W.face_connectivity(X1)
    m0 = Mesh(p, X0, nbr0, bc0, kappa=1.0)
    m1 = Mesh(p, X1, nbr, bc, kappa=1.0, nbr_face=nf, nbr_orient=no)
    perm = node_perm(X0, X1)
    r = np.random.default_rng(3).standard_normal(m0.n_dof())
    z0 = Schwarz(m0, 1).apply(r).ravel()
    z1 = TopoSchwarz(m1, 1).apply(r[perm]).ravel()
    assert np.abs(z1 - z0[perm]).max() < 1e-12 * np.abs(z0).max()


def _wrap_close(a, b, period):
    d = a - b
    if period is not None:
        d = d - period * np.round(d / period)
    return np.abs(d).max(axis=-1) < 1e-10


def test_diamond_blocks_follow_the_elements_around_edges_and_vertices():
    """Periodic diamond mesh (no boundary, every ring closed): an edge block is mapped exactly when
    four elements share the edge, zero-filled when three do, merged when more do, and the merged
    nodes belong to the surplus elements; vertex blocks likewise from the elements at the vertex."""
    p, period = 2, 1.0
    X, nbr, nf, no, bc = diamond(p, nc=3, layers=3, periodic=True)
    m = Mesh(p, X, nbr, bc, nbr_face=nf, nbr_orient=no)
    T = TopoSchwarz(m, 1)
    n, E = m.n, m.E
    corners = X[:, :, ::n - 1, ::n - 1, ::n - 1].reshape(E, 3, 8).transpose(0, 2, 1)   # (E, 8, 3)

    def sharing(points):
        """Elements that have every one of `points` among their corners."""
        out = set()
        for x in range(E):
            if all(np.any(_wrap_close(corners[x], q[None, :], period)) for q in points):
                out.add(x)
        return out

    valences = set()
    for sd in T.sub:
        e = sd['e']
        fnb = {(a, s): int(nbr[e, 2 * a + s]) for a in range(3) for s in (0, 1)}
        n3, n2, n1 = sd['shape']
        qs = [np.array([dl * n + l for (dl, l) in sd['v'][d]['nodes']]) for d in range(3)]
        q = np.stack([qs[0][sd['slot'] % n1], qs[1][(sd['slot'] // n1) % n2], qs[2][sd['slot'] // (n1 * n2)]], 1)
        slot_blk = (q >= n).astype(int) - (q < 0).astype(int)
        for blk, kind in sd['kinds'].items():
            nz = [a for a in range(3) if blk[a]]
            if len(nz) < 2:
                continue
            side = {a: (1 if blk[a] > 0 else 0) for a in nz}
            # the corner nodes of e on the edge or vertex
            pts = []
            for c in range(8):
                q = (c & 1, (c >> 1) & 1, c >> 2)
                if all(q[a] == side[a] for a in nz):
                    pts.append(X[e, :, q[2] * (n - 1), q[1] * (n - 1), q[0] * (n - 1)])
            around = sharing(pts) - {e}
            faces = {fnb[(a, side[a])] for a in nz}
            if len(nz) == 2:
                valences.add(len(around) + 1)
                surplus = around - faces
                expect = 'map' if len(around) + 1 == 4 else ('zero' if not surplus else 'merge')
            else:
                edge_elems = set()
                for a, b in ((0, 1), (0, 2), (1, 2)):
                    pe = [X[e, :, q[2] * (n - 1), q[1] * (n - 1), q[0] * (n - 1)]
                          for q in [(c & 1, (c >> 1) & 1, c >> 2) for c in range(8)]
                          if q[a] == side[a] and q[b] == side[b]]
                    edge_elems |= sharing(pe) - {e}
                surplus = around - faces - edge_elems
                regular = len(around) + 1 == 8 and len(surplus) == 1
                expect = 'map' if regular else ('zero' if not surplus else 'merge')
            assert kind == expect, (e, blk, kind, expect, len(around))
            if kind == 'merge':
                # the merged nodes belong to exactly the surplus elements
                inb = np.all(slot_blk == np.array(blk), axis=1)
                assert set((sd['gidx'][inb] // n ** 3).tolist()) == surplus, (e, blk)
    assert {3, 4, 8} <= valences


@pytest.mark.parametrize('periodic', [False, True])
def test_diamond_innermost_nodes_are_the_elements_boundary_nodes(periodic):
    p = 3
    X, nbr, nf, no, bc = diamond(p, nc=2, layers=3, periodic=periodic)
    m = Mesh(p, X, nbr, bc, nbr_face=nf, nbr_orient=no)
    T = TopoSchwarz(m, 1)
    n = m.n
    Xf = X.transpose(0, 2, 3, 4, 1).reshape(-1, 3)
    period = 1.0 if periodic else None
    checked = 0
    for sd in T.sub:
        e = sd['e']
        n3, n2, n1 = sd['shape']
        qs = [np.array([dl * n + l for (dl, l) in sd['v'][d]['nodes']]) for d in range(3)]
        s1, s2, s3 = sd['slot'] % n1, (sd['slot'] // n1) % n2, sd['slot'] // (n1 * n2)
        q = np.stack([qs[0][s1], qs[1][s2], qs[2][s3]], axis=1)
        inner = np.all((q >= -1) & (q <= n), axis=1) & ~np.all((q >= 0) & (q < n), axis=1)
        qc = np.clip(q[inner], 0, n - 1)
        own = Xf[e * n ** 3 + (qc[:, 2] * n + qc[:, 1]) * n + qc[:, 0]]
        assert np.all(_wrap_close(Xf[sd['gidx'][inner]], own, period))
        checked += int(inner.sum())
    assert checked > 1000


def _cg(apply, b, tol=1e-11, maxit=3000):
    x = np.zeros_like(b)
    r = b.copy()
    d = r.copy()
    rr = r @ r
    for _ in range(maxit):
        q = apply(d)
        a = rr / (d @ q)
        x += a * d
        r -= a * q
        rn = r @ r
        if np.sqrt(rn) <= tol * np.sqrt(b @ b):
            break
        d = r + (rn / rr) * d
        rr = rn
    return x


def test_diamond_operator_is_symmetric_and_converges_spectrally():
    errs = []
    k = np.pi
    for p in (2, 3):
        X, nbr, nf, no, bc = diamond(p)
        m = Mesh(p, X, nbr, bc, mu_star=5.0, nbr_face=nf, nbr_orient=no)
        rng = np.random.default_rng(p)
        x, y = rng.standard_normal((2, m.n_dof()))
        Ax = oop.apply(m, x).ravel()
        Ay = oop.apply(m, y).ravel()
        assert abs(y @ Ax - x @ Ay) < 1e-12 * np.abs(Ax).max() * np.abs(y).sum()
        assert x @ Ax > 0
        uex = np.sin(k * X[:, 0]) * np.sin(k * X[:, 1]) * np.sin(k * X[:, 2])
        b = oop.rhs(m, 3 * k * k * uex, uD=np.zeros_like(uex)).ravel()
        u = _cg(lambda v: oop.apply(m, v).ravel(), b)
        errs.append(oop.l2_error(m, u, uex))
    assert errs[1] < errs[0] / 10 and errs[1] < 1e-3, errs


def test_diamond_fas_converges_with_scg_and_was_does_not():
    """Sec. 6.2.4: on the diamond mesh the tensor-product subdomains are distorted and WAS-based
    cycles fail, while SCG smoothing still converges."""
    p = 3
    X, nbr, nf, no, bc = diamond(p)
    levels = osv.build_levels(p, X, nbr, bc, kappa=1.0, mu_star=5.0, nbr_face=nf, nbr_orient=no)
    n = p + 1
    b = np.random.default_rng(6).uniform(-1, 1, (len(X), n, n, n))
    _, h = osv.solve(levels, np.zeros_like(b), b, osv.Options('scg', 8, 4), max_cycles=12, rtol=1e-10)
    assert h[-1] <= 1e-10 and len(h) - 1 <= 10, h
    _, hw = osv.solve(levels, np.zeros_like(b), b, osv.Options('was', 2, 2), max_cycles=4, rtol=1e-10)
    assert hw[-1] > 1.0, hw
