"""Schwarz subdomains on unstructured hexahedral meshes (oracle; test infrastructure only).

Sec. 4.3.1, design principles 1-6 and 8-10, with the neighbour data of Sec. 5.1 (neighbour,
related face, relative orientation per face).  Each element-centred subdomain is the tile of
the structured case (the element plus m node layers from each interior side), but its nodes
are found by walking across oriented faces:

* face blocks take the face neighbour's m layers through the orientation;
* an edge block takes the edge neighbour's nodes when the elements around the edge form a
  closed ring of four (the regular case, a one-to-one mapping); with fewer elements it is
  zero-filled; with more (or an open ring), the surplus elements' nodes on the edge itself,
  the innermost ones, are averaged into the block's innermost row and the rest is zero;
* a vertex block likewise: mapped when exactly one element around the vertex is left after
  the element, its face neighbours and the elements around its three edges there, and all
  six walking orders reach it with the same node map; zero-filled when none is left; else
  the vertex nodes of the elements left are averaged into the innermost slot.

R_s is the restriction-and-merge operator: a merged slot gathers the mean of its k nodes and
hands its correction back with weight 1/k to each.  The surrogate, its fast-diagonalisation
solve and the tensor-product weights are those of the structured case (oracle.schwarz).

Readings (Sec. 4.3.1 is terse here):
* "innermost" edge or vertex nodes are the surplus elements' own nodes on the shared edge or
  vertex; they go to the slot of the regular edge or vertex neighbour's node there;
* the combined correction is normalised, z = C^-1 sum_s R_s^T W_s A~_s^-1 R_s r with
  C = sum_s R_s^T W_s R_s 1 (quintic weights only), as for the degree jumps of mixed meshes:
  zero fill and merging break the partition of unity.  On a regular mesh C = 1;
* the optional inclusion of irregular edge nodes next to face neighbours (item 7) is not
  taken.
"""
import itertools

import numpy as np

from .schwarz import variant_1d, surrogate_coefficients, side_codes

# face-node layout (first axis, second axis) of face phi, axes as 0 = xi_1, 1 = xi_2, 2 = xi_3
LAYOUT = {0: (2, 1), 1: (2, 1), 2: (2, 0), 3: (2, 0), 4: (1, 0), 5: (1, 0)}


def cross(mesh, e, phi, q):
    """Points q (..., 3) in e's extended node coordinates (integers; the neighbour across
    face phi holds the layers n, n+1, ... beyond the + face and -1, -2, ... beyond the - face)
    in the neighbour's own node coordinates.  Returns (neighbour, points, axis map), where the
    axis map sends each of e's axes to the neighbour's axis along which it runs."""
    n = mesh.n
    en = int(mesh.nbr[e, phi])
    nf = int(mesh.nbr_face[e, phi])
    o = int(mesh.nbr_orient[e, phi])
    c, s = phi >> 1, phi & 1
    c2, s2 = nf >> 1, nf & 1
    q = np.asarray(q, dtype=np.int64)
    l = q[..., c] - n if s else -1 - q[..., c]          # layer counted from the shared face
    out = np.empty_like(q)
    out[..., c2] = (n - 1 - l) if s2 else l
    fa, fb = LAYOUT[phi]
    ga, gb = LAYOUT[nf]
    a, b = q[..., fa], q[..., fb]
    x, y = (b, a) if o & 1 else (a, b)
    out[..., ga] = n - 1 - x if o & 2 else x
    out[..., gb] = n - 1 - y if o & 4 else y
    amap = [0, 0, 0]
    amap[c] = c2
    amap[fa], amap[fb] = (gb, ga) if o & 1 else (ga, gb)
    return en, out, amap


def locate(mesh, e, q, order):
    """Walk the points q of one block of e's subdomain (all outside e along the same axes)
    across faces in the given order of e's axes.  Returns (element, points) or None at a
    boundary."""
    n = mesh.n
    cur, pts = e, np.asarray(q, dtype=np.int64)
    ax = [0, 1, 2]
    for c in order:
        a = ax[c]
        v = pts.reshape(-1, 3)[0, a]
        if 0 <= v < n:
            continue
        phi = 2 * a + (1 if v >= n else 0)
        if mesh.nbr[cur, phi] < 0:
            return None
        cur, pts, amap = cross(mesh, cur, phi, pts)
        ax = [amap[x] for x in ax]
    return cur, pts


def _onto_face(mesh, e, phi, pts):
    """Points of e on face phi (inside e) -> the same physical nodes of the neighbour."""
    en, q, _ = cross(mesh, e, phi, pts)
    nf = int(mesh.nbr_face[e, phi])
    q[..., nf >> 1] = mesh.n - 1 if nf & 1 else 0
    return en, q


def _ends(mesh, pts):
    """Axes along which all of pts sit on one end of the element: {axis: side}."""
    n = mesh.n
    P = pts.reshape(-1, 3)
    out = {}
    for a in range(3):
        if np.all(P[:, a] == 0):
            out[a] = 0
        elif np.all(P[:, a] == n - 1):
            out[a] = 1
    return out


def edge_ring(mesh, e, f1, f2):
    """Elements around the edge of e shared by faces f1 and f2 (each (axis, side)).

    Returns (side1, side2, closed): side1 walks from e across f1 around the edge, side2 across
    f2; each is a list of (element, edge nodes (n, 3) ordered like e's edge nodes).  For a
    closed ring side2 is empty and side1 ends with the neighbour across f2."""
    n = mesh.n
    c3 = 3 - f1[0] - f2[0]
    pts0 = np.zeros((n, 3), dtype=np.int64)
    pts0[:, f1[0]] = n - 1 if f1[1] else 0
    pts0[:, f2[0]] = n - 1 if f2[1] else 0
    pts0[:, c3] = np.arange(n)

    def walk(first, other):
        seq = []
        cur, pts, fc = e, pts0, first
        for _ in range(64):
            phi = 2 * fc[0] + fc[1]
            if mesh.nbr[cur, phi] < 0:
                return seq, False
            en, q = _onto_face(mesh, cur, phi, pts)
            if en == e and np.array_equal(q, pts0):
                return seq, True
            seq.append((en, q))
            entry = int(mesh.nbr_face[cur, phi]) >> 1
            ends = _ends(mesh, q)
            nxt = [a for a in ends if a != entry]
            if len(nxt) != 1:
                raise ValueError('edge walk lost the edge')
            cur, pts, fc = en, q, (nxt[0], ends[nxt[0]])
        raise ValueError('edge ring longer than 64 elements')

    side1, closed = walk(f1, f2)
    if closed:
        return side1, [], True
    side2, _ = walk(f2, f1)
    return side1, side2, False


def vertex_star(mesh, e, corner):
    """Elements around the vertex of e at corner (s1, s2, s3): {element: its vertex node}."""
    n = mesh.n
    q0 = np.array([n - 1 if s else 0 for s in corner], dtype=np.int64)
    seen = {e: q0}
    todo = [(e, q0)]
    while todo:
        cur, q = todo.pop()
        for a in range(3):
            phi = 2 * a + (1 if q[a] == n - 1 else 0)
            if mesh.nbr[cur, phi] < 0:
                continue
            en, qn = _onto_face(mesh, cur, phi, q)
            if en not in seen:
                seen[en] = qn
                todo.append((en, qn))
    return seen


class TopoSchwarz:
    """Weighted overlapping Schwarz method on an unstructured mesh (oriented faces, irregular
    edges and vertices), with the interface of oracle.schwarz.Schwarz."""

    def __init__(self, mesh, m, weighting='quintic', subset=None):
        """subset: build only these elements' subdomains (sampled checks on large meshes; the
        weight sums, and so z, are then exact at the nodes that only these subdomains reach,
        e.g. the nodes of an element when every element sharing a vertex with it is in the
        subset)."""
        self.mesh, self.m, self.weighting = mesh, m, weighting
        self.g = surrogate_coefficients(mesh)
        self.variants = {}
        self.sub = [self._subdomain(int(e)) for e in (range(mesh.E) if subset is None else subset)]
        if weighting == 'quintic':
            C = np.zeros(mesh.n_dof())
            for sd in self.sub:
                np.add.at(C, sd['gidx'], sd['coef'] * sd['W'].ravel()[sd['slot']])
            self.C = C
        else:
            self.C = None

    def _variant(self, lr):
        if lr not in self.variants:
            self.variants[lr] = variant_1d(self.mesh.p, self.m, lr[0], lr[1], self.mesh.mu_star, self.weighting)
        return self.variants[lr]

    # -- classification of the edge and vertex blocks of element e --------------------------
    def _edge(self, e, f1, f2):
        side1, side2, closed = edge_ring(self.mesh, e, f1, f2)
        ring = side1 + side2
        faces = {side1[0][0] if side1 else None, (side1[-1][0] if closed else (side2[0][0] if side2 else None))}
        if closed:
            others = side1[1:-1]
        else:
            others = side1[1:] + side2[1:]
        others = [(x, q) for (x, q) in others if x not in faces and x != e]
        ring_elems = {x for x, _ in ring}
        if closed and len(side1) == 3 and len(others) == 1:
            return 'map', others, ring_elems
        if not others:
            return 'zero', [], ring_elems
        return 'merge', others, ring_elems

    def _vertex(self, e, corner, edge_elems):
        star = vertex_star(self.mesh, e, corner)
        faces = set()
        for a in range(3):
            nb = self.mesh.nbr[e, 2 * a + corner[a]]
            if nb >= 0:
                faces.add(int(nb))
        others = [(x, q) for x, q in star.items() if x != e and x not in faces and x not in edge_elems]
        return others

    def _subdomain(self, e):
        mesh, n = self.mesh, self.mesh.n
        key = side_codes(mesh, e)
        v = [self._variant(key[d]) for d in range(3)]
        qs = [np.array([dl * n + l for (dl, l) in v[d]['nodes']]) for d in range(3)]
        blocks = [np.array([dl for (dl, _) in v[d]['nodes']]) for d in range(3)]
        n1, n2, n3 = len(qs[0]), len(qs[1]), len(qs[2])
        S3, S2, S1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing='ij')
        slot_all = ((S3 * n2 + S2) * n1 + S1).ravel()
        Q = np.stack([qs[0][S1.ravel()], qs[1][S2.ravel()], qs[2][S3.ravel()]], axis=1)
        B = np.stack([blocks[0][S1.ravel()], blocks[1][S2.ravel()], blocks[2][S3.ravel()]], axis=1)
        slot, gidx, coef = [], [], []
        kinds = {}

        def put(sl, el, pts, c):
            pts = np.asarray(pts).reshape(-1, 3)
            slot.append(np.atleast_1d(sl))
            gidx.append(el * n ** 3 + (pts[:, 2] * n + pts[:, 1]) * n + pts[:, 0])
            coef.append(np.full(len(pts), c))

        edge_cache = {}
        for blk in sorted({tuple(b) for b in B}):
            sel = np.nonzero(np.all(B == blk, axis=1))[0]
            nz = [a for a in range(3) if blk[a] != 0]
            pts = Q[sel]
            if len(nz) <= 1:
                res = locate(mesh, e, pts, nz)
                if res is None:
                    raise ValueError('face block beyond a boundary')
                put(slot_all[sel], res[0], res[1], 1.0)
                kinds[blk] = 'face' if nz else 'own'
                continue
            if len(nz) == 2:
                f1, f2 = (nz[0], 1 if blk[nz[0]] > 0 else 0), (nz[1], 1 if blk[nz[1]] > 0 else 0)
                kind, others, ring = self._edge(e, f1, f2)
                edge_cache[(f1, f2)] = ring
                kinds[blk] = kind
                if kind == 'map':
                    r1 = locate(mesh, e, pts, nz)
                    r2 = locate(mesh, e, pts, nz[::-1])
                    if r1 is None or r2 is None or r1[0] != r2[0] or not np.array_equal(r1[1], r2[1]):
                        kind = kinds[blk] = 'merge'
                    else:
                        put(slot_all[sel], r1[0], r1[1], 1.0)
                        continue
                if kind == 'merge':
                    c3 = 3 - nz[0] - nz[1]
                    inner = [(n if blk[a] > 0 else -1) for a in nz]
                    row = sel[(pts[:, nz[0]] == inner[0]) & (pts[:, nz[1]] == inner[1])]
                    t = Q[row, c3]                   # position along the edge, 0..n-1
                    for x, qe in others:
                        put(slot_all[row], x, qe[t], 1.0 / len(others))
                continue
            corner = tuple(1 if blk[a] > 0 else 0 for a in range(3))
            edge_elems = set()
            for a, b in ((0, 1), (0, 2), (1, 2)):
                f1, f2 = (a, corner[a]), (b, corner[b])
                ring = edge_cache.get((f1, f2))
                if ring is None:
                    ring = self._edge(e, f1, f2)[2]
                edge_elems |= ring
            others = self._vertex(e, corner, edge_elems)
            if not others:
                kinds[blk] = 'zero'
                continue
            if len(others) == 1:
                res = [locate(mesh, e, pts, list(o)) for o in itertools.permutations(range(3))]
                if all(r is not None for r in res) and all(r[0] == others[0][0] and np.array_equal(r[1], res[0][1])
                                                           for r in res):
                    put(slot_all[sel], res[0][0], res[0][1], 1.0)
                    kinds[blk] = 'map'
                    continue
            inner = [(n if blk[a] > 0 else -1) for a in range(3)]
            one = sel[np.all(pts == inner, axis=1)]
            for x, qv in others:
                put(one, x, qv, 1.0 / len(others))
            kinds[blk] = 'merge'
        Wt = v[2]['W'][:, None, None] * v[1]['W'][None, :, None] * v[0]['W'][None, None, :]
        return dict(e=e, v=v, shape=(n3, n2, n1), W=Wt, kinds=kinds,
                    slot=np.concatenate(slot), gidx=np.concatenate(gidx), coef=np.concatenate(coef))

    # -- application ------------------------------------------------------------------------
    def local_solve(self, sd, rs):
        """Fast diagonalisation (S3 x S2 x S1) D^-1 (S3^T x S2^T x S1^T) rs of one subdomain."""
        v, g = sd['v'], self.g[sd['e']]
        S1, S2, S3 = v[0]['S'], v[1]['S'], v[2]['S']
        t = np.einsum('kc,jb,ia,kji->cba', S3, S2, S1, rs)
        Dg = (g[0] + g[1] * v[0]['lam'][None, None, :] + g[2] * v[1]['lam'][None, :, None]
              + g[3] * v[2]['lam'][:, None, None])
        return np.einsum('kc,jb,ia,cba->kji', S3, S2, S1, t / Dg)

    def gather(self, sd, r):
        """R_s r on the subdomain tile (merged slots take the mean, zero-filled slots zero)."""
        rs = np.zeros(int(np.prod(sd['shape'])))
        np.add.at(rs, sd['slot'], sd['coef'] * r[sd['gidx']])
        return rs.reshape(sd['shape'])

    def apply(self, r, elements=None):
        """z = C^-1 sum_s R_s^T W_s A~_s^-1 R_s r (quintic weights; plain weights: C = 1)."""
        r = np.asarray(r, dtype=np.float64).ravel()
        z = np.zeros_like(r)
        for sd in self.sub:
            if elements is not None and sd['e'] not in set(int(x) for x in elements):
                continue
            du = (sd['W'] * self.local_solve(sd, self.gather(sd, r))).ravel()
            np.add.at(z, sd['gidx'], sd['coef'] * du[sd['slot']])
        if self.C is not None:
            cov = self.C > 0                     # every node, unless only a subset is built
            z = np.where(cov, z / np.where(cov, self.C, 1.0), 0.0)
        return z.reshape(self.mesh.E, self.mesh.n, self.mesh.n, self.mesh.n)
