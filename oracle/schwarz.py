"""Weighted overlapping Schwarz method with fast diagonalisation (oracle; test infrastructure only).

Sec. 4.3.1.  For every element e an element-centred subdomain takes the whole
element plus m node layers from each neighbour across an interior side,
including edge and vertex neighbours.  The subdomain operator is replaced by
the tensor-product surrogate of eq. schwarz:tpo on a 3x3x3 patch of copies of
the element's surrogate cuboid, inverted by fast diagonalisation, and the
corrections are combined with tensor-product weights (eq. schwarz:correction).

Readings (the paper refers to other work for these):
* 1D matrices M, L of a face-condition variant: principal submatrix of the
  1D SIPG operator on a 3-element reference patch (element length 2, penalty
  mu_star p(p+1)/4) on the nodes (last m of the left element, all of the
  centre, first m of the right); a Dirichlet side has no overlap and carries
  the Dirichlet terms, a Neumann side has no overlap and no face term.
* Surrogate cuboid: linear Legendre coefficients a_b of the map, edge lengths
  2|a_b|, rescaled by (vol / prod)^(1/3) with vol = sum w J.
* Weights: on an interior side with overlap m, a node at normalised signed
  distance d from the shared face (positive inside the centre element) gets
  s((d + a) / (2a)), a = (1 + xi_m)/2, s(t) = 10t^3 - 15t^4 + 6t^5 clamped
  to [0, 1]; sides without overlap give weight 1.  This is a partition of unity.
"""
import numpy as np
import scipy.linalg

from .gll import gll, legendre
from .sipg1d import sipg_1d

FACE_OF = {(0, -1): 0, (0, 1): 1, (1, -1): 2, (1, 1): 3, (2, -1): 4, (2, 1): 5}


def surrogate_dx(mesh):
    """Edge lengths Delta x_b (E, 3) of the volume-preserving surrogate cuboid (Sec. 4.3.1, steps 1-3)."""
    p = mesh.p
    x, _ = gll(p)
    V = np.stack([legendre(i, x)[0] for i in range(p + 1)], axis=1)   # V[q, i] = L_i(x_q)
    Vinv = np.linalg.inv(V)
    # modal coefficients xh[e, coord, c3, c2, c1] of each coordinate
    xh = np.einsum('zk,yj,xi,eakji->eazyx', Vinv, Vinv, Vinv, mesh.X)
    # linear coefficient along xi_b: Legendre index 1 in direction b, 0 in the others
    a1 = xh[:, :, 0, 0, 1]
    a2 = xh[:, :, 0, 1, 0]
    a3 = xh[:, :, 1, 0, 0]
    ell = 2.0 * np.stack([np.linalg.norm(a1, axis=1), np.linalg.norm(a2, axis=1), np.linalg.norm(a3, axis=1)], axis=1)
    scale = (mesh.vol / np.prod(ell, axis=1)) ** (1.0 / 3.0)
    return ell * scale[:, None]


def surrogate_coefficients(mesh, dx=None):
    """g0 = kappa dx1 dx2 dx3 / 8, g_i = nu dx_j dx_k / (2 dx_i) (eq. schwarz:tpo), with the
    element's averaged nu (its own value: nu is constant per element)."""
    dx = surrogate_dx(mesh) if dx is None else dx
    nu = mesh.nu_e
    g0 = mesh.kappa * np.prod(dx, axis=1) / 8.0
    g1 = nu * dx[:, 1] * dx[:, 2] / (2.0 * dx[:, 0])
    g2 = nu * dx[:, 2] * dx[:, 0] / (2.0 * dx[:, 1])
    g3 = nu * dx[:, 0] * dx[:, 1] / (2.0 * dx[:, 2])
    return np.stack([g0, g1, g2, g3], axis=1)


def quintic(t):
    t = np.clip(t, 0.0, 1.0)
    return 10 * t ** 3 - 15 * t ** 4 + 6 * t ** 5


def variant_1d(p, m, left, right, mu_star, weighting='quintic'):
    """1D subdomain data of a face-condition variant (left, right) in {'i','d','n'}.
    weighting 'plain' gives W = 1 (plain additive Schwarz, no partition of unity).

    Returns dict with 'nodes' [(delta, local index)], diagonal mass 'M', stiffness 'L',
    eigenvectors 'S' (S^T M S = I), eigenvalues 'lam' (S^T L S = diag lam) and weights 'W'.
    """
    n = p + 1
    elems = []
    if left == 'i':
        elems.append(-1)
    elems.append(0)
    if right == 'i':
        elems.append(1)
    K = len(elems)
    end_l = 'd' if left == 'd' else 'n'
    end_r = 'd' if right == 'd' else 'n'
    Mg, Lg = sipg_1d(p, K, 2.0, mu_star, end_l, end_r)
    nodes, sel = [], []
    for pos, dlt in enumerate(elems):
        if dlt == -1:
            locs = range(n - m, n)
        elif dlt == 1:
            locs = range(0, m)
        else:
            locs = range(n)
        for l in locs:
            nodes.append((dlt, l))
            sel.append(pos * n + l)
    sel = np.array(sel, dtype=int)
    L = Lg[np.ix_(sel, sel)]
    M = np.diag(Mg)[sel]
    lam, S = scipy.linalg.eigh(L, np.diag(M))
    # weights
    x, _ = gll(p)
    a = 0.5 * (1.0 + x[m]) if m > 0 else None
    W = np.ones(len(nodes))
    for s, (dlt, l) in enumerate(nodes):
        wl = wr = 1.0
        if left == 'i' and m > 0:
            d = 0.5 * (1.0 + x[l]) if dlt == 0 else (-0.5 * (1.0 - x[l]) if dlt == -1 else None)
            if d is not None:
                wl = quintic((d + a) / (2 * a))
        if right == 'i' and m > 0:
            d = 0.5 * (1.0 - x[l]) if dlt == 0 else (-0.5 * (1.0 + x[l]) if dlt == 1 else None)
            if d is not None:
                wr = quintic((d + a) / (2 * a))
        W[s] = wl * wr
    if weighting == 'plain':
        W = np.ones(len(nodes))
    return dict(nodes=nodes, M=M, L=L, S=S, lam=lam, W=W)


def side_codes(mesh, e):
    """Face condition per direction: (left, right) each 'i' interior, 'd' Dirichlet, 'n' Neumann."""
    out = []
    for d in range(3):
        pair = []
        for s in (0, 1):
            phi = 2 * d + s
            if mesh.nbr[e, phi] >= 0:
                pair.append('i')
            else:
                pair.append('d' if mesh.bc[e, phi] == 1 else 'n')
        out.append(tuple(pair))
    return tuple(out)


def neighbour_27(mesh, e, delta):
    """Element at offset delta = (d1, d2, d3) in {-1,0,1}^3, by walking face neighbours."""
    cur = e
    for d in range(3):
        if delta[d] != 0:
            cur = mesh.nbr[cur, FACE_OF[(d, delta[d])]]
            if cur < 0:
                return -1
    return cur


class Schwarz:
    """Precomputed subdomain data of one mesh level with overlap m."""

    def __init__(self, mesh, m, weighting='quintic'):
        self.mesh, self.m, self.weighting = mesh, m, weighting
        self.g = surrogate_coefficients(mesh)
        self.variants = {}
        self.groups = {}
        n = mesh.n
        for e in range(mesh.E):
            key = side_codes(mesh, e)
            self.groups.setdefault(key, []).append(e)
        for key, els in self.groups.items():
            v = [self._variant(key[d]) for d in range(3)]
            els = np.array(els)
            # global indices of the subdomain nodes: idx[g, s3, s2, s1]
            n1, n2, n3 = (len(v[d]['nodes']) for d in range(3))
            idx = np.empty((len(els), n3, n2, n1), dtype=np.int64)
            for s3, (d3, l3) in enumerate(v[2]['nodes']):
                for s2, (d2, l2) in enumerate(v[1]['nodes']):
                    for s1, (d1, l1) in enumerate(v[0]['nodes']):
                        nb = np.array([neighbour_27(mesh, e, (d1, d2, d3)) for e in els])
                        assert np.all(nb >= 0)
                        idx[:, s3, s2, s1] = nb * n ** 3 + (l3 * n + l2) * n + l1
            Wt = v[2]['W'][:, None, None] * v[1]['W'][None, :, None] * v[0]['W'][None, None, :]
            self.groups[key] = dict(els=els, idx=idx, v=v, W=Wt)

    def _variant(self, lr):
        if lr not in self.variants:
            self.variants[lr] = variant_1d(self.mesh.p, self.m, lr[0], lr[1], self.mesh.mu_star, self.weighting)
        return self.variants[lr]

    def fd_solve(self, grp, rs, sel=None):
        """Fast diagonalisation: (S3 x S2 x S1) D^-1 (S3^T x S2^T x S1^T) rs for a batch."""
        v = grp['v']
        S1, S2, S3 = v[0]['S'], v[1]['S'], v[2]['S']
        g = self.g[grp['els'] if sel is None else grp['els'][sel]]
        t = np.einsum('kc,jb,ia,ekji->ecba', S3, S2, S1, rs)
        Dg = (g[:, 0, None, None, None]
              + g[:, 1, None, None, None] * v[0]['lam'][None, None, None, :]
              + g[:, 2, None, None, None] * v[1]['lam'][None, None, :, None]
              + g[:, 3, None, None, None] * v[2]['lam'][None, :, None, None])
        t = t / Dg
        return np.einsum('kc,jb,ia,ecba->ekji', S3, S2, S1, t)

    def apply(self, r, elements=None):
        """z = sum_e R_s^T W^e (A~_s^e)^-1 R_s r (eq. schwarz:correction).

        With `elements`, only those subdomains contribute (for sampled checks).
        """
        r = np.asarray(r, dtype=np.float64).ravel()
        z = np.zeros_like(r)
        want = None if elements is None else set(int(e) for e in elements)
        for key, grp in self.groups.items():
            if want is None:
                sel = None
                idx = grp['idx']
            else:
                sel = np.array([i for i, e in enumerate(grp['els']) if int(e) in want], dtype=int)
                if len(sel) == 0:
                    continue
                idx = grp['idx'][sel]
            du = self.fd_solve(grp, r[idx], sel)
            np.add.at(z, idx.ravel(), (grp['W'][None] * du).ravel())
        return z.reshape(self.mesh.E, self.mesh.n, self.mesh.n, self.mesh.n)

    def subdomain_indices(self, e):
        for grp in self.groups.values():
            hit = np.nonzero(grp['els'] == e)[0]
            if len(hit):
                return grp['idx'][hit[0]], grp
        raise KeyError(e)


def overlap_layers(p, delta):
    """Reading of Sec. 4.3.1 item 3: m = number of neighbour GLL nodes with (1+xi)/2 <= delta."""
    x, _ = gll(p)
    return int(np.sum(0.5 * (1.0 + x) <= delta + 1e-14))


def local_pair(mesh, schwarz, A_dense, r, e):
    """Learned-correction training pair of element e (not in the paper; test infrastructure):
    subdomain residual r_s = R_s r, its FD solve and the exact local solve (R_s A R_s^T)^-1 r_s
    by dense Cholesky of the principal submatrix of the assembled operator."""
    idx, grp = schwarz.subdomain_indices(e)
    i = idx.ravel()
    rs = np.asarray(r).ravel()[i]
    As = A_dense[np.ix_(i, i)]
    exact = scipy.linalg.cho_solve(scipy.linalg.cho_factor(As), rs)
    sel = np.nonzero(grp['els'] == e)[0]
    fd = schwarz.fd_solve(grp, rs.reshape((1,) + idx.shape), sel).ravel()
    return idx.shape, rs, fd, exact


def linear_jacobian(mesh):
    """[a1 a2 a3] / det^(1/3) per element (E, 3, 3): the linear Legendre coefficients of the map."""
    from .gll import gll as _gll
    p = mesh.p
    x, _ = _gll(p)
    V = np.stack([legendre(i, x)[0] for i in range(p + 1)], axis=1)
    Vinv = np.linalg.inv(V)
    xh = np.einsum('zk,yj,xi,eakji->eazyx', Vinv, Vinv, Vinv, mesh.X)
    A = np.stack([xh[:, :, 0, 0, 1], xh[:, :, 0, 1, 0], xh[:, :, 1, 0, 0]], axis=2)   # A[e][a][b]
    return A / np.cbrt(np.linalg.det(A))[:, None, None]
