"""h-coarsening of box meshes: levels of 2x2x2 merged elements at a fixed degree
(oracle; test infrastructure only).

Sec. 3.1 builds the multilevel mesh by successive h- or p-refinements; with h-refinement
every element of level l is subdivided regularly into eight children on level l+1.  Sec. 3.2
defines the transfers: the coarse-to-fine interpolation I is the embedded interpolation (exact,
the spaces are nested), the residual restriction is R = I^T, and the solution projection P is
the embedded interpolation of the children's solution at the parent's GLL nodes, averaged at
shared target nodes (those on the planes between children, present for even p).

Readings:
* A box mesh of nx x ny x nz elements numbered e = ex + nx (ey + ny ez) coarsens when every
  dimension is even: the children of parent (Ex, Ey, Ez) are (2Ex + bx, 2Ey + by, 2Ez + bz),
  child (bx, by, bz) covering the parent's reference sub-cube of xi_d in [-1, 0] (b = 0) or
  [0, 1] (b = 1).
* The parent's faces take their neighbours (and boundary codes) from the children on them.
* The parent's geometry is P applied to the children's nodal coordinates (the isoparametric
  map of the children evaluated at the parent's nodes).
* With h-only coarsening the root is the coarsest h-level at the fine degree, solved by SCG.
"""
import numpy as np

from .gll import gll, lagrange_eval
from .mesh import Mesh, OPPOSITE


def child_matrices(p):
    """1D matrices of the two children of an interval, b = 0 (left) and 1 (right):
    I[b][i, j] = l_j(xi_P(i)), the parent's basis at child node i, xi_P = (xi_c + 2b - 1)/2;
    P[b][i, j] = w_b(i) l_j(2 xi_i - (2b - 1)), the child's basis at parent node i, with the
    weight w_b(i) = 1 in the child's open half, 1/2 at the shared midpoint, 0 elsewhere."""
    x, _ = gll(p)
    I, P = [], []
    for b in (0, 1):
        I.append(lagrange_eval(x, (x + (2 * b - 1)) / 2.0))
        mid = np.abs(x) < 1e-14
        inside = (x < 0) if b == 0 else (x > 0)
        wgt = np.where(mid, 0.5, np.where(inside, 1.0, 0.0))
        xc = np.clip(2.0 * x - (2 * b - 1), -1.0, 1.0)     # rows outside the half get weight 0
        P.append(wgt[:, None] * lagrange_eval(x, xc))
    return I, P


def _t3(Tz, Ty, Tx, u):
    return np.einsum('ck,bj,ai,...kji->...cba', Tz, Ty, Tx, u)


class HTransfer:
    """Transfers between a fine box level (nx, ny, nz) and its 2x2x2-merged parent level."""

    def __init__(self, p, box):
        nx, ny, nz = box
        if nx % 2 or ny % 2 or nz % 2:
            raise ValueError('box dimensions must be even to coarsen')
        self.p, self.box = p, (nx, ny, nz)
        self.cbox = (nx // 2, ny // 2, nz // 2)
        NX, NY, NZ = self.cbox
        Ec = NX * NY * NZ
        self.children = np.empty((Ec, 8), dtype=np.int64)
        for E in range(Ec):
            Ex, Ey, Ez = E % NX, (E // NX) % NY, E // (NX * NY)
            for c in range(8):
                bx, by, bz = c & 1, (c >> 1) & 1, c >> 2
                self.children[E, c] = (2 * Ex + bx) + nx * ((2 * Ey + by) + ny * (2 * Ez + bz))
        self.I, self.P = child_matrices(p)

    def _bits(self, c):
        return c & 1, (c >> 1) & 1, c >> 2

    def prolong(self, uc):
        """I: parent -> children (E_f, n, n, n)."""
        n = self.p + 1
        uc = np.asarray(uc).reshape((-1, n, n, n))
        out = np.zeros((int(np.prod(self.box)), n, n, n))
        for c in range(8):
            bx, by, bz = self._bits(c)
            out[self.children[:, c]] = _t3(self.I[bz], self.I[by], self.I[bx], uc)
        return out

    def restrict(self, rf):
        """R = I^T: children -> parent."""
        n = self.p + 1
        rf = np.asarray(rf).reshape((-1, n, n, n))
        out = np.zeros((len(self.children), n, n, n))
        for c in range(8):
            bx, by, bz = self._bits(c)
            out += _t3(self.I[bz].T, self.I[by].T, self.I[bx].T, rf[self.children[:, c]])
        return out

    def project(self, uf):
        """P: the children's solution evaluated at the parent's nodes, averaged where shared."""
        n = self.p + 1
        uf = np.asarray(uf).reshape((-1, n, n, n))
        out = 0.0
        for c in range(8):
            bx, by, bz = self._bits(c)
            out = out + _t3(self.P[bz], self.P[by], self.P[bx], uf[self.children[:, c]])
        return out

    def coarsen_topology(self, nbr, bc):
        """Parent face neighbours and boundary codes from the children on each face."""
        NX, NY, _ = self.cbox
        nx, ny, _ = self.box
        Ec = len(self.children)
        nbrc = -np.ones((Ec, 6), dtype=np.int64)
        bcc = np.zeros((Ec, 6), dtype=np.int64)

        def parent(e):
            ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
            return ex // 2 + NX * (ey // 2 + NY * (ez // 2))

        for E in range(Ec):
            for phi in range(6):
                ax, side = phi >> 1, phi & 1
                c = side << ax                       # a child on that face
                ch = self.children[E, c]
                en = nbr[ch, phi]
                if en >= 0:
                    nbrc[E, phi] = parent(en)
                else:
                    bcc[E, phi] = bc[ch, phi]
        return nbrc, bcc


def build_hlevels(p, X, nbr, bc, box, h_levels, m=1, nu=1.0, kappa=0.0, mu_star=2.0, p_coarsen=False,
                  weighting='quintic'):
    """Level list (root first): h_levels 2x2x2 coarsenings of the box mesh at degree p, then, with
    p_coarsen, the p-levels max(1, p // 2) ... 1 of the coarsest h-mesh.  Every level carries
    `down`, the transfer to the next coarser level: an HTransfer or None (p-coarsening)."""
    from .solvers import Level, build_levels
    X = np.asarray(X, dtype=np.float64)
    nbr, bc = np.asarray(nbr), np.asarray(bc)
    nu = np.asarray(nu, dtype=np.float64)
    fine = []
    cur_box = tuple(box)
    for _ in range(h_levels):
        ht = HTransfer(p, cur_box)
        lv = Level(Mesh(p, X, nbr, bc, nu=nu, kappa=kappa, mu_star=mu_star), m, weighting)
        lv.down = ht
        fine.append(lv)
        X = np.stack([ht.project(X[:, a]) for a in range(3)], axis=1)
        if nu.ndim == 4:                     # a nodal coefficient follows the geometry
            nu = ht.project(nu)
        elif nu.ndim == 1:
            raise ValueError('h-coarsening takes a scalar or nodal nu')
        nbr, bc = ht.coarsen_topology(nbr, bc)
        cur_box = ht.cbox
    if p_coarsen:
        coarse = build_levels(p, X, nbr, bc, m=m, nu=nu, kappa=kappa, mu_star=mu_star, weighting=weighting)
        for lv in coarse:
            lv.down = None
    else:
        root = Level(Mesh(p, X, nbr, bc, nu=nu, kappa=kappa, mu_star=mu_star), m, weighting)
        root.down = None
        coarse = [root]
    return coarse + fine[::-1]


def dense_transfers(ht):
    """Dense (I, R, P) of an HTransfer for the brute-force pins."""
    n = ht.p + 1
    n3 = n ** 3
    Ef, Ec = int(np.prod(ht.box)), len(ht.children)
    I = np.zeros((Ef * n3, Ec * n3))
    P = np.zeros((Ec * n3, Ef * n3))
    for c in range(8):
        bx, by, bz = c & 1, (c >> 1) & 1, c >> 2
        Ic = np.kron(np.kron(ht.I[bz], ht.I[by]), ht.I[bx])
        Pc = np.kron(np.kron(ht.P[bz], ht.P[by]), ht.P[bx])
        for E in range(Ec):
            ch = ht.children[E, c]
            I[ch * n3:(ch + 1) * n3, E * n3:(E + 1) * n3] = Ic
            P[E * n3:(E + 1) * n3, ch * n3:(ch + 1) * n3] = Pc
    return I, I.T.copy(), P
