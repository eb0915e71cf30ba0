"""Isoparametric hexahedral mesh and its geometry (oracle; test infrastructure only).

Follows Sec. 2.2: each element has a map x = x^e(xi) from [-1,1]^3, given
isoparametrically by nodal coordinates at the GLL nodes of the element's
degree (Remark on basis functions).  Volume arrays are indexed
[e, k, j, i] with i along xi_1 (fastest), j along xi_2, k along xi_3.
Faces are numbered 0:-xi_1, 1:+xi_1, 2:-xi_2, 3:+xi_2, 4:-xi_3, 5:+xi_3.

Readings (where the paper is silent):
* surface measure and normal at a face node come from the face's own
  tangential derivatives (cross product), so both sides of an interior face
  see the same value;
* h_perp of an element at a face is vol(element) / area(face);
* the penalty on an interior face is mu_star times the average of
  p(p+1)/(2 h_perp) over the two sides (eq. helmholtz:dgm), on a Dirichlet
  face the one-sided value (the form itself carries the factor 2).
"""
import numpy as np

from .gll import gll, diff_matrix

OPPOSITE = np.array([1, 0, 3, 2, 5, 4])


def d_ref(D, u, c):
    """Reference derivative d/dxi_{c+1} of volume array(s) u[..., k, j, i]."""
    if c == 0:
        return np.einsum('im,...kjm->...kji', D, u)
    if c == 1:
        return np.einsum('jm,...kmi->...kji', D, u)
    return np.einsum('km,...mji->...kji', D, u)


def dT_ref(D, v, c):
    """Transpose of d_ref: (D_c^T v)."""
    if c == 0:
        return np.einsum('im,...kji->...kjm', D, v)
    if c == 1:
        return np.einsum('jm,...kji->...kmi', D, v)
    return np.einsum('km,...kji->...mji', D, v)


def face_view(V, phi):
    """View of the face-phi node layer of V[..., k, j, i].

    Layout of the face array: phi 0/1 -> (k, j); 2/3 -> (k, i); 4/5 -> (j, i).
    For two aligned neighbours the shared face has the same layout on both sides.
    """
    s = 0 if phi % 2 == 0 else -1
    if phi < 2:
        return V[..., :, :, s]
    if phi < 4:
        return V[..., :, s, :]
    return V[..., s, :, :]


def _tangential(D, F, phi):
    """(d/dxi_t1 F, d/dxi_t2 F) on a face array, (t1, t2) cyclic after the normal axis."""
    d_last = np.einsum('bm,...am->...ab', D, F)
    d_first = np.einsum('am,...mb->...ab', D, F)
    if phi < 2:      # normal xi_1: t1 = xi_2 (last axis), t2 = xi_3 (first axis)
        return d_last, d_first
    if phi < 4:      # normal xi_2: t1 = xi_3 (first), t2 = xi_1 (last)
        return d_first, d_last
    return d_last, d_first   # normal xi_3: t1 = xi_1 (last), t2 = xi_2 (first)


def orient_index(n, o):
    """Neighbour face-node indices (ap[a, b], bp[a, b]) of our face node (a, b) under the
    relative orientation o (Sec. 5.1 keeps one per face): bit 0 exchanges the two face axes,
    bits 1 and 2 then reverse the first and the second."""
    A, B = np.meshgrid(np.arange(n), np.arange(n), indexing='ij')
    x, y = (B, A) if o & 1 else (A, B)
    return (n - 1 - x if o & 2 else x), (n - 1 - y if o & 4 else y)


class Mesh:
    """Single-level conforming hex mesh of uniform degree p.

    X: (E, 3, n, n, n) nodal coordinates; nbr: (E, 6) neighbour ids (-1 = boundary);
    bc: (E, 6) boundary codes on boundary faces (1 Dirichlet, 2 Neumann).
    nbr_face, nbr_orient: (E, 6) the neighbour's face and the relative orientation code of
    `orient_index` (Sec. 5.1: neighbour, related face, relative orientation); None means aligned
    neighbours (face phi ^ 1, code 0).
    nu: the diffusivity (eq. helmholtz:pde), a positive scalar, one value per element or one
    value per node (E, n, n, n).  nu_n holds it per node, nu_e the element averages
    int_e nu dx / int_e dx taken with the GLL quadrature (the averaged coefficient of the
    Schwarz surrogate, Sec. 4.3.1).
    """

    def __init__(self, p, X, nbr, bc, nu=1.0, kappa=0.0, mu_star=2.0, nbr_face=None, nbr_orient=None):
        self.p, self.n = p, p + 1
        self.X = np.asarray(X, dtype=np.float64)
        self.E = self.X.shape[0]
        self.nbr = np.asarray(nbr, dtype=np.int64)
        self.bc = np.asarray(bc, dtype=np.int64)
        aligned_face = np.where(self.nbr >= 0, OPPOSITE[None, :], -1)
        self.nbr_face = aligned_face if nbr_face is None else np.where(self.nbr >= 0, np.asarray(nbr_face, dtype=np.int64), -1)
        self.nbr_orient = (np.zeros_like(self.nbr) if nbr_orient is None
                           else np.where(self.nbr >= 0, np.asarray(nbr_orient, dtype=np.int64), 0))
        self.oriented = bool(np.any(self.nbr_face != aligned_face) or np.any(self.nbr_orient != 0))
        n = self.n
        nu = np.asarray(nu, dtype=np.float64)
        if nu.ndim == 1:
            nu = nu[:, None, None, None]
        self.nu_n = np.broadcast_to(nu, (self.E, n, n, n)).copy()
        # the blade case's nu = 1 + cos cos cos vanishes at isolated points (Sec. 6.2.5): nodal
        # values may be zero, element averages may not
        if not np.all(self.nu_n >= 0):
            raise ValueError('nu must be non-negative')
        self.nu = float(nu) if nu.ndim == 0 else None
        self.kappa, self.mu_star = float(kappa), float(mu_star)
        self.x1d, self.w1d = gll(p)
        self.D = diff_matrix(p)
        w = self.w1d
        self.w3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
        self._volume_metric()
        wj = self.w3 * self.detJ
        self.nu_e = np.sum(wj * self.nu_n, axis=(1, 2, 3)) / np.sum(wj, axis=(1, 2, 3))
        if not np.all(self.nu_e > 0):
            raise ValueError('the element averages of nu must be positive')
        self._face_geometry()
        self._penalty()

    # -- Sec. 2.2: Jacobian of the isoparametric map ------------------------
    def _volume_metric(self):
        E, n = self.E, self.n
        Jac = np.empty((E, n, n, n, 3, 3))
        for a in range(3):
            for b in range(3):
                Jac[..., a, b] = d_ref(self.D, self.X[:, a], b)   # dx_a / dxi_b
        self.Jac = Jac
        self.detJ = np.linalg.det(Jac)
        if np.any(self.detJ <= 0):
            raise ValueError("map is not orientation preserving")
        self.dxi = np.linalg.inv(Jac)        # [.., b, a] = dxi_b / dx_a
        self.vol = np.einsum('kji,ekji->e', self.w3, self.detJ)

    def _face_geometry(self):
        """omega*s*n_out at each face node from tangential derivatives only."""
        w = self.w1d
        omega = w[:, None] * w[None, :]
        self.face_Nw, self.face_ws, self.face_n = [], [], []
        self.area = np.zeros((self.E, 6))
        for phi in range(6):
            Xf = face_view(self.X, phi)                  # (E, 3, n, n)
            t1, t2 = _tangential(self.D, Xf, phi)
            N = np.cross(t1, t2, axis=1)                 # = J grad(xi_normal), points to +xi
            sign = 1.0 if phi % 2 == 1 else -1.0
            Nw = sign * omega[None, None] * N
            ws = np.sqrt(np.sum(Nw ** 2, axis=1))
            self.face_Nw.append(Nw)
            self.face_ws.append(ws)
            self.face_n.append(Nw / ws[:, None])
            self.area[:, phi] = ws.sum(axis=(1, 2))
        self.hperp = self.vol[:, None] / self.area

    def _penalty(self):
        """mu on every element face: eq. helmholtz:dgm, mu = mu_star * avg(p(p+1)/(2 h_perp))."""
        p = self.p
        own = p * (p + 1) / (2.0 * self.hperp)
        mu = np.empty((self.E, 6))
        for phi in range(6):
            nb = self.nbr[:, phi]
            interior = nb >= 0
            mu[:, phi] = self.mu_star * own[:, phi]
            nbv = own[nb[interior], self.nbr_face[interior, phi]]
            mu[interior, phi] = self.mu_star * 0.5 * (own[interior, phi] + nbv)
        self.mu = mu

    def neighbour_face(self, V, phi, sel):
        """The neighbours' face layers of V[E, ..., k, j, i] across face phi of the elements
        `sel` (a boolean mask of interior faces), each in the own face's node order."""
        idx = np.nonzero(sel)[0]
        en = self.nbr[idx, phi]
        if not self.oriented:
            return face_view(V[en], OPPOSITE[phi])
        code = self.nbr_face[idx, phi] * 8 + self.nbr_orient[idx, phi]
        out = np.empty((len(idx),) + V.shape[1:-3] + (self.n, self.n))
        for c in np.unique(code):
            hit = code == c
            ap, bp = orient_index(self.n, int(c) % 8)
            out[hit] = face_view(V[en[hit]], int(c) // 8)[..., ap, bp]
        return out

    # -- helpers --------------------------------------------------------------
    def grad(self, u):
        """Physical gradient at every node: sum_c grad(xi_c) d u/d xi_c -> (E, 3, n, n, n)."""
        du = [d_ref(self.D, u, c) for c in range(3)]
        return np.stack([sum(self.dxi[..., c, a] * du[c] for c in range(3)) for a in range(3)], axis=1)

    def n_dof(self):
        return self.E * self.n ** 3
