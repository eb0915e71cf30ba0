"""SIPG operator, Schwarz smoother and V-cycle on meshes with a degree per element
(oracle; test infrastructure only).

The paper keeps one degree per level (Sec. 3.1); mixed degrees are an addition, so every
step here is a reading, stated where it is used:

* A face between elements of degrees p and p' is integrated with the GLL rule of the finer
  side, whose omega*s are the face weights.  Each side's trace and normal flux
  nu n.grad u are interpolated from its own face nodes to that grid; the penalty uses both
  degrees, mu = mu_star (p(p+1)/(2h) + p'(p'+1)/(2h'))/2 (eq. helmholtz:dgm).  Test functions
  are the element's own basis evaluated on the finer grid, so row terms are restricted back
  with the transposed interpolation, and the lifting term -{nu grad v}.[u] uses the restricted
  jump times the element's own nu n.grad xi at its face nodes.  The form stays symmetric.
  With equal degrees it is the conforming form (pinned).
* Schwarz: a side toward a neighbour of another degree has no overlap ("i0": the 1D matrix
  keeps the interior face terms of the own element only); edge and vertex neighbours of
  another degree are zero-filled and receive nothing (Sec. 4.3.1 item 5 fills neighbours
  without a counterpart with zeros).  Near a degree jump the tensor-product weights of the
  subdomains that reach a node then no longer add up to one (two subdomains can disagree
  about who covers a shared node), so the combined correction is normalised:
  z = C^-1 sum_s R_s^T W_s A~_s^-1 R_s r with the diagonal C = sum_s R_s^T W_s R_s 1.
  Every node is covered by its own element's subdomain with a positive weight, so C > 0;
  where the tensor weights already add up to one (all of a uniform mesh) C = 1.
* Levels: p_{l-1} = max(1, floor(p_l / 2)) per element; elements at degree 1 stay there.

Elements are stored element-major with offsets; inside an element the layout is that of
`mesh.Mesh` ([k, j, i], i fastest).
"""
import numpy as np
import scipy.linalg

from .gll import gll, lagrange_eval
from .mesh import Mesh, d_ref, dT_ref, face_view, OPPOSITE
from .schwarz import quintic, FACE_OF
from .sipg1d import sipg_1d
from . import transfer as tr


class MixedMesh:
    def __init__(self, degrees, coords, nbr, bc, nu=1.0, kappa=0.0, mu_star=2.0):
        self.p = np.asarray(degrees, dtype=np.int64)
        self.E = len(self.p)
        self.nbr = np.asarray(nbr, dtype=np.int64)
        self.bc = np.asarray(bc, dtype=np.int64)
        self.nu, self.kappa, self.mu_star = float(nu), float(kappa), float(mu_star)
        self.n = self.p + 1
        self.off = np.concatenate(([0], np.cumsum(self.n ** 3)))
        # per-element geometry from single-element meshes (no neighbour data needed)
        self.el = []
        dummy_nbr = -np.ones((1, 6), dtype=np.int64)
        dummy_bc = np.ones((1, 6), dtype=np.int64)
        for e in range(self.E):
            self.el.append(Mesh(int(self.p[e]), np.asarray(coords[e])[None], dummy_nbr, dummy_bc,
                                nu=nu, kappa=kappa, mu_star=mu_star))
        self.hperp = np.array([m.hperp[0] for m in self.el])

    def n_dof(self):
        return int(self.off[-1])

    def block(self, v, e):
        n = int(self.n[e])
        return np.asarray(v)[self.off[e]:self.off[e + 1]].reshape(n, n, n)

    def mu_face(self, e, phi):
        en = self.nbr[e, phi]
        pe = self.p[e]
        own = pe * (pe + 1) / (2.0 * self.hperp[e, phi])
        if en < 0:
            return self.mu_star * own
        pn = self.p[en]
        oth = pn * (pn + 1) / (2.0 * self.hperp[en, OPPOSITE[phi]])
        return self.mu_star * 0.5 * (own + oth)

    def _face_data(self, e, u_e, phi):
        """(trace, nu n_out.grad u, nu n_out.grad xi_c for c = 0..2) at the face nodes of e."""
        m = self.el[e]
        grad = m.grad(u_e[None])[0]                          # (3, n, n, n)
        nvec = m.face_n[phi][0]                              # (3, n, n)
        tr_ = face_view(u_e, phi)
        q = self.nu * np.einsum('axy,axy->xy', nvec, face_view(grad, phi))
        ng = []
        for c in range(3):
            dxi_c = face_view(np.moveaxis(m.dxi[0][..., c, :], -1, 0), phi)   # (3, n, n)
            ng.append(self.nu * np.einsum('axy,axy->xy', nvec, dxi_c))
        return tr_, q, ng

    def apply(self, u):
        u = np.asarray(u, dtype=np.float64).ravel()
        out = np.zeros_like(u)
        for e in range(self.E):
            m = self.el[e]
            ue = self.block(u, e)
            n = int(self.n[e])
            grad = m.grad(ue[None])[0]
            res = self.kappa * m.w3 * m.detJ[0] * ue
            for b in range(3):
                flux = self.nu * m.w3 * m.detJ[0] * np.einsum('kjia,akji->kji', m.dxi[0][..., b, :], grad)
                res = res + dT_ref(m.D, flux, b)
            lift = [np.zeros((n, n, n)) for _ in range(3)]
            for phi in range(6):
                t_o, q_o, ng_o = self._face_data(e, ue, phi)
                ws_o = m.face_ws[phi][0]
                en = self.nbr[e, phi]
                row = np.zeros((n, n))
                S = np.zeros((n, n))        # restricted lifting weight at own face nodes (includes omega s)
                if en >= 0:
                    un = self.block(u, en)
                    t_n, q_n, _ = self._face_data(en, un, OPPOSITE[phi])
                    mu = self.mu_face(e, phi)
                    pF = max(self.p[e], self.p[en])
                    xF, _ = gll(int(pF))
                    Io = lagrange_eval(gll(int(self.p[e]))[0], xF)
                    In = lagrange_eval(gll(int(self.p[en]))[0], xF)
                    wF = ws_o if self.p[e] >= self.p[en] else self.el[en].face_ws[OPPOSITE[phi]][0]
                    tF = Io @ t_o @ Io.T - In @ t_n @ In.T
                    qF = Io @ q_o @ Io.T - In @ q_n @ In.T
                    rowF = wF * (mu * self.nu * tF - 0.5 * qF)
                    row = Io.T @ rowF @ Io
                    S = Io.T @ (-0.5 * wF * tF) @ Io
                elif self.bc[e, phi] == 1:
                    mu = self.mu_face(e, phi)
                    row = ws_o * (2.0 * mu * self.nu * t_o - q_o)
                    S = -ws_o * t_o
                fv = face_view(res, phi)
                fv += row
                for c in range(3):
                    lv = face_view(lift[c], phi)
                    lv += S * ng_o[c]
            for c in range(3):
                res = res + dT_ref(m.D, lift[c], c)
            out[self.off[e]:self.off[e + 1]] = res.ravel()
        return out

    def rhs(self, f, uD=None):
        """b = w J f + Dirichlet terms (2 mu nu omega s u_D, lifting -nu omega s u_D n.grad phi)."""
        f = np.asarray(f, dtype=np.float64).ravel()
        out = np.zeros_like(f)
        for e in range(self.E):
            m = self.el[e]
            n = int(self.n[e])
            be = m.w3 * m.detJ[0] * self.block(f, e)
            lift = [np.zeros((n, n, n)) for _ in range(3)]
            if uD is not None:
                ude = self.block(uD, e)
                for phi in range(6):
                    if self.nbr[e, phi] >= 0 or self.bc[e, phi] != 1:
                        continue
                    _, _, ng = self._face_data(e, ude, phi)
                    ws = m.face_ws[phi][0]
                    tD = face_view(ude, phi)
                    fv = face_view(be, phi)
                    fv += 2.0 * self.mu_face(e, phi) * self.nu * ws * tD
                    for c in range(3):
                        lv = face_view(lift[c], phi)
                        lv += -ws * tD * ng[c]
            for c in range(3):
                be = be + dT_ref(m.D, lift[c], c)
            out[self.off[e]:self.off[e + 1]] = be.ravel()
        return out

    def assemble(self):
        N = self.n_dof()
        A = np.empty((N, N))
        v = np.zeros(N)
        for j in range(N):
            v[j] = 1.0
            A[:, j] = self.apply(v)
            v[j] = 0.0
        return A


# ---------------------------------------------------------------------------- Schwarz
def variant_1d_sides(p, m_left, m_right, left, right, mu_star):
    """1D subdomain matrices with a separate overlap per side (0 gives the 'i0' variant)."""
    n = p + 1
    elems = ([-1] if left == 'i' else []) + [0] + ([1] if right == 'i' else [])
    K = len(elems)
    Mg, Lg = sipg_1d(p, K, 2.0, mu_star, 'd' if left == 'd' else 'n', 'd' if right == 'd' else 'n')
    nodes, sel = [], []
    for pos, dlt in enumerate(elems):
        locs = range(n - m_left, n) if dlt == -1 else (range(0, m_right) if dlt == 1 else range(n))
        for l in locs:
            nodes.append((dlt, l))
            sel.append(pos * n + l)
    sel = np.array(sel, dtype=int)
    L = Lg[np.ix_(sel, sel)]
    M = np.diag(Mg)[sel]
    lam, S = scipy.linalg.eigh(L, np.diag(M))
    x, _ = gll(p)
    W = np.ones(len(nodes))
    for s, (dlt, l) in enumerate(nodes):
        w = 1.0
        if left == 'i' and m_left > 0:
            a = 0.5 * (1.0 + x[m_left])
            d = 0.5 * (1.0 + x[l]) if dlt == 0 else (-0.5 * (1.0 - x[l]) if dlt == -1 else None)
            if d is not None:
                w *= quintic((d + a) / (2 * a))
        if right == 'i' and m_right > 0:
            a = 0.5 * (1.0 + x[m_right])
            d = 0.5 * (1.0 - x[l]) if dlt == 0 else (-0.5 * (1.0 + x[l]) if dlt == 1 else None)
            if d is not None:
                w *= quintic((d + a) / (2 * a))
        W[s] = w
    return dict(nodes=nodes, M=M, L=L, S=S, lam=lam, W=W)


def _walk(mesh, e, delta):
    cur = e
    for d in range(3):
        if delta[d]:
            cur = mesh.nbr[cur, FACE_OF[(d, delta[d])]]
            if cur < 0:
                return -1
    return cur


class MixedSchwarz:
    def __init__(self, mesh, m):
        from .schwarz import surrogate_coefficients
        self.mesh, self.m = mesh, m
        self.sub = []
        for e in range(mesh.E):
            el = mesh.el[e]
            g = surrogate_coefficients(el)[0]
            p = int(mesh.p[e])
            vs = []
            for d in range(3):
                sides, ms = [], []
                for s in (0, 1):
                    phi = 2 * d + s
                    en = mesh.nbr[e, phi]
                    if en >= 0:
                        sides.append('i')
                        ms.append(m if mesh.p[en] == p else 0)
                    else:
                        sides.append('d' if mesh.bc[e, phi] == 1 else 'n')
                        ms.append(0)
                vs.append(variant_1d_sides(p, ms[0], ms[1], sides[0], sides[1], mesh.mu_star))
            n = p + 1
            shape = tuple(len(vs[d]['nodes']) for d in (2, 1, 0))
            idx = np.full(shape, -1, dtype=np.int64)
            for s3, (d3, l3) in enumerate(vs[2]['nodes']):
                for s2, (d2, l2) in enumerate(vs[1]['nodes']):
                    for s1, (d1, l1) in enumerate(vs[0]['nodes']):
                        nb = _walk(mesh, e, (d1, d2, d3))
                        if nb >= 0 and mesh.p[nb] == p:      # other-degree edge/vertex neighbours: zero fill
                            idx[s3, s2, s1] = mesh.off[nb] + (l3 * n + l2) * n + l1
            W = vs[2]['W'][:, None, None] * vs[1]['W'][None, :, None] * vs[0]['W'][None, None, :]
            self.sub.append(dict(idx=idx, v=vs, g=g, W=W))
        # C = sum_s R_s^T W_s R_s 1, the weight sum at every node
        C = np.zeros(mesh.n_dof())
        for sd in self.sub:
            valid = sd['idx'] >= 0
            np.add.at(C, sd['idx'][valid], sd['W'][valid])
        self.C = C

    @staticmethod
    def local_solve(sd, rs):
        """Fast diagonalisation (S3 x S2 x S1) D^-1 (S3^T x S2^T x S1^T) rs of one subdomain."""
        v, g = sd['v'], sd['g']
        S1, S2, S3 = v[0]['S'], v[1]['S'], v[2]['S']
        t = np.einsum('kc,jb,ia,kji->cba', S3, S2, S1, rs)
        Dg = (g[0] + g[1] * v[0]['lam'][None, None, :] + g[2] * v[1]['lam'][None, :, None]
              + g[3] * v[2]['lam'][:, None, None])
        return np.einsum('kc,jb,ia,cba->kji', S3, S2, S1, t / Dg)

    def apply(self, r):
        """z = C^-1 sum_s R_s^T W_s A~_s^-1 R_s r (eq. schwarz:correction, normalised weights)."""
        r = np.asarray(r, dtype=np.float64).ravel()
        z = np.zeros_like(r)
        for sd in self.sub:
            idx = sd['idx']
            valid = idx >= 0
            rs = np.where(valid, r[np.where(valid, idx, 0)], 0.0)
            du = self.local_solve(sd, rs)
            np.add.at(z, idx[valid], (sd['W'] * du)[valid])
        return z / self.C


# ---------------------------------------------------------------------------- levels / cycle
class MixedLevel:
    def __init__(self, mesh, m):
        self.mesh = mesh
        self.schwarz = MixedSchwarz(mesh, m)

    def A(self, u):
        return self.mesh.apply(u)

    def B(self, r):
        return self.schwarz.apply(r)


def coarse_degrees(p):
    return np.maximum(1, np.asarray(p) // 2)


def build_mixed_levels(degrees, coords, nbr, bc, m=1, nu=1.0, kappa=0.0, mu_star=2.0):
    """Level list (root first); level count from the largest degree's chain."""
    degs = [np.asarray(degrees, dtype=np.int64)]
    while degs[-1].max() > 1:
        degs.append(coarse_degrees(degs[-1]))
    coords_l = [list(coords)]
    for li in range(1, len(degs)):
        prev = coords_l[-1]
        cur = []
        for e in range(len(degrees)):
            pf, pc = int(degs[li - 1][e]), int(degs[li][e])
            cur.append(prev[e] if pf == pc else tr.coarse_coords(pc, pf, np.asarray(prev[e])[None])[0])
        coords_l.append(cur)
    levels = [MixedLevel(MixedMesh(degs[li], coords_l[li], nbr, bc, nu=nu, kappa=kappa, mu_star=mu_star), m)
              for li in range(len(degs))]
    return levels[::-1]


def _per_element(fn, mesh_from, mesh_to, v):
    out = np.zeros(mesh_to.n_dof())
    for e in range(mesh_from.E):
        pf, pt = int(mesh_from.p[e]), int(mesh_to.p[e])
        blk = mesh_from.block(v, e)[None]
        res = blk if pf == pt else fn(blk, pf, pt)
        out[mesh_to.off[e]:mesh_to.off[e + 1]] = res.ravel()
    return out


def project(fine, coarse, u):
    return _per_element(lambda b, pf, pc: tr.project(pc, pf, b), fine, coarse, u)


def restrict(fine, coarse, r):
    return _per_element(lambda b, pf, pc: tr.restrict(pc, pf, b), fine, coarse, r)


def prolong(coarse, fine, u):
    return _per_element(lambda b, pc, pf: tr.prolong(pc, pf, b), coarse, fine, u)


def fas_vcycle(levels, u_top, f_top, opts):
    """Alg. 2 with per-element p-coarsening (transfers element by element)."""
    from . import solvers as sv
    L = len(levels)
    u, g, ubar = [None] * L, [None] * L, [None] * L
    u[L - 1], g[L - 1] = np.asarray(u_top, dtype=np.float64).ravel(), np.asarray(f_top, dtype=np.float64).ravel()
    for l in range(L - 1, 0, -1):
        lv, lc = levels[l], levels[l - 1]
        u[l] = sv.smooth(lv, u[l], g[l], opts.ns1, opts)
        r = g[l] - lv.A(u[l])
        ubar[l - 1] = project(lv.mesh, lc.mesh, u[l])
        u[l - 1] = ubar[l - 1].copy()
        g[l - 1] = lc.A(u[l - 1]) + restrict(lv.mesh, lc.mesh, r)
    r0 = sv.norm(g[0] - levels[0].A(u[0]))
    u[0] = sv.scg(levels[0], u[0], g[0], opts.root_maxit, opts.root_rtol * r0, opts.first_dir)
    for l in range(1, L):
        lv, lc = levels[l], levels[l - 1]
        u[l] = u[l] + prolong(lc.mesh, lv.mesh, u[l - 1] - ubar[l - 1])
        u[l] = sv.smooth(lv, u[l], g[l], opts.ns2, opts)
    return u[L - 1]


def solve(levels, u0, f, opts, max_cycles=30, rtol=1e-10):
    from . import solvers as sv
    top = levels[-1]
    u = np.asarray(u0, dtype=np.float64).ravel().copy()
    r0 = sv.norm(f - top.A(u))
    hist = [1.0]
    for _ in range(max_cycles):
        u = fas_vcycle(levels, u, f, opts)
        hist.append(sv.norm(f - top.A(u)) / r0)
        if hist[-1] <= rtol:
            break
    return u, hist
