"""Local h-refinement: the multilevel mesh with twig, leaf and frozen elements and the FAS
V-cycle on it (oracle; test infrastructure only).

Sec. 3.1 builds level l+1 from level l by regular refinement of the marked active elements
(their eight children are active) and irregular refinement of the marked elements'
neighbours (their children are frozen, with values interpolated from the parent).  Active
elements are twigs (refined regularly) or leaves.  Sec. 3.2 restricts residuals and projects
solutions from active children to twig parents; Sec. 3.3 (eq. helmholtz:fas) couples a
level to its frozen elements through the DG operator, gives twigs the FAS right-hand side
and leaves the original one; Alg. 2 adds the frozen update I^{f,l} after the coarse solve.

Readings:
* The base level is a box mesh of nx x ny x nz elements (numbered e = ex + nx (ey + ny ez)),
  all of one degree p, every element active.  Optionally the global p-levels of Sec. 3.1
  (p -> max(1, p / 2) down to 1, every element a twig) lie below it; the root is then p = 1.
* An active element of level k may be refined only if every neighbour of its 3 x 3 x 3 block
  inside the domain exists on level k and is active.  Then the children of a refined
  element find all their in-domain neighbours on level k+1 (active or frozen), and every
  frozen element has a leaf parent, as eq. helmholtz:fas:frozen requires.  The neighbours
  taken for irregular refinement are the 26 of the block ("a layer of frozen elements that
  encloses the active children").
* The children of an element are numbered c = bx + 2 by + 4 bz (b = 0 the lower half of the
  parent's reference interval along that axis); level k+1 lists, for every parent in order
  of its id, the eight children of a refined or irregularly refined parent.  A child's
  geometry is the parent's isoparametric map evaluated at the child's nodes (so the spaces
  nest).
* A face of a level element without a neighbour on that level is a domain boundary face,
  with the parent's boundary code, or a face of a frozen element toward the unrefined region,
  which is given the Neumann code: frozen rows are never used, and the code only keeps the
  level a valid mesh.
* Smoothing acts on active elements: the operator's frozen rows are dropped (r^f = 0, Alg. 5)
  and the Schwarz subdomains are those of the active elements.  A side toward a frozen
  neighbour has no overlap (its interior face terms stay in the 1D surrogate), frozen edge and
  vertex neighbours are filled with zeros (Sec. 4.3.1 item 5), frozen nodes receive no
  correction, and the combined correction is normalised by the weight sum C at every active
  node (C = 1 wherever the quintic weights already form a partition of unity).
* Convergence is measured on the composite problem, eq. helmholtz:fas:converged:leaves: the
  2-norm of f^l - A u over the leaf rows of every level, relative to its value for the initial
  state.
* FMG start-up (Alg. 4): stage l runs a V-cycle on levels 1..l in which level l is the top, so
  its twigs act as leaves with that level's own discrete right-hand side on all its active
  elements; then u_{l+1} = I u_l, i.e. the active children take the interpolation of their twig
  parents and the frozen children that of their leaf parents.  Levels below the base are global
  p-levels and take their own discrete right-hand side as well.
"""
import numpy as np

from .gll import gll
from .hmg import child_matrices, _t3
from .mesh import Mesh
from .mixed import variant_1d_sides
from .schwarz import FACE_OF, surrogate_coefficients
from . import operator as op
from . import solvers as sv
from . import transfer as tr

TWIG, LEAF, FROZEN = 0, 1, 2


def _walk(mesh, e, delta):
    cur = e
    for d in range(3):
        if delta[d]:
            cur = mesh.nbr[cur, FACE_OF[(d, delta[d])]]
            if cur < 0:
                return -1
    return cur


class LocalSchwarz:
    """Weighted Schwarz over the active elements of a level (frozen elements are data)."""

    def __init__(self, mesh, active, m, weighting='quintic'):
        self.mesh, self.active, self.m = mesh, np.asarray(active, dtype=bool), m
        g = surrogate_coefficients(mesh)
        n, p = mesh.n, mesh.p
        self.sub = []
        for e in np.nonzero(self.active)[0]:
            vs = []
            for d in range(3):
                sides, ms = [], []
                for s in (0, 1):
                    phi = 2 * d + s
                    en = mesh.nbr[e, phi]
                    if en >= 0:
                        sides.append('i')
                        ms.append(m if self.active[en] else 0)
                    else:
                        sides.append('d' if mesh.bc[e, phi] == 1 else 'n')
                        ms.append(0)
                v = variant_1d_sides(p, ms[0], ms[1], sides[0], sides[1], mesh.mu_star)
                if weighting == 'plain':
                    v = dict(v, W=np.ones_like(v['W']))
                vs.append(v)
            shape = tuple(len(vs[d]['nodes']) for d in (2, 1, 0))
            idx = np.full(shape, -1, dtype=np.int64)
            for s3, (d3, l3) in enumerate(vs[2]['nodes']):
                for s2, (d2, l2) in enumerate(vs[1]['nodes']):
                    for s1, (d1, l1) in enumerate(vs[0]['nodes']):
                        nb = _walk(mesh, e, (d1, d2, d3))
                        if nb >= 0 and self.active[nb]:
                            idx[s3, s2, s1] = nb * n ** 3 + (l3 * n + l2) * n + l1
            W = vs[2]['W'][:, None, None] * vs[1]['W'][None, :, None] * vs[0]['W'][None, None, :]
            self.sub.append(dict(idx=idx, v=vs, g=g[e], W=W))
        C = np.zeros(mesh.n_dof())
        for sd in self.sub:
            ok = sd['idx'] >= 0
            np.add.at(C, sd['idx'][ok], sd['W'][ok])
        self.C = C

    def apply(self, r):
        from .mixed import MixedSchwarz
        r = np.asarray(r, dtype=np.float64).ravel()
        z = np.zeros_like(r)
        for sd in self.sub:
            idx = sd['idx']
            ok = idx >= 0
            rs = np.where(ok, r[np.where(ok, idx, 0)], 0.0)
            du = MixedSchwarz.local_solve(sd, rs)
            np.add.at(z, idx[ok], (sd['W'] * du)[ok])
        covered = self.C > 0
        z[covered] /= self.C[covered]
        return z.reshape(self.mesh.E, self.mesh.n, self.mesh.n, self.mesh.n)


class LocalLevel:
    """One level: the mesh of all its elements, their classes and the smoother's data."""

    def __init__(self, mesh, cls, m=1, weighting='quintic'):
        self.mesh, self.p = mesh, mesh.p
        self.cls = np.asarray(cls, dtype=np.int64)
        self.active = self.cls != FROZEN
        self._mask = self.active[:, None, None, None].astype(np.float64)
        self.schwarz = LocalSchwarz(mesh, self.active, m, weighting)
        self.down = None          # transfer to the next coarser level (LocalH) or None (p)

    def A(self, u):
        """Rows of the active elements of A u (frozen rows dropped: r^f = 0, Alg. 5)."""
        return op.apply(self.mesh, u) * self._mask

    def B(self, r):
        return self.schwarz.apply(r)


class LocalH:
    """Transfers between a level and its parent level (Sec. 3.2): kind[E_parent] is TWIG for a
    regularly refined parent (active children), FROZEN for an irregularly refined one (frozen
    children) and -1 otherwise; children[E_parent] holds the eight child ids."""

    def __init__(self, p, kind, children):
        self.p = p
        self.kind, self.children = np.asarray(kind), np.asarray(children)
        self.I, self.P = child_matrices(p)

    def _bits(self, c):
        return c & 1, (c >> 1) & 1, c >> 2

    def project(self, uf, n_parent):
        """u^t = P^{t,a} u^a: the children's solution at the parent's nodes, averaged where
        shared; zero on parents that are not twigs."""
        n = self.p + 1
        uf = np.asarray(uf).reshape((-1, n, n, n))
        out = np.zeros((n_parent, n, n, n))
        tw = np.nonzero(self.kind == TWIG)[0]
        for c in range(8):
            bx, by, bz = self._bits(c)
            out[tw] += _t3(self.P[bz], self.P[by], self.P[bx], uf[self.children[tw, c]])
        return out

    def restrict(self, rf, n_parent):
        """r^t = R^{t,a} r^a with R = I^T over the active children."""
        n = self.p + 1
        rf = np.asarray(rf).reshape((-1, n, n, n))
        out = np.zeros((n_parent, n, n, n))
        tw = np.nonzero(self.kind == TWIG)[0]
        for c in range(8):
            bx, by, bz = self._bits(c)
            out[tw] += _t3(self.I[bz].T, self.I[by].T, self.I[bx].T, rf[self.children[tw, c]])
        return out

    def prolong(self, uc, uf, kind):
        """uf at the children of the parents of `kind` set to I uc (returns a new array)."""
        n = self.p + 1
        uc = np.asarray(uc).reshape((-1, n, n, n))
        out = np.array(uf, dtype=np.float64).reshape((-1, n, n, n))
        sel = np.nonzero(self.kind == kind)[0]
        for c in range(8):
            bx, by, bz = self._bits(c)
            out[self.children[sel, c]] = _t3(self.I[bz], self.I[by], self.I[bx], uc[sel])
        return out


def _cells_of_box(nx, ny, nz):
    e = np.arange(nx * ny * nz)
    return np.stack([e % nx, (e // nx) % ny, e // (nx * ny)], axis=1)


def _block_neighbours(cells, index, res):
    """For every cell, its in-domain 3x3x3 block neighbours: (ids or -1 where absent, in-domain mask)."""
    offs = np.array([(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1) if (a, b, c) != (0, 0, 0)])
    ids = -np.ones((len(cells), len(offs)), dtype=np.int64)
    inside = np.zeros((len(cells), len(offs)), dtype=bool)
    for q, o in enumerate(offs):
        nb = cells + o
        ok = np.all((nb >= 0) & (nb < np.asarray(res)), axis=1)
        inside[:, q] = ok
        for i in np.nonzero(ok)[0]:
            ids[i, q] = index.get(tuple(nb[i]), -1)
    return ids, inside


def build_local_mesh(p, box, X, nbr, bc, marks):
    """Level data (base first) of the locally refined multilevel mesh.

    marks: one callable per h-step, mark(centres) -> bool per element of that level, with
    centres the means of the elements' nodal coordinates.  Returns a list of dicts with X, nbr,
    bc, cls and (above the base) the parent transfer data kind/children of the level below."""
    nx, ny, nz = box
    x, _ = gll(p)
    Ich, _ = child_matrices(p)
    cells = _cells_of_box(nx, ny, nz)
    cur = dict(cells=cells, res=(nx, ny, nz), X=np.asarray(X, dtype=np.float64), nbr=np.asarray(nbr),
               bc=np.asarray(bc), cls=np.full(len(cells), LEAF, dtype=np.int64))
    out = [cur]
    for mark in marks:
        E = len(cur['cells'])
        index = {tuple(c): i for i, c in enumerate(cur['cells'])}
        ids, inside = _block_neighbours(cur['cells'], index, cur['res'])
        active = cur['cls'] != FROZEN
        want = np.asarray(mark(cur['X'].mean(axis=(2, 3, 4))), dtype=bool) & active
        # nesting: every in-domain block neighbour exists and is active
        ok = np.all(~inside | ((ids >= 0) & active[np.maximum(ids, 0)]), axis=1)
        refine = want & ok
        irregular = np.zeros(E, dtype=bool)
        for e in np.nonzero(refine)[0]:
            nb = ids[e][ids[e] >= 0]
            irregular[nb] = True
        irregular &= ~refine
        assert np.all(cur['cls'][irregular] != FROZEN)
        cur['cls'] = np.where(refine, TWIG, cur['cls'])
        kind = np.where(refine, TWIG, np.where(irregular, FROZEN, -1))
        parents = np.nonzero(kind >= 0)[0]
        res = tuple(2 * r for r in cur['res'])
        n_f = 8 * len(parents)
        children = -np.ones((E, 8), dtype=np.int64)
        fcells = np.empty((n_f, 3), dtype=np.int64)
        fX = np.empty((n_f, 3, p + 1, p + 1, p + 1))
        fcls = np.empty(n_f, dtype=np.int64)
        parent_of = np.empty(n_f, dtype=np.int64)
        for q, e in enumerate(parents):
            for c in range(8):
                b = np.array([c & 1, (c >> 1) & 1, c >> 2])
                f = 8 * q + c
                children[e, c] = f
                fcells[f] = 2 * cur['cells'][e] + b
                fX[f] = np.stack([_t3(Ich[b[2]], Ich[b[1]], Ich[b[0]], cur['X'][e, a]) for a in range(3)])
                fcls[f] = LEAF if kind[e] == TWIG else FROZEN
                parent_of[f] = e
        findex = {tuple(c): i for i, c in enumerate(fcells)}
        fnbr = -np.ones((n_f, 6), dtype=np.int64)
        fbc = np.zeros((n_f, 6), dtype=np.int64)
        for f in range(n_f):
            for phi in range(6):
                ax, s = phi >> 1, phi & 1
                c = fcells[f].copy()
                c[ax] += 1 if s else -1
                if 0 <= c[ax] < res[ax]:
                    fnbr[f, phi] = findex.get(tuple(c), -1)
                    if fnbr[f, phi] < 0:
                        fbc[f, phi] = 2            # toward the unrefined region (frozen only)
                else:
                    fbc[f, phi] = cur['bc'][parent_of[f], phi]
        nxt = dict(cells=fcells, res=res, X=fX, nbr=fnbr, bc=fbc, cls=fcls, kind=kind, children=children)
        out.append(nxt)
        cur = nxt
    return out


def build_local_levels(p, box, X, nbr, bc, marks, m=1, nu=1.0, kappa=0.0, mu_star=2.0, p_coarsen=False,
                       weighting='quintic'):
    """LocalLevel list, root first: the optional global p-levels below the base, the base box
    mesh and one level per entry of `marks`."""
    data = build_local_mesh(p, box, X, nbr, bc, marks)
    levels = []
    if p_coarsen and p > 1:
        for lv in sv.build_levels(p, data[0]['X'], data[0]['nbr'], data[0]['bc'], m=m, nu=nu, kappa=kappa,
                                  mu_star=mu_star, weighting=weighting)[:-1]:
            ll = LocalLevel(lv.mesh, np.full(lv.mesh.E, TWIG), m, weighting)
            levels.append(ll)
    for k, d in enumerate(data):
        mesh = Mesh(p, d['X'], d['nbr'], d['bc'], nu=nu, kappa=kappa, mu_star=mu_star)
        ll = LocalLevel(mesh, d['cls'], m, weighting)
        if k > 0:
            ll.down = LocalH(p, d['kind'], d['children'])
        levels.append(ll)
    return levels


# ----------------------------------------------------------------------------- the cycle
def _project(lc, lv, u):
    if lv.down is not None:
        return lv.down.project(u, lc.mesh.E)
    return tr.project(lc.p, lv.p, u)


def _restrict(lc, lv, r):
    if lv.down is not None:
        return lv.down.restrict(r, lc.mesh.E)
    return tr.restrict(lc.p, lv.p, r)


def _prolong_active(lc, lv, dc, uf):
    """uf + I^{a,t} dc: the coarse twigs' correction added at their active children."""
    if lv.down is not None:
        return uf + lv.down.prolong(dc, np.zeros_like(uf), TWIG)
    return uf + tr.prolong(lc.p, lv.p, dc)


def _frozen_update(lc, lv, uc, uf):
    """u^f = I^{f,l} u^l_{l-1} (eq. helmholtz:fas:frozen)."""
    if lv.down is None:
        return uf
    return lv.down.prolong(uc, uf, FROZEN)


def level_rhs(levels, b):
    """Per level: b_l on the leaves (b given per level, root first), zero elsewhere."""
    return [np.where((lv.cls == LEAF)[:, None, None, None], np.asarray(bl).reshape(lv.mesh.E, lv.mesh.n, lv.mesh.n,
                                                                                      lv.mesh.n), 0.0)
            for lv, bl in zip(levels, b)]


def fas_vcycle(levels, us, gs, opts):
    """Alg. 2 on the locally refined levels; us, gs per level (root first), updated in place."""
    L = len(levels)
    ubar = [None] * L
    for l in range(L - 1, 0, -1):
        lv, lc = levels[l], levels[l - 1]
        us[l] = sv.smooth(lv, us[l], gs[l], opts.ns1, opts)
        r = gs[l] - lv.A(us[l])
        tw = (lc.cls == TWIG)[:, None, None, None]
        us[l - 1] = np.where(tw, _project(lc, lv, us[l]), us[l - 1])
        ubar[l - 1] = us[l - 1].copy()
        gs[l - 1] = np.where(tw, lc.A(us[l - 1]) + _restrict(lc, lv, r), gs[l - 1])
    us[0] = sv.root_solve(levels[0], us[0], gs[0], opts)
    for l in range(1, L):
        lv, lc = levels[l], levels[l - 1]
        us[l] = _frozen_update(lc, lv, us[l - 1], us[l])
        us[l] = _prolong_active(lc, lv, us[l - 1] - ubar[l - 1], us[l])
        us[l] = sv.smooth(lv, us[l], gs[l], opts.ns2, opts)
    return us


def _interpolate_up(lc, lv, uc, uf):
    """u_l = I u_{l-1} (Alg. 4): active children of twigs and frozen children of leaves."""
    if lv.down is None:
        return tr.prolong(lc.p, lv.p, uc)
    out = lv.down.prolong(uc, uf, TWIG)
    return lv.down.prolong(uc, out, FROZEN)


def fmg_start(levels, b_full, opts):
    """Alg. 4 on the locally refined levels; b_full: every level's discrete right-hand side on
    all its elements (root first).  Returns the start values of every level."""
    L = len(levels)
    us = [np.zeros((lv.mesh.E, lv.mesh.n, lv.mesh.n, lv.mesh.n)) for lv in levels]
    gs = level_rhs(levels, b_full)
    for top in range(L - 1):
        act = levels[top].active[:, None, None, None]
        sub_g = gs[:top] + [np.where(act, np.asarray(b_full[top]).reshape(us[top].shape), 0.0)]
        us[:top + 1] = fas_vcycle(levels[:top + 1], us[:top + 1], sub_g, opts)
        us[top + 1] = _interpolate_up(levels[top], levels[top + 1], us[top], us[top + 1])
    return us


def composite_residual(levels, us, gs):
    """2-norm of the leaf rows of g_l - A u_l over all levels (g_l = b_l on leaves)."""
    s = 0.0
    for lv, u, g in zip(levels, us, gs):
        r = (g - lv.A(u))[lv.cls == LEAF]
        s += float(np.sum(r * r))
    return np.sqrt(s)


def solve(levels, b, opts, max_cycles=30, rtol=1e-10):
    """V-cycles from u = 0 (after the FMG start-up when opts.start == 'fmg') until the composite
    residual falls by rtol relative to that of u = 0; returns (us, history).  b: every level's
    discrete right-hand side (the leaf rows enter the cycle, the FMG start-up takes all active
    rows)."""
    us = [np.zeros((lv.mesh.E, lv.mesh.n, lv.mesh.n, lv.mesh.n)) for lv in levels]
    gs = level_rhs(levels, b)
    r0 = composite_residual(levels, us, gs)
    if opts.start == 'fmg':
        us = fmg_start(levels, b, opts)
    hist = [1.0]
    for _ in range(max_cycles):
        us = fas_vcycle(levels, us, gs, opts)
        hist.append(composite_residual(levels, us, gs) / r0)
        if hist[-1] <= rtol:
            break
    return us, hist


def composite_state(levels, z):
    """Every level's vector from the leaf values z (concatenated over levels, root first):
    twigs are the projections of their active children (top down, eq.
    helmholtz:fas:converged:twigs), frozen values the interpolation of their leaf parents
    (eq. helmholtz:fas:converged:frozen)."""
    L = len(levels)
    us, o = [], 0
    for lv in levels:
        n3 = lv.mesh.n ** 3
        u = np.zeros((lv.mesh.E, lv.mesh.n, lv.mesh.n, lv.mesh.n))
        leaf = lv.cls == LEAF
        k = int(leaf.sum()) * n3
        u[leaf] = z[o:o + k].reshape(-1, lv.mesh.n, lv.mesh.n, lv.mesh.n)
        o += k
        us.append(u)
    for l in range(L - 2, -1, -1):
        lv, lc = levels[l + 1], levels[l]
        tw = (lc.cls == TWIG)[:, None, None, None]
        us[l] = np.where(tw, _project(lc, lv, us[l + 1]), us[l])
    for l in range(1, L):
        us[l] = _frozen_update(levels[l - 1], levels[l], us[l - 1], us[l])
    return us


def composite_dense(levels, b):
    """Dense solve of eq. helmholtz:fas:converged for the leaf values (tiny meshes only): the
    leaf rows of A_l u_l = b_l with u_l from composite_state.  Returns every level's vector."""
    nz = sum(int((lv.cls == LEAF).sum()) * lv.mesh.n ** 3 for lv in levels)

    def leaf_rows(us):
        return np.concatenate([lv.A(u)[lv.cls == LEAF].ravel() for lv, u in zip(levels, us)])

    K = np.empty((nz, nz))
    e = np.zeros(nz)
    for j in range(nz):
        e[j] = 1.0
        K[:, j] = leaf_rows(composite_state(levels, e))
        e[j] = 0.0
    rhs = np.concatenate([np.asarray(bl).reshape(lv.mesh.E, -1)[lv.cls == LEAF].ravel()
                          for lv, bl in zip(levels, b)])
    z = np.linalg.solve(K, rhs)
    return composite_state(levels, z)
