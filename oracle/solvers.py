"""Smoothers, Krylov root solver and V-cycles (oracle; test infrastructure only).

* WAS  - Alg. 5: r = f - A u; u = u + sum_e R^T W A~^-1 R r, n_i times.
* SCG  - Alg. 6, the inexact Schwarz-preconditioned CG of Golub and Ye,
         with the flexible beta = z^T (r - r0) / gamma.  Reading: the first
         search direction is p = z (the standard PCG start); the literal
         p = r of the printed algorithm is kept behind `first_dir='r'`.
* FAS  - Alg. 2 with global p-coarsening (every coarse element is a twig, no
         frozen elements): the projected coarse solution u_bar = P u_l is
         stored and reused in the prolongation u_l += I (u_{l-1} - u_bar).
* CS   - Alg. 1, the linear correction scheme, for the FAS == CS check.
* CMG  - Alg. 3, cascadic start-up: root solve, then on every level up to L-1 the
         interpolated coarser solution smoothed with n_s0 steps (Sec. 3.3, FAS-CMG).
* FMG  - Alg. 4, full multigrid start-up: a V-cycle on levels 1..l, then interpolation
         to level l+1, for l = 1..L-1 (Sec. 3.3, FAS-FMG).
* Crossover smoothing (Sec. 6.1 method names): between two consecutive cycles the top
  level gets n_sc smoothing steps in place of the n_s2 post- plus n_s1 pre-smoothing steps.

Readings (the paper leaves these open):
* Level right-hand sides of the start-ups: f_{l-1} = R f_l, the fine load vector tested with
  the coarse basis (Alg. 3 and 4 take f on every level; with global coarsening no coarse
  element is a leaf).
* Start values on coarser levels: the projection P of the next finer level's start value
  (zero when the top level starts from zero).
* Alg. 3 ends its loop at level L-1; the top level then receives u_L = I u_{L-1}, which the
  first V-cycle smooths.
* Crossover: cycle k > 1 begins with n_sc - n_s2 top-level pre-smoothing steps, so the steps
  between the residual checks of two cycles add up to n_sc (the total of the cost model,
  eq. mg-method:cost:total); the coarser levels keep n_s1.
"""
import numpy as np

from . import operator as op
from .mesh import Mesh
from .schwarz import Schwarz
from .unstructured import TopoSchwarz
from . import transfer as tr


class Level:
    """One p-level.  A mesh that carries its neighbours' faces and orientations (an
    unstructured mesh, Sec. 5.1) takes the topology-walking Schwarz method of
    oracle.unstructured; on a regular mesh both give the same subdomains."""

    def __init__(self, mesh, m, weighting='quintic', topology=False):
        self.mesh = mesh
        self.schwarz = TopoSchwarz(mesh, m, weighting) if topology else Schwarz(mesh, m, weighting)
        self.p = mesh.p

    def A(self, u):
        return op.apply(self.mesh, u)

    def B(self, r):
        return self.schwarz.apply(r)


def build_levels(p, X, nbr, bc, m=1, nu=1.0, kappa=0.0, mu_star=2.0, weighting='quintic', delta=None,
                 nbr_face=None, nbr_orient=None):
    """Level list (root first) for global p-coarsening of a uniform-degree mesh.  With `delta`
    the overlap of every level follows from its degree (Sec. 4.3.1 item 3), else it is m.
    A nodal nu (E, n, n, n) at the fine degree is, like the geometry, evaluated at the nodes of
    each coarser level (reading: every level rediscretises the same coefficient field).
    nbr_face / nbr_orient describe an unstructured mesh (every level keeps the topology)."""
    from .schwarz import overlap_layers
    chain = tr.degree_chain(p)
    levels = [None] * len(chain)
    Xl = np.asarray(X, dtype=np.float64)
    nul = np.asarray(nu, dtype=np.float64)
    nodal = nul.ndim == 4
    for li in range(len(chain) - 1, -1, -1):
        pl = chain[li]
        if li < len(chain) - 1:
            Xl = tr.coarse_coords(pl, chain[li + 1], Xl)
            if nodal:
                nul = tr.coarse_coords(pl, chain[li + 1], nul[:, None])[:, 0]
        ml = min(overlap_layers(pl, delta), pl) if delta is not None else m
        mesh = Mesh(pl, Xl, nbr, bc, nu=nul, kappa=kappa, mu_star=mu_star, nbr_face=nbr_face, nbr_orient=nbr_orient)
        levels[li] = Level(mesh, ml, weighting, topology=nbr_face is not None)
    return levels


def norm(v):
    return float(np.sqrt(np.sum(np.asarray(v) ** 2)))


# transfers between level lv and the next coarser level lc: p-coarsening (Sec. 3.2, per element)
# or, when lv carries an h-coarsening in `down` (oracle.hmg), the parent/children transfers
def t_project(lc, lv, u, kind='interp'):
    ht = getattr(lv, 'down', None)
    return ht.project(u) if ht is not None else tr.project(lc.p, lv.p, u, kind)


def t_restrict(lc, lv, r):
    ht = getattr(lv, 'down', None)
    return ht.restrict(r) if ht is not None else tr.restrict(lc.p, lv.p, r)


def t_prolong(lc, lv, uc):
    ht = getattr(lv, 'down', None)
    return ht.prolong(uc) if ht is not None else tr.prolong(lc.p, lv.p, uc)


def was(level, u, f, n_i):
    """Alg. 5 (weighted additive Schwarz)."""
    for _ in range(n_i):
        r = f - level.A(u)
        u = u + level.B(r)
    return u


def project_range(v):
    """v minus its mean: the component orthogonal to the constants, which span the null space
    of A when kappa = 0 and no face is Dirichlet (the range of the symmetric A)."""
    return v - np.mean(v)


def scg(level, u, f, n_i, r_max=0.0, first_dir='z', precond=None, stats=None, project=None):
    """Alg. 6 (Schwarz-preconditioned inexact CG); exits when ||r|| <= r_max, or when p^T A p <= 0
    makes the step length undefined (breakdown), with the last iterate.  With `project` the
    residual and every preconditioned residual are projected (remark on IPCG for semidefinite
    systems, Sec. 4.3.2)."""
    B = level.B if precond is None else precond
    if project is not None:
        B0 = B
        B = lambda v: project(B0(v))
    r = f - level.A(u)
    if project is not None:
        r = project(r)
    p = r.copy() if first_dir == 'r' else None
    gamma = None
    r0 = None
    it = 0
    for i in range(1, n_i + 1):
        z = B(r)
        if i > 1:
            beta = np.sum(z * (r - r0)) / gamma
            p = beta * p + z
        elif first_dir == 'z':
            p = z.copy()
        q = level.A(p)
        gamma = np.sum(z * r)
        pq = np.sum(p * q)
        if not pq > 0:          # alpha = gamma / p^T A p is undefined: stop with the last iterate
            break
        alpha = gamma / pq
        r0 = r
        r = r - alpha * q
        u = u + alpha * p
        it = i
        if norm(r) <= r_max:
            break
    if stats is not None:
        stats['iters'] = it
    return u


class Options:
    """Cycle parameters: smoother 'was'|'scg', ns1, ns2; root 'scg' (to root_rtol) or 'direct';
    start None | 'cmg' | 'fmg' with n_s0 CMG steps per level (default ns1 + ns2); crossover
    steps nsc on the top level between cycles (default ns1 + ns2, i.e. none); null_space: the
    operator is semidefinite (kappa = 0, no Dirichlet face) and the root SCG projects its
    residuals onto the range of A (remark on IPCG, Sec. 4.3.2; the right-hand side must have
    zero mean)."""

    def __init__(self, smoother='was', ns1=2, ns2=2, root_rtol=1e-12, root_maxit=500, first_dir='z',
                 root='scg', start=None, ns0=None, nsc=None, projection='interp', null_space=False):
        self.smoother, self.ns1, self.ns2 = smoother, ns1, ns2
        self.null_space = null_space
        self.projection = projection
        self.root_rtol, self.root_maxit, self.first_dir = root_rtol, root_maxit, first_dir
        self.root = root
        self.start = start
        self.ns0 = ns1 + ns2 if ns0 is None else ns0
        self.nsc = ns1 + ns2 if nsc is None else nsc
        if self.nsc < ns2:
            raise ValueError('crossover needs nsc >= ns2')


def smooth(level, u, g, n, opts):
    if n == 0:
        return u
    if opts.smoother == 'was':
        return was(level, u, g, n)
    return scg(level, u, g, n, 0.0, opts.first_dir)


def root_solve(level, u, g, opts, stats=None):
    if opts.root == 'direct':
        A = op.assemble(level.mesh)
        return np.linalg.solve(A, g.ravel()).reshape(u.shape)
    pr = project_range if opts.null_space else None
    r = g - level.A(u)
    r0 = norm(r if pr is None else pr(r))
    return scg(level, u, g, opts.root_maxit, opts.root_rtol * r0, opts.first_dir, stats=stats, project=pr)


def fas_vcycle(levels, u_top, f_top, opts, ns1_top=None):
    """Alg. 2 with global p-coarsening; returns the new top-level solution.  ns1_top replaces
    ns1 on the top level (crossover smoothing)."""
    L = len(levels)
    u = [None] * L
    g = [None] * L
    ubar = [None] * L
    u[L - 1], g[L - 1] = u_top, f_top
    for l in range(L - 1, 0, -1):
        lv, lc = levels[l], levels[l - 1]
        n1 = ns1_top if (l == L - 1 and ns1_top is not None) else opts.ns1
        u[l] = smooth(lv, u[l], g[l], n1, opts)
        r = g[l] - lv.A(u[l])
        ubar[l - 1] = t_project(lc, lv, u[l], opts.projection)
        u[l - 1] = ubar[l - 1].copy()
        g[l - 1] = lc.A(u[l - 1]) + t_restrict(lc, lv, r)
    u[0] = root_solve(levels[0], u[0], g[0], opts)
    for l in range(1, L):
        lv, lc = levels[l], levels[l - 1]
        u[l] = u[l] + t_prolong(lc, lv, u[l - 1] - ubar[l - 1])
        u[l] = smooth(lv, u[l], g[l], opts.ns2, opts)
    return u[L - 1]


def cs_vcycle(levels, u_top, f_top, opts):
    """Alg. 1 (correction scheme)."""
    L = len(levels)
    u = [None] * L
    f = [None] * L
    u[L - 1], f[L - 1] = u_top, f_top
    for l in range(L - 1, 0, -1):
        lv, lc = levels[l], levels[l - 1]
        u[l] = smooth(lv, u[l], f[l], opts.ns1, opts)
        u[l - 1] = np.zeros((lc.mesh.E, lc.mesh.n, lc.mesh.n, lc.mesh.n))
        f[l - 1] = tr.restrict(lc.p, lv.p, f[l] - lv.A(u[l]))
    u[0] = root_solve(levels[0], u[0], f[0], opts)
    for l in range(1, L):
        lv, lc = levels[l], levels[l - 1]
        u[l] = u[l] + tr.prolong(lc.p, lv.p, u[l - 1])
        u[l] = smooth(lv, u[l], f[l], opts.ns2, opts)
    return u[L - 1]


def level_rhs(levels, f_top):
    """f_l on every level (root first), f_{l-1} = R f_l."""
    fs = [None] * len(levels)
    fs[-1] = f_top
    for l in range(len(levels) - 1, 0, -1):
        fs[l - 1] = t_restrict(levels[l - 1], levels[l], fs[l])
    return fs


def _start_values(levels, u_top):
    us = [None] * len(levels)
    us[-1] = u_top
    for l in range(len(levels) - 1, 0, -1):
        us[l - 1] = t_project(levels[l - 1], levels[l], us[l])
    return us


def cmg_start(levels, u_top, f_top, opts):
    """Alg. 3 (FAS-CMG start-up); returns the top-level start value I u_{L-1}."""
    L = len(levels)
    fs, us = level_rhs(levels, f_top), _start_values(levels, u_top)
    u = root_solve(levels[0], us[0], fs[0], opts)
    for l in range(1, L - 1):
        u = t_prolong(levels[l - 1], levels[l], u)
        u = smooth(levels[l], u, fs[l], opts.ns0, opts)
    return t_prolong(levels[L - 2], levels[L - 1], u) if L > 1 else u


def fmg_start(levels, u_top, f_top, opts):
    """Alg. 4 (FAS-FMG start-up): for l = 1..L-1 a V-cycle on levels 1..l, then u_{l+1} = I u_l."""
    L = len(levels)
    fs, us = level_rhs(levels, f_top), _start_values(levels, u_top)
    u = us[0]
    for l in range(1, L):
        u = fas_vcycle(levels[:l], u, fs[l - 1], opts)
        u = t_prolong(levels[l - 1], levels[l], u)
    return u if L > 1 else fas_vcycle(levels, u, fs[0], opts)


def solve(levels, u0, f, opts, max_cycles=30, rtol=1e-10, cycle=fas_vcycle):
    """Optional start-up (opts.start), then V-cycles until ||r||/||r0|| <= rtol, with
    r0 = f - A u0; returns (u, history of relative residuals after each cycle)."""
    top = levels[-1]
    u = u0.copy()
    r0 = norm(f - top.A(u))
    if opts.start == 'cmg':
        u = cmg_start(levels, u, f, opts)
    elif opts.start == 'fmg':
        u = fmg_start(levels, u, f, opts)
    hist = [1.0]
    for k in range(max_cycles):
        if cycle is fas_vcycle:
            u = cycle(levels, u, f, opts, ns1_top=None if k == 0 else opts.nsc - opts.ns2)
        else:
            u = cycle(levels, u, f, opts)
        hist.append(norm(f - top.A(u)) / r0)
        if hist[-1] <= rtol:
            break
    return u, hist
