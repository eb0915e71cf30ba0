"""O1: the FP64 matrix-free C/OpenMP oracle (oracle/o1.c) behind a small numpy interface
(oracle; test infrastructure only).

The C library runs the same method as the numpy oracle of this package, at full size and on
every host core.  Its small 1D tables come from the numpy oracle (pinned in its own tests):
GLL nodes and weights, the differentiation matrix, rows 0 and 1 of the inverse
Legendre-Vandermonde matrix (the linear coefficients of the surrogate cuboid), the 1D
Schwarz variants of Sec. 4.3.1 and the interpolation matrices of Sec. 3.2.  Nothing here
touches the HIP library.

Levels count from 1 (root) to L (finest), as in the paper.  Vectors are flat float64 arrays
in element-major layout with i fastest.
"""
import ctypes
import os
import subprocess

import numpy as np

from .gll import gll, diff_matrix, legendre
from .schwarz import variant_1d
from .transfer import degree_chain, interp_1d

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, 'o1.c')
LIB = os.path.join(HERE, 'libo1.so')
NSMAX = 24
SIDES = ('i', 'd', 'n')


def build(verbose=False):
    """Compile o1.c with gcc and OpenMP into oracle/libo1.so."""
    tmp = LIB + '.tmp'
    cmd = ['gcc', '-O3', '-fopenmp', '-fPIC', '-shared', '-std=c99', '-Wall', '-o', tmp, SRC, '-lm']
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError('O1 build failed: %s\n%s%s' % (' '.join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print('built', LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        V, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.o1_create.restype = V
        L.o1_create.argtypes = [I, V, I, V, V, D, D, D]
        L.o1_set_level.argtypes = [V, I, V, V, V, V, V, I, V, V, V, V, V, I, V, V]
        L.o1_set_coords.restype = I
        L.o1_set_coords.argtypes = [V, V]
        L.o1_destroy.argtypes = [V]
        L.o1_apply.argtypes = [V, I, V, V]
        L.o1_residual.argtypes = [V, I, V, V, V]
        L.o1_rhs.argtypes = [V, V, V, V]
        L.o1_schwarz.argtypes = [V, I, V, V]
        L.o1_transfer.argtypes = [V, I, I, V, V]
        L.o1_smooth.argtypes = [V, I, I, V, V, I]
        L.o1_solve.restype = I
        L.o1_solve.argtypes = [V, V, V, I, I, I, I, D, I, D, V, V]
        L.o1_threads.restype = I
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data


def _legendre_rows(p):
    """Rows 0 and 1 of the inverse of V[q, i] = L_i(x_q): the Legendre coefficients 0 and 1."""
    x, _ = gll(p)
    Vm = np.stack([legendre(i, x)[0] for i in range(p + 1)], axis=1)
    Vinv = np.linalg.inv(Vm)
    return np.ascontiguousarray(Vinv[0]), np.ascontiguousarray(Vinv[1])


class O1:
    """Uniform-degree mesh of degree p with global p-coarsening p_{l-1} = max(1, p_l // 2).

    X: (E, 3, n, n, n) coordinates at the oracle's GLL nodes; nbr, bc: (E, 6).  The overlap is m
    on every level (capped at the degree), or with `delta` the number of the neighbour's GLL
    nodes with (1 + xi)/2 <= delta at each level's degree (Sec. 4.3.1 item 3)."""

    def __init__(self, p, X, nbr, bc, m=1, kappa=0.0, nu=1.0, mu_star=2.0, delta=None):
        from .schwarz import overlap_layers
        self.L = lib()
        self.chain = degree_chain(p)
        self.E = int(np.asarray(X).shape[0])
        self.nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        self.bc = np.ascontiguousarray(bc, dtype=np.int32)
        deg = np.array(self.chain, dtype=np.int32)
        self.h = self.L.o1_create(len(deg), _p(deg), self.E, _p(self.nbr), _p(self.bc), kappa, nu, mu_star)
        self._keep = [deg]
        for li, pl in enumerate(self.chain):
            n = pl + 1
            x, w = gll(pl)
            Dm = np.ascontiguousarray(diff_matrix(pl))
            v0, v1 = _legendre_rows(pl)
            ml = min(overlap_layers(pl, delta) if delta is not None else m, pl)
            nv = np.zeros(9, dtype=np.int32)
            mp = -np.ones((9, NSMAX), dtype=np.int32)
            S = np.zeros((9, NSMAX * NSMAX))
            lam = np.ones((9, NSMAX))
            W = np.zeros((9, NSMAX))
            for a, left in enumerate(SIDES):
                for b, right in enumerate(SIDES):
                    v = variant_1d(pl, ml, left, right, mu_star)
                    k = a * 3 + b
                    ns = len(v['nodes'])
                    nv[k] = ns
                    mp[k, :ns] = [(d + 1) * 64 + loc for d, loc in v['nodes']]
                    S[k, :ns * ns] = v['S'].ravel()
                    lam[k, :ns] = v['lam']
                    W[k, :ns] = v['W']
            if li > 0:
                pc = self.chain[li - 1]
                P = np.ascontiguousarray(interp_1d(pl, pc))
                I = np.ascontiguousarray(interp_1d(pc, pl))
                nc = pc + 1
            else:
                P = I = np.zeros(1)
                nc = 0
            arrs = [x, w, Dm, v0, v1, nv, mp, S, lam, W, P, I]
            arrs = [np.ascontiguousarray(a) for a in arrs]
            self._keep += arrs
            x, w, Dm, v0, v1, nv, mp, S, lam, W, P, I = arrs
            self.L.o1_set_level(self.h, li, _p(x), _p(w), _p(Dm), _p(v0), _p(v1), ml, _p(nv), _p(mp), _p(S),
                                _p(lam), _p(W), nc, _p(P), _p(I))
        Xc = np.ascontiguousarray(X, dtype=np.float64)
        if self.L.o1_set_coords(self.h, _p(Xc)) != 0:
            raise ValueError('map is not orientation preserving')
        self.ndof = {l + 1: self.E * (pl + 1) ** 3 for l, pl in enumerate(self.chain)}

    def close(self):
        if getattr(self, 'h', None):
            self.L.o1_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_levels(self):
        return len(self.chain)

    def _v(self, a, level):
        a = np.ascontiguousarray(a, dtype=np.float64).ravel()
        if a.size != self.ndof[level]:
            raise ValueError('vector of %d values, level %d has %d' % (a.size, level, self.ndof[level]))
        return a

    def apply(self, level, u):
        u = self._v(u, level)
        out = np.empty_like(u)
        self.L.o1_apply(self.h, level, _p(u), _p(out))
        return out

    def residual(self, level, u, g):
        u, g = self._v(u, level), self._v(g, level)
        out = np.empty_like(u)
        self.L.o1_residual(self.h, level, _p(u), _p(g), _p(out))
        return out

    def rhs(self, f, uD=None):
        L = self.n_levels
        f = self._v(f, L)
        uD = None if uD is None else self._v(uD, L)
        b = np.empty_like(f)
        self.L.o1_rhs(self.h, _p(f), None if uD is None else _p(uD), _p(b))
        return b

    def schwarz(self, level, r):
        r = self._v(r, level)
        z = np.empty_like(r)
        self.L.o1_schwarz(self.h, level, _p(r), _p(z))
        return z

    def project(self, level, u):
        u = self._v(u, level)
        out = np.empty(self.ndof[level - 1])
        self.L.o1_transfer(self.h, level, 0, _p(u), _p(out))
        return out

    def restrict(self, level, r):
        r = self._v(r, level)
        out = np.empty(self.ndof[level - 1])
        self.L.o1_transfer(self.h, level, 1, _p(r), _p(out))
        return out

    def prolong_add(self, level, uc, uf):
        uc = self._v(uc, level - 1)
        uf = self._v(uf, level).copy()
        self.L.o1_transfer(self.h, level, 2, _p(uc), _p(uf))
        return uf

    def smooth(self, level, u, g, n, smoother='was'):
        u = self._v(u, level).copy()
        g = self._v(g, level)
        self.L.o1_smooth(self.h, level, 0 if smoother == 'was' else 1, _p(u), _p(g), n)
        return u

    def solve(self, f, u0=None, smoother='scg', ns1=3, ns2=2, root_maxit=500, root_rtol=1e-12, max_cycles=30,
              rtol=1e-10):
        """FAS V-cycles (Alg. 2); returns (u, history of relative residuals, root iterations)."""
        L = self.n_levels
        f = self._v(f, L)
        u = np.zeros_like(f) if u0 is None else self._v(u0, L).copy()
        hist = np.zeros(max_cycles + 1)
        its = np.zeros(max_cycles, dtype=np.int32)
        k = self.L.o1_solve(self.h, _p(u), _p(f), 0 if smoother == 'was' else 1, ns1, ns2, root_maxit, root_rtol,
                            max_cycles, rtol, _p(hist), _p(its))
        return u, hist[:k + 1].tolist(), its[:k].tolist()


def threads():
    return lib().o1_threads()
