"""ctypes binding of libdgfas.so (include/dgfas.h).

Argument marshalling only: every computation runs inside the HIP library.
Device vectors are passed as torch CUDA tensors (float64, contiguous); host
arrays as numpy arrays.  If the shared library is missing this module raises
at import time: there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libdgfas.so')

if not os.path.exists(LIB_PATH):
    raise ImportError("libdgfas.so not built: run __graft_entry__.build() (or "
                      "python paper_2608_14123_amd/csrc/build.py) first")
# The library links the HIP runtime by its soname, and torch ships its own copy under the same
# soname: whichever is loaded first serves both.  torch cannot initialise the GPU on a runtime
# loaded before it, so it is imported first whenever it is installed.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = ctypes.CDLL(LIB_PATH)

DGFAS_OK, DGFAS_ENOTCONV = 0, 1
DGFAS_EINVAL, DGFAS_ENOMEM, DGFAS_EHIP, DGFAS_EUNSUPPORTED, DGFAS_EBREAKDOWN = -1, -2, -3, -4, -5
INTERIOR, DIRICHLET, NEUMANN = 0, 1, 2
WAS, SCG = 0, 1
FP64, FP32, BF16, FP32_MFMA = 0, 1, 2, 3
BATCH_PER_DEGREE, BATCH_ONE_LAUNCH, BATCH_TUNED, BATCH_PERSISTENT = 0, 1, 2, 3
ORDER_NATURAL, ORDER_MORTON = 0, 1
START_NONE, START_CMG, START_FMG = 0, 1, 2
WEIGHT_QUINTIC, WEIGHT_PLAIN = 0, 1
PROJECT_INTERP, PROJECT_L2 = 0, 1

c_dp = ctypes.POINTER(ctypes.c_double)


class MeshDesc(ctypes.Structure):
    _fields_ = [('n_elem', ctypes.c_int32), ('degree', ctypes.c_void_p), ('coords', ctypes.c_void_p),
                ('face_nbr', ctypes.c_void_p), ('face_bc', ctypes.c_void_p), ('box', ctypes.c_int32 * 3),
                ('nu_nodal', ctypes.c_void_p), ('refine_count', ctypes.c_void_p), ('refine_list', ctypes.c_void_p),
                ('face_nbr_face', ctypes.c_void_p), ('face_orient', ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [('kappa', ctypes.c_double), ('nu', ctypes.c_double), ('mu_star', ctypes.c_double),
                ('overlap', ctypes.c_int32), ('smoother', ctypes.c_int32), ('ns1', ctypes.c_int32),
                ('ns2', ctypes.c_int32), ('root_max_iter', ctypes.c_int32), ('root_rtol', ctypes.c_double),
                ('precision', ctypes.c_int32), ('n_rhs', ctypes.c_int32), ('batch', ctypes.c_int32),
                ('graph', ctypes.c_int32), ('order', ctypes.c_int32), ('start', ctypes.c_int32),
                ('ns0', ctypes.c_int32), ('nsc', ctypes.c_int32), ('weighting', ctypes.c_int32),
                ('delta', ctypes.c_double), ('projection', ctypes.c_int32), ('h_levels', ctypes.c_int32),
                ('h_only', ctypes.c_int32), ('local_steps', ctypes.c_int32), ('null_space', ctypes.c_int32)]


class DgfasError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__('dgfas error %d: %s' % (code, msg))
        self.code = code


_V = ctypes.c_void_p
_I = ctypes.c_int32
_sig = {
    'dgfas_default_options': (None, [ctypes.POINTER(Options)]),
    'dgfas_gll': (_I, [_I, c_dp, c_dp]),
    'dgfas_schwarz_tables_1d': (_I, [_I, _I, _I, _I, ctypes.c_double, ctypes.POINTER(_I), c_dp, c_dp, c_dp]),
    'dgfas_create': (_I, [ctypes.POINTER(MeshDesc), ctypes.POINTER(Options), _V, ctypes.POINTER(_V)]),
    'dgfas_destroy': (None, [_V]),
    'dgfas_levels': (_I, [_V, ctypes.POINTER(_I)]),
    'dgfas_level_info': (_I, [_V, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_int64)]),
    'dgfas_level_overlap': (_I, [_V, _I, ctypes.POINTER(_I)]),
    'dgfas_level_blocks': (_I, [_V, _I, ctypes.POINTER(ctypes.c_int64)]),
    'dgfas_workspace_size': (_I, [_V, ctypes.POINTER(ctypes.c_size_t)]),
    'dgfas_set_workspace': (_I, [_V, _V, ctypes.c_size_t]),
    'dgfas_rhs': (_I, [_V, _V, _V, _V, _V]),
    'dgfas_level_classes': (_I, [_V, _I, _V]),
    'dgfas_level_coords': (_I, [_V, _I, c_dp]),
    'dgfas_level_rhs': (_I, [_V, _I, _V, _V, _V, _V]),
    'dgfas_set_level_rhs': (_I, [_V, _I, _V]),
    'dgfas_level_solution': (_I, [_V, _I, _V]),
    'dgfas_apply': (_I, [_V, _I, _V, _V]),
    'dgfas_residual': (_I, [_V, _I, _V, _V, _V]),
    'dgfas_schwarz': (_I, [_V, _I, _V, _V]),
    'dgfas_schwarz_noalloc': (_I, [_V, _I, _V, _V]),
    'dgfas_smooth': (_I, [_V, _I, _V, _V, _I]),
    'dgfas_restrict': (_I, [_V, _I, _V, _V]),
    'dgfas_project': (_I, [_V, _I, _V, _V]),
    'dgfas_prolong_add': (_I, [_V, _I, _V, _V, _V]),
    'dgfas_root_solve': (_I, [_V, _V, _V, ctypes.POINTER(_I)]),
    'dgfas_vcycle': (_I, [_V, _V, _V]),
    'dgfas_startup': (_I, [_V, _V, _V]),
    'dgfas_solve': (_I, [_V, _V, _V, _I, ctypes.c_double, c_dp, ctypes.POINTER(_I)]),
    'dgfas_norm': (_I, [_V, _I, _V, c_dp]),
    'dgfas_autotune': (_I, [_V, ctypes.c_char_p, _I, c_dp]),
    'dgfas_last_error': (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sig)


def _check(code, warn_ok=False):
    if code == DGFAS_OK or (warn_ok and code > 0):
        return code
    raise DgfasError(code, _lib.dgfas_last_error().decode())


def _dev(t, n, name, dtype='float64'):
    """Device pointer of a contiguous GPU tensor of `dtype` with at least n elements (None
    passes through): the kernels take the pointer as it is, so a host tensor, another dtype
    or a short vector is refused here rather than read out of bounds on the device."""
    if t is None:
        return None
    if not hasattr(t, 'data_ptr') or not hasattr(t, 'is_cuda'):
        raise TypeError('%s: expected a torch tensor' % name)
    if not t.is_cuda:
        raise ValueError('%s: expected a device tensor' % name)
    if str(t.dtype) != 'torch.' + dtype:
        raise TypeError('%s: expected %s, got %s' % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError('%s: tensor must be contiguous' % name)
    if t.numel() < n:
        raise ValueError('%s: %d elements, at least %d needed' % (name, t.numel(), n))
    return t.data_ptr()


def default_options(**kw):
    o = Options()
    _lib.dgfas_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def gll(p):
    x = np.zeros(p + 1)
    w = np.zeros(p + 1)
    _check(_lib.dgfas_gll(p, x.ctypes.data_as(c_dp), w.ctypes.data_as(c_dp)))
    return x, w


def schwarz_tables_1d(p, m, left, right, mu_star):
    nsmax = p + 1 + 2 * m
    ns = _I()
    S = np.zeros(nsmax * nsmax)
    lam = np.zeros(nsmax)
    W = np.zeros(nsmax)
    _check(_lib.dgfas_schwarz_tables_1d(p, m, left, right, mu_star, ctypes.byref(ns), S.ctypes.data_as(c_dp),
                                        lam.ctypes.data_as(c_dp), W.ctypes.data_as(c_dp)))
    k = ns.value
    return S[:k * k].reshape(k, k), lam[:k], W[:k]


class Solver:
    """One level hierarchy on the current device (see dgfas_create)."""

    def __init__(self, degree, coords, face_nbr, face_bc, options=None, stream=None, box=None, nu=None,
                 refine=None, nbr_face=None, nbr_orient=None):
        """refine: with options.local_steps > 0, one list of element ids per refinement step
        (ids of the level being refined; see dgfas_mesh_desc.refine_list).  nbr_face, nbr_orient:
        (n_elem, 6) the neighbour's face and the relative orientation code of an unstructured mesh
        (dgfas_mesh_desc.face_nbr_face / face_orient)."""
        degree = np.ascontiguousarray(degree, dtype=np.int32)
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        face_nbr = np.ascontiguousarray(face_nbr, dtype=np.int32)
        face_bc = np.ascontiguousarray(face_bc, dtype=np.int8)
        E = len(degree)
        if face_nbr.shape != (E, 6) or face_bc.shape != (E, 6):
            raise ValueError('face tables must be (n_elem, 6)')
        if coords.size != int(3 * np.sum((degree.astype(np.int64) + 1) ** 3)):
            raise ValueError('coords must hold 3 (p_e+1)^3 values per element')
        if nu is not None:
            nu = np.ascontiguousarray(nu, dtype=np.float64)
            if nu.size * 3 != coords.size:
                raise ValueError('nu must hold (p_e+1)^3 values per element')
        rc = rl = None
        if refine is not None:
            rc = np.ascontiguousarray([len(r) for r in refine], dtype=np.int32)
            rl = np.ascontiguousarray(np.concatenate([np.asarray(r, dtype=np.int32) for r in refine])
                                      if len(refine) else np.zeros(0), dtype=np.int32)
        nf = no = None
        if nbr_face is not None:
            nf = np.ascontiguousarray(nbr_face, dtype=np.int8)
            if nf.shape != (E, 6):
                raise ValueError('nbr_face must be (n_elem, 6)')
        if nbr_orient is not None:
            no = np.ascontiguousarray(nbr_orient, dtype=np.int8)
            if no.shape != (E, 6):
                raise ValueError('nbr_orient must be (n_elem, 6)')
        self._keep = (degree, coords, face_nbr, face_bc, nu, rc, rl, nf, no)
        desc = MeshDesc(E, degree.ctypes.data, coords.ctypes.data, face_nbr.ctypes.data, face_bc.ctypes.data,
                        (ctypes.c_int32 * 3)(*(box or (0, 0, 0))), None if nu is None else nu.ctypes.data,
                        None if rc is None else rc.ctypes.data, None if rl is None or rl.size == 0 else rl.ctypes.data,
                        None if nf is None else nf.ctypes.data, None if no is None else no.ctypes.data)
        self.options = options if options is not None else default_options()
        h = _V()
        st = None if stream is None else _V(stream)
        _check(_lib.dgfas_create(ctypes.byref(desc), ctypes.byref(self.options), st, ctypes.byref(h)))
        self._h = h
        nl = _I()
        _check(_lib.dgfas_levels(self._h, ctypes.byref(nl)))
        self.n_levels = nl.value
        self.n_rhs = int(self.options.n_rhs)
        self._ndof = {l: self.level_info(l)[1] for l in range(1, self.n_levels + 1)}

    def _n(self, level):
        """Elements of a vector argument on `level`: n_rhs * n_dof."""
        if level not in self._ndof:
            raise ValueError('level %d outside 1..%d' % (level, self.n_levels))
        return self.n_rhs * self._ndof[level]

    def close(self):
        if getattr(self, '_h', None):
            _lib.dgfas_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level):
        d = _I()
        nd = ctypes.c_int64()
        _check(_lib.dgfas_level_info(self._h, level, ctypes.byref(d), ctypes.byref(nd)))
        return d.value, nd.value

    def workspace_size(self):
        n = ctypes.c_size_t()
        _check(_lib.dgfas_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    def set_workspace(self, buf):
        """Use a caller-owned device tensor (uint8, at least workspace_size() bytes) as the
        workspace, or None for a library-owned block; the tensor is kept alive here."""
        if buf is None:
            _check(_lib.dgfas_set_workspace(self._h, None, 0))
        else:
            _check(_lib.dgfas_set_workspace(self._h, _dev(buf, self.workspace_size(), 'workspace', 'uint8'),
                                            buf.numel()))
        self._ws = buf

    def level_overlap(self, level):
        m = _I()
        _check(_lib.dgfas_level_overlap(self._h, level, ctypes.byref(m)))
        return m.value

    def level_blocks(self, level):
        """Subdomain block counts of an unstructured level: (element, face, mapped, zero-filled,
        merged), summed over its subdomains (zeros on a structured level)."""
        c = (ctypes.c_int64 * 5)()
        _check(_lib.dgfas_level_blocks(self._h, level, c))
        return np.array(list(c), dtype=np.int64)

    def rhs(self, f, b, uD=None, qN=None):
        n = self._n(self.n_levels)
        _check(_lib.dgfas_rhs(self._h, _dev(f, n, 'f'), _dev(uD, n, 'uD'), _dev(qN, n, 'qN'), _dev(b, n, 'b')))

    def apply(self, level, u, Au):
        n = self._n(level)
        _check(_lib.dgfas_apply(self._h, level, _dev(u, n, 'u'), _dev(Au, n, 'Au')))

    def residual(self, level, u, g, r):
        n = self._n(level)
        _check(_lib.dgfas_residual(self._h, level, _dev(u, n, 'u'), _dev(g, n, 'g'), _dev(r, n, 'r')))

    def schwarz(self, level, r, z):
        n = self._n(level)
        _check(_lib.dgfas_schwarz(self._h, level, _dev(r, n, 'r'), _dev(z, n, 'z')))

    def schwarz_noalloc(self, level, r, z):
        """z = B r with the overlap inbox in the library's static device array (no allocation)."""
        n = self._n(level)
        _check(_lib.dgfas_schwarz_noalloc(self._h, level, _dev(r, n, 'r'), _dev(z, n, 'z')))

    def smooth(self, level, u, g, n_steps):
        n = self._n(level)
        _check(_lib.dgfas_smooth(self._h, level, _dev(u, n, 'u'), _dev(g, n, 'g'), n_steps))

    def restrict(self, level, r_fine, r_coarse):
        nf, nc = self._n(level), self._n(level - 1)
        _check(_lib.dgfas_restrict(self._h, level, _dev(r_fine, nf, 'r_fine'), _dev(r_coarse, nc, 'r_coarse')))

    def project(self, level, u_fine, u_coarse):
        nf, nc = self._n(level), self._n(level - 1)
        _check(_lib.dgfas_project(self._h, level, _dev(u_fine, nf, 'u_fine'), _dev(u_coarse, nc, 'u_coarse')))

    def prolong_add(self, level, u_coarse, u_fine, ubar=None):
        nf, nc = self._n(level), self._n(level - 1)
        _check(_lib.dgfas_prolong_add(self._h, level, _dev(u_coarse, nc, 'u_coarse'), _dev(ubar, nc, 'ubar'),
                                      _dev(u_fine, nf, 'u_fine')))

    def root_solve(self, u, g):
        n = self._n(1)
        it = _I()
        _check(_lib.dgfas_root_solve(self._h, _dev(u, n, 'u'), _dev(g, n, 'g'), ctypes.byref(it)))
        return it.value

    def startup(self, u, f):
        """The configured CMG / FMG start-up: u (finest level) receives the start value."""
        n = self._n(self.n_levels)
        _check(_lib.dgfas_startup(self._h, _dev(u, n, 'u'), _dev(f, n, 'f')))

    def vcycle(self, u, f):
        n = self._n(self.n_levels)
        _check(_lib.dgfas_vcycle(self._h, _dev(u, n, 'u'), _dev(f, n, 'f')))

    def level_classes(self, level):
        """Element classes of a level: 0 twig, 1 leaf, 2 frozen (numpy int8)."""
        E = self.level_elements(level)
        out = np.zeros(E, dtype=np.int8)
        _check(_lib.dgfas_level_classes(self._h, level, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def level_elements(self, level):
        deg = _I()
        nd = ctypes.c_int64()
        _check(_lib.dgfas_level_info(self._h, level, ctypes.byref(deg), ctypes.byref(nd)))
        return int(nd.value // (deg.value + 1) ** 3)

    def level_coords(self, level):
        """Nodal coordinates of a level, (n_elem, 3, n, n, n) numpy."""
        deg = _I()
        nd = ctypes.c_int64()
        _check(_lib.dgfas_level_info(self._h, level, ctypes.byref(deg), ctypes.byref(nd)))
        n = deg.value + 1
        out = np.zeros((nd.value // n ** 3, 3, n, n, n))
        _check(_lib.dgfas_level_coords(self._h, level, out.ctypes.data_as(c_dp)))
        return out

    def level_rhs(self, level, f, b, uD=None, qN=None):
        n = self._n(level)
        _check(_lib.dgfas_level_rhs(self._h, level, _dev(f, n, 'f'), _dev(uD, n, 'uD'), _dev(qN, n, 'qN'),
                                    _dev(b, n, 'b')))

    def set_level_rhs(self, level, b):
        _check(_lib.dgfas_set_level_rhs(self._h, level, _dev(b, self._n(level), 'b')))

    def level_solution(self, level, u):
        _check(_lib.dgfas_level_solution(self._h, level, _dev(u, self._n(level), 'u')))

    def solve(self, u, f, max_cycles=30, rtol=1e-10):
        hist, code = solve_status(self, u, f, max_cycles, rtol)
        return hist, code == DGFAS_OK

    def autotune(self, cache_path=None, reps=10):
        """Time per-degree, one-launch and persistent batches per level and stage (see
        dgfas_autotune); returns [n_levels][3][3] median times in ms."""
        rep = np.zeros((self.n_levels, 3, 3))
        path = None if cache_path is None else str(cache_path).encode()
        _check(_lib.dgfas_autotune(self._h, path, reps, rep.ctypes.data_as(c_dp)))
        return rep

    def norm(self, level, v):
        """Euclidean norm per right-hand side (numpy array of n_rhs values)."""
        out = np.zeros(self.options.n_rhs)
        _check(_lib.dgfas_norm(self._h, level, _dev(v, self._n(level), 'v'), out.ctypes.data_as(c_dp)))
        return out


_mlp_sig = {
    'dgfas_mlp_create': (_I, [_I, _I, _I, ctypes.c_uint64, _V, ctypes.POINTER(_V)]),
    'dgfas_mlp_destroy': (None, [_V]),
    'dgfas_mlp_num_params': (_I, [_V, ctypes.POINTER(ctypes.c_int64)]),
    'dgfas_mlp_get_params': (_I, [_V, _V]),
    'dgfas_mlp_set_params': (_I, [_V, _V]),
    'dgfas_mlp_forward': (_I, [_V, _V, _I, _V]),
    'dgfas_mlp_gradient': (_I, [_V, _V, _V, _I, _V, c_dp]),
    'dgfas_mlp_train': (_I, [_V, _V, _V, ctypes.c_int64, _I, _I, ctypes.c_float, ctypes.c_float, _I, c_dp]),
}
for _name, (_res, _args) in _mlp_sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
EXPORTED = EXPORTED + tuple(_mlp_sig)


class Mlp:
    """Learned subdomain-correction network (dgfas_mlp_*); device arrays are torch float32 tensors."""

    def __init__(self, n_in, n_hidden, n_out, seed=5, stream=None):
        h = _V()
        _check(_lib.dgfas_mlp_create(n_in, n_hidden, n_out, seed, None if stream is None else _V(stream),
                                     ctypes.byref(h)))
        self._h = h
        self.n_in, self.n_hidden, self.n_out = n_in, n_hidden, n_out
        n = ctypes.c_int64()
        _check(_lib.dgfas_mlp_num_params(self._h, ctypes.byref(n)))
        self.n_params = n.value

    def close(self):
        if getattr(self, '_h', None):
            _lib.dgfas_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(_lib.dgfas_mlp_get_params(self._h, out.ctypes.data))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        if theta.size != self.n_params:
            raise ValueError('wrong parameter count')
        _check(_lib.dgfas_mlp_set_params(self._h, theta.ctypes.data))

    def forward(self, X, Y):
        rows = X.shape[0]
        _check(_lib.dgfas_mlp_forward(self._h, _dev(X, rows * self.n_in, 'X', 'float32'), rows,
                                      _dev(Y, rows * self.n_out, 'Y', 'float32')))

    def gradient(self, X, T, grad=None):
        rows = X.shape[0]
        loss = ctypes.c_double()
        _check(_lib.dgfas_mlp_gradient(self._h, _dev(X, rows * self.n_in, 'X', 'float32'),
                                       _dev(T, rows * self.n_out, 'T', 'float32'), rows,
                                       _dev(grad, self.n_params, 'grad', 'float32'), ctypes.byref(loss)))
        return loss.value

    def train(self, X, T, batch, steps, lr0=1e-3, lr_min=1e-5, total_steps=None):
        rows = X.shape[0]
        losses = np.zeros(max(steps, 1))
        _check(_lib.dgfas_mlp_train(self._h, _dev(X, rows * self.n_in, 'X', 'float32'),
                                    _dev(T, rows * self.n_out, 'T', 'float32'), rows, batch, steps, lr0, lr_min,
                                    total_steps or steps, losses.ctypes.data_as(c_dp)))
        return losses[:steps]


_learn_sig = {
    'dgfas_set_learned': (_I, [_V, _V, _I]),
    'dgfas_learned_pairs': (_I, [_V, _V, _V, _I, _V, _V, ctypes.POINTER(_I)]),
}
for _name, (_res, _args) in _learn_sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
EXPORTED = EXPORTED + tuple(_learn_sig)
DGFAS_EFALLBACK = 2


def set_learned(solver, mlp, enabled=True, judge=True):
    code = (1 if judge else 2) if enabled else 0
    _check(_lib.dgfas_set_learned(solver._h, mlp._h if mlp is not None else None, code))


def learned_pairs(solver, r, centers, X, T):
    """Training pairs for the listed centre elements (numpy int array); returns PCG iterations."""
    c = np.ascontiguousarray(centers, dtype=np.int32)
    it = _I()
    # the library writes n (ns^3 + 9) values to X and n ns^3 to T, ns from its finest level
    L = solver.n_levels
    ns3 = (solver.level_info(L)[0] + 1 + 2 * solver.level_overlap(L)) ** 3
    _check(_lib.dgfas_learned_pairs(solver._h, _dev(r, solver._n(solver.n_levels), 'r'), c.ctypes.data, len(c),
                                    _dev(X, len(c) * (ns3 + 9), 'X', 'float32'), _dev(T, len(c) * ns3, 'T', 'float32'),
                                    ctypes.byref(it)))
    return it.value


def solve_status(solver, u, f, max_cycles=30, rtol=1e-10):
    """Like Solver.solve but also returns the status code (0 ok, 1 not converged, 2 fallback)."""
    hist = np.zeros(max_cycles + 1)
    nd = _I()
    n = solver._n(solver.n_levels)
    code = _check(_lib.dgfas_solve(solver._h, _dev(u, n, 'u'), _dev(f, n, 'f'), max_cycles, rtol,
                                   hist.ctypes.data_as(c_dp), ctypes.byref(nd)), warn_ok=True)
    return hist[:nd.value + 1], code
