"""Shared set-up for the GPU parity tests: the same seeded workload built twice.

The oracle side evaluates the workload geometry at the oracle's GLL nodes; the
library side at the library's own GLL nodes (dgfas_gll).  Nothing computed by
the library ever feeds the oracle.
"""
import numpy as np

from oracle import solvers as osv
from oracle.gll import gll as oracle_gll
from oracle.mesh import Mesh
from paper_2608_14123_amd import workloads as W


class Case:
    def __init__(self, name, p, ne, amp=0.0, bc_code=1, kappa=0.0, mu_star=2.0, periodic=False, lengths=(1, 1, 1),
                 perturb=None, m=1, weighting='quintic', delta=None):
        self.name, self.p, self.ne, self.amp = name, p, ne, amp
        self.kappa, self.mu_star, self.m = kappa, mu_star, m
        self.weighting, self.delta = weighting, delta
        self.nbr, self.bc = W.box_topology(ne, ne, ne, periodic=(periodic,) * 3, bc_code=bc_code)
        V = W.box_vertices(ne, ne, ne, lengths=lengths)
        if perturb is not None:
            V = W.perturb_vertices(V, perturb[0], perturb[1])
        self.V = V
        self.map = (lambda X: W.sine_bump_map(X, amp)) if amp else None
        self.E = ne ** 3

    def coords(self, xi):
        return W.element_coords(self.V, xi, self.map)

    def oracle_levels(self):
        X = self.coords(oracle_gll(self.p)[0])
        return osv.build_levels(self.p, X, self.nbr, self.bc, m=self.m, kappa=self.kappa, mu_star=self.mu_star,
                                weighting=self.weighting, delta=self.delta)

    def library(self, binding, **opt):
        X = self.coords(binding.gll(self.p)[0])
        extra = dict(weighting=binding.WEIGHT_PLAIN if self.weighting == 'plain' else binding.WEIGHT_QUINTIC)
        if self.delta is not None:
            extra.update(overlap=-1, delta=self.delta)
        else:
            extra.update(overlap=self.m)
        o = binding.default_options(kappa=self.kappa, mu_star=self.mu_star, **extra, **opt)
        return binding.Solver(np.full(self.E, self.p, dtype=np.int32), X, self.nbr, self.bc, o)

    def __repr__(self):
        return self.name


CASES = [
    Case('cart_p4_4^3', 4, 4),
    Case('curved_p3_3^3', 3, 3, amp=0.03),
    Case('curved_p7_3^3', 7, 3, amp=0.03),
    Case('curved_p8_2^3', 8, 2, amp=0.03),
    Case('curved_p2_5^3', 2, 5, amp=0.02),
    Case('neumann_kappa_p5_3^3', 5, 3, amp=0.03, bc_code=2, kappa=0.7),
    Case('neumann_kappa_p7_3^3', 7, 3, amp=0.03, bc_code=2, kappa=0.7),
    Case('periodic_p7_4^3', 7, 4, periodic=True, kappa=0.5),
    Case('stretched_p8_3^3', 8, 3, lengths=(1.0, 1.0, 100.0), perturb=(0.2, 4), mu_star=5.0),
]


def block_submesh(X_full, nbr_full, bc_full, ne, center, radius, p, kappa=0.0, mu_star=2.0):
    """Oracle mesh on the (2r+1)^3 element block around `center` of an ne^3 box grid.

    Faces leaving the block become Dirichlet faces of the sub-mesh; elements
    within distance `radius - k` of the centre see exact data for anything that
    reaches k elements (operator: 1, Schwarz: 2, sweep: 3).
    """
    cx, cy, cz = center % ne, (center // ne) % ne, center // (ne * ne)
    rng = [range(max(0, c - radius), min(ne, c + radius + 1)) for c in (cx, cy, cz)]
    ids = [x + ne * (y + ne * z) for z in rng[2] for y in rng[1] for x in rng[0]]
    loc = {g: i for i, g in enumerate(ids)}
    nbr = np.full((len(ids), 6), -1, dtype=np.int64)
    bc = np.zeros((len(ids), 6), dtype=np.int64)
    for i, g in enumerate(ids):
        for f in range(6):
            en = nbr_full[g, f]
            if en >= 0 and en in loc:
                nbr[i, f] = loc[en]
            else:
                bc[i, f] = bc_full[g, f] if en < 0 else 1
    mesh = Mesh(p, X_full[ids], nbr, bc, kappa=kappa, mu_star=mu_star)
    return mesh, np.array(ids), loc[center]


class MixedCase:
    """A box mesh with a degree per element (element-major vectors with offsets)."""

    def __init__(self, name, ne, degrees, amp=0.0, bc_code=1, kappa=0.0, mu_star=2.0, m=1):
        self.name, self.ne = name, ne
        self.degrees = np.asarray(degrees, dtype=np.int32)
        self.kappa, self.mu_star, self.m = kappa, mu_star, m
        self.nbr, self.bc = W.box_topology(ne, ne, ne, bc_code=bc_code)
        self.V = W.box_vertices(ne, ne, ne)
        self.map = (lambda X: W.sine_bump_map(X, amp)) if amp else None
        self.E = ne ** 3
        n3 = (self.degrees.astype(np.int64) + 1) ** 3
        self.off = np.concatenate(([0], np.cumsum(n3)))

    def coords(self, xi_of):
        return W.element_coords_mixed(self.V, self.degrees, xi_of, self.map)

    def oracle_levels(self):
        from oracle import mixed as mx
        X = self.coords(lambda p: oracle_gll(p)[0])
        return mx.build_mixed_levels(self.degrees, X, self.nbr, self.bc, m=self.m, kappa=self.kappa,
                                     mu_star=self.mu_star)

    def library(self, binding, **opt):
        X = self.coords(lambda p: binding.gll(p)[0])
        flat = np.concatenate([x.ravel() for x in X])
        o = binding.default_options(kappa=self.kappa, mu_star=self.mu_star, overlap=self.m, **opt)
        return binding.Solver(self.degrees, flat, self.nbr, self.bc, o)

    def __repr__(self):
        return self.name


def mixed_block(case, center, radius):
    """Oracle MixedMesh on the (2r+1)^3 element block around `center` (faces leaving the
    block become Dirichlet faces), the block's element ids and the centre's local index."""
    from oracle import mixed as mx
    ne = case.ne
    cx, cy, cz = center % ne, (center // ne) % ne, center // (ne * ne)
    rng = [range(max(0, c - radius), min(ne, c + radius + 1)) for c in (cx, cy, cz)]
    ids = [x + ne * (y + ne * z) for z in rng[2] for y in rng[1] for x in rng[0]]
    loc = {g: i for i, g in enumerate(ids)}
    nbr = np.full((len(ids), 6), -1, dtype=np.int64)
    bc = np.zeros((len(ids), 6), dtype=np.int64)
    for i, g in enumerate(ids):
        for f in range(6):
            en = case.nbr[g, f]
            if en >= 0 and en in loc:
                nbr[i, f] = loc[en]
            else:
                bc[i, f] = case.bc[g, f] if en < 0 else 1
    # the block's own vertex grid lists its elements in the same order as ids
    Vb = case.V[rng[2][0]:rng[2][-1] + 2, rng[1][0]:rng[1][-1] + 2, rng[0][0]:rng[0][-1] + 2]
    degs = case.degrees[ids]
    X = W.element_coords_mixed(Vb, degs, lambda p: oracle_gll(p)[0], case.map)
    mesh = mx.MixedMesh(degs, X, nbr, bc, kappa=case.kappa, mu_star=case.mu_star)
    return mesh, np.array(ids), loc[center]
