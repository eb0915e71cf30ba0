"""Seeded synthetic workloads: mesh topology, vertex geometry, maps and RHS values.

This module holds no arithmetic of the discretisation or the solver.  It
produces the inputs of the boundary: neighbour tables of structured hex
grids, physical coordinates at caller-supplied reference points (each side
passes its own GLL nodes), analytic maps and seeded nodal data.

Element index: e = ex + nx * (ey + ny * ez).  Faces: 0:-x 1:+x 2:-y 3:+y 4:-z 5:+z.
Element-local nodes are lexicographic with i (along x) fastest, then j, k.
"""
import numpy as np

DIRICHLET, NEUMANN = 1, 2


def box_topology(nx, ny, nz, periodic=(False, False, False), bc_code=DIRICHLET):
    """Face-neighbour table (E, 6) int32 (-1 = boundary) and boundary codes (E, 6) int8."""
    E = nx * ny * nz
    ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing='ij')
    ex, ey, ez = ex.transpose(2, 1, 0).ravel(), ey.transpose(2, 1, 0).ravel(), ez.transpose(2, 1, 0).ravel()
    nbr = np.full((E, 6), -1, dtype=np.int32)
    dims = (nx, ny, nz)
    coords = [ex, ey, ez]
    for d in range(3):
        for s, step in ((0, -1), (1, 1)):
            c = [ex.copy(), ey.copy(), ez.copy()]
            c[d] = coords[d] + step
            if periodic[d]:
                c[d] %= dims[d]
                ok = np.ones(E, dtype=bool)
            else:
                ok = (c[d] >= 0) & (c[d] < dims[d])
            idx = c[0] + nx * (c[1] + ny * c[2])
            nbr[ok, 2 * d + s] = idx[ok]
    bc = np.where(nbr < 0, bc_code, 0).astype(np.int8)
    return nbr, bc


def box_vertices(nx, ny, nz, lengths=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
    """Vertex grid V[kz, ky, kx, 3] of a uniform box partition."""
    xs = [origin[d] + lengths[d] * np.arange(m + 1) / m for d, m in enumerate((nx, ny, nz))]
    V = np.empty((nz + 1, ny + 1, nx + 1, 3))
    V[..., 0] = xs[0][None, None, :]
    V[..., 1] = xs[1][None, :, None]
    V[..., 2] = xs[2][:, None, None]
    return V


def perturb_vertices(V, fraction, seed):
    """Displace every coordinate of every interior vertex by U[-fraction, fraction] * h_min.

    h_min is the shortest edge of the grid, so stretched elements keep their faces close to
    the box planes (a per-axis scale would tilt the short faces of 1:100 elements by up to
    ~88 degrees)."""
    rng = np.random.default_rng(seed)
    V = V.copy()
    h = min(np.diff(V[0, 0, :, 0]).min(), np.diff(V[0, :, 0, 1]).min(), np.diff(V[:, 0, 0, 2]).min())
    disp = rng.uniform(-fraction, fraction, size=V.shape) * h
    interior = np.zeros(V.shape[:3], dtype=bool)
    interior[1:-1, 1:-1, 1:-1] = True
    V[interior] += disp[interior]
    return V


def element_coords(V, xi, map_fn=None):
    """Coordinates (E, 3, n, n, n) at tensor points xi (1D, ascending) of every element.

    Trilinear interpolation of the vertex grid (one direction at a time), then the optional
    pointwise map.
    """
    xi = np.asarray(xi, dtype=np.float64)
    nz, ny, nx = (s - 1 for s in V.shape[:3])
    lo, hi = 0.5 * (1.0 - xi), 0.5 * (1.0 + xi)
    E, n = nx * ny * nz, len(xi)
    V = np.asarray(V, dtype=np.float64)
    # along x: (nz+1, ny+1, nx, n_i, 3)
    A = lo[None, None, None, :, None] * V[:, :, :-1, None, :] + hi[None, None, None, :, None] * V[:, :, 1:, None, :]
    # along y: (nz+1, ny, n_j, nx, n_i, 3)
    Bv = (lo[None, None, :, None, None, None] * A[:, :-1, None] + hi[None, None, :, None, None, None] * A[:, 1:, None])
    del A
    # along z: (nz, n_k, ny, n_j, nx, n_i, 3)
    C = (lo[None, :, None, None, None, None, None] * Bv[:-1, None] + hi[None, :, None, None, None, None, None] * Bv[1:, None])
    del Bv
    X = C.transpose(0, 2, 4, 1, 3, 5, 6).reshape(E, n, n, n, 3)    # (ez, ey, ex, k, j, i, coord)
    del C
    if map_fn is not None:
        X = map_fn(X)
    return np.ascontiguousarray(np.moveaxis(X, -1, 1))


def sine_bump_map(X, amplitude=0.1):
    """x'_a = x_a + amplitude * sin(2 pi x) sin(2 pi y) sin(2 pi z) for every component a."""
    s = amplitude * np.sin(2 * np.pi * X[..., 0]) * np.sin(2 * np.pi * X[..., 1]) * np.sin(2 * np.pi * X[..., 2])
    return X + s[..., None]


def seeded_bump_map(seed, amplitude=(0.04, 0.08)):
    """A random member of the sine-bump family, zero on the boundary of the unit cube:
    x'_a = x_a + c_a prod_d sin(pi k_ad x_d) with amplitudes c_a (random sign) and wave
    numbers k_ad in {1, 2} drawn from `seed`."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(amplitude[0], amplitude[1], size=3) * rng.choice([-1.0, 1.0], size=3)
    k = rng.integers(1, 3, size=(3, 3))

    def fn(X):
        Y = X.copy()
        for a in range(3):
            s = np.ones(X.shape[:-1])
            for d in range(3):
                s = s * np.sin(np.pi * k[a, d] * X[..., d])
            Y[..., a] += amp[a] * s
        return Y
    return fn


def uniform_nodal(shape, seed):
    """Nodal values ~ U[-1, 1] from numpy's PCG64 with the given seed."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=shape)


def sine_solution(X, k=np.pi):
    """u = sin(k x) sin(k y) sin(k z) at coordinates X (E, 3, ...)."""
    return np.sin(k * X[:, 0]) * np.sin(k * X[:, 1]) * np.sin(k * X[:, 2])


# --- named workloads -----------------------------------------------------------------

def cosine_diffusivity(X, k=2 * np.pi):
    """nu = 1 + cos(k x) cos(k y) cos(k z) at coordinates X (E, 3, ...): the variable
    diffusivity of the paper's blade case (Sec. 6.2.5), between 0 and 2."""
    return 1.0 + np.cos(k * X[:, 0]) * np.cos(k * X[:, 1]) * np.cos(k * X[:, 2])


def cosine_diffusivity_source(X, k=2 * np.pi, kappa=1.0):
    """f = kappa u - div(nu grad u) for u = sine_solution(X, k) and nu = cosine_diffusivity(X, k):
    with s_a = sin(k x_a), c_a = cos(k x_a), grad nu . grad u = -3 k^2 (s c)_1 (s c)_2 (s c)_3
    and nu lap u = -3 k^2 nu u."""
    s = [np.sin(k * X[:, a]) for a in range(3)]
    c = [np.cos(k * X[:, a]) for a in range(3)]
    u = s[0] * s[1] * s[2]
    nu = 1.0 + c[0] * c[1] * c[2]
    return kappa * u + 3.0 * k * k * nu * u + 3.0 * k * k * (s[0] * c[0]) * (s[1] * c[1]) * (s[2] * c[2])


def local_refine_lists(ne, zones):
    """Element ids to refine per local step on an ne^3 box mesh of the unit cube: on the grid of
    step k (ne 2^k cells per axis) the active cells whose centre lies within zone k's radius of
    its centre and whose in-domain 3 x 3 x 3 block is all active.  Cells are numbered as the
    library numbers the levels it builds: the base e = ex + ne (ey + ne ez), a refined level
    parent by parent in id order with children c = bx + 2 by + 4 bz; the block of a refined
    cell is refined irregularly (frozen children).  zones: [(centre, radius), ...] in the
    unmapped unit cube."""
    offs = [(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1) if (a, b, c) != (0, 0, 0)]
    e = np.arange(ne ** 3)
    cells = np.stack([e % ne, (e // ne) % ne, e // (ne * ne)], axis=1)
    frozen = np.zeros(len(cells), dtype=bool)
    n = ne
    out = []
    for centre, radius in zones:
        index = {tuple(c): i for i, c in enumerate(cells)}
        mid = (cells + 0.5) / n
        want = (np.linalg.norm(mid - np.asarray(centre), axis=1) < radius) & ~frozen
        marked = np.zeros(len(cells), dtype=bool)
        for i in np.nonzero(want)[0]:
            ok = True
            for o in offs:
                nb = cells[i] + o
                if np.all((nb >= 0) & (nb < n)):
                    j = index.get(tuple(nb), -1)
                    ok = ok and j >= 0 and not frozen[j]
            marked[i] = ok
        irregular = np.zeros(len(cells), dtype=bool)
        for i in np.nonzero(marked)[0]:
            for o in offs:
                j = index.get(tuple(cells[i] + o), -1)
                if j >= 0 and not marked[j]:
                    irregular[j] = True
        out.append(np.nonzero(marked)[0].astype(np.int32))
        parents = np.nonzero(marked | irregular)[0]
        kids = np.array([[c & 1, (c >> 1) & 1, c >> 2] for c in range(8)])
        cells = (2 * cells[parents][:, None, :] + kids[None]).reshape(-1, 3)
        frozen = np.repeat(irregular[parents], 8)
        n *= 2
    return out


def gaussian_source(X, centre=(0.5, 0.5, 0.5), a=50.0):
    """f = exp(-a |x - centre|^2) at coordinates X (E, 3, ...): a localised source."""
    d2 = sum((X[:, k] - centre[k]) ** 2 for k in range(3))
    return np.exp(-a * d2)


def cartesian_unit_cube(ne):
    """ne^3 uniform cubes on [0,1]^3 with Dirichlet boundary."""
    nbr, bc = box_topology(ne, ne, ne)
    return box_vertices(ne, ne, ne), nbr, bc


def curved_cube(ne):
    """ne^3 elements on [0,1]^3 under the sine-bump map (boundary fixed by the map)."""
    nbr, bc = box_topology(ne, ne, ne)
    return box_vertices(ne, ne, ne), nbr, bc, sine_bump_map


def stretched_perturbed(ne, aspect=100.0, fraction=0.2, seed=4):
    """ne^3 elements on [0,1]^2 x [0,aspect] with interior vertices perturbed."""
    nbr, bc = box_topology(ne, ne, ne)
    V = box_vertices(ne, ne, ne, lengths=(1.0, 1.0, aspect))
    return perturb_vertices(V, fraction, seed), nbr, bc


# --- hp-adaptive spherical front (degrees per element) ---------------------------------

def front_degrees(ne, center=(0.0, 0.0, 0.0), r0=0.7, pmin=2, pmax=8):
    """Degree per element of ne^3 cubes on [0,1]^3: d_e = distance of the element box from the
    sphere |x - c| = r0, p_e = max(pmin, pmax - floor(d_e / h)); elements cut by the sphere get pmax."""
    h = 1.0 / ne
    idx = np.arange(ne)
    ex, ey, ez = np.meshgrid(idx, idx, idx, indexing='ij')
    ex, ey, ez = (a.transpose(2, 1, 0).ravel() for a in (ex, ey, ez))
    lo = np.stack([ex, ey, ez], 1) * h - np.asarray(center)
    hi = lo + h
    near = np.where(lo > 0, lo, np.where(hi < 0, -hi, 0.0))       # closest point offsets
    far = np.maximum(np.abs(lo), np.abs(hi))
    rmin = np.linalg.norm(near, axis=1)
    rmax = np.linalg.norm(far, axis=1)
    d = np.where(rmax < r0, r0 - rmax, np.where(rmin > r0, rmin - r0, 0.0))
    return np.maximum(pmin, pmax - np.floor(d / h + 1e-12).astype(np.int64)).astype(np.int32)


def front_solution(X, alpha=50.0, r0=0.7, center=(0.0, 0.0, 0.0)):
    """u = atan(alpha (|x - c| - r0)) at coordinates X (3, ...)."""
    rho = np.sqrt(sum((X[a] - center[a]) ** 2 for a in range(3)))
    return np.arctan(alpha * (rho - r0))


def front_source(X, alpha=50.0, r0=0.7, center=(0.0, 0.0, 0.0), rho_min=1e-6):
    """f = -laplace(u) for the spherical front, with rho clipped at rho_min at the centre."""
    rho = np.maximum(np.sqrt(sum((X[a] - center[a]) ** 2 for a in range(3))), rho_min)
    s = alpha * (rho - r0)
    du = alpha / (1.0 + s * s)
    d2u = -2.0 * alpha ** 3 * (rho - r0) / (1.0 + s * s) ** 2
    return -(d2u + 2.0 * du / rho)


def element_coords_mixed(V, degrees, xi_of, map_fn=None):
    """Coordinates per element at the reference points xi_of(p) of its own degree (list of (3,n,n,n))."""
    nz, ny, nx = (s - 1 for s in V.shape[:3])
    out = []
    cache = {}
    for e, p in enumerate(np.asarray(degrees)):
        p = int(p)
        if p not in cache:
            cache[p] = element_coords(V, xi_of(p), map_fn)
        out.append(cache[p][e])
    return out


def front_workload(ne, xi_of, center=(0.0, 0.0, 0.0), r0=0.7, alpha=50.0):
    """The hp front problem on ne^3 unit cubes: degrees by `front_degrees`, coordinates per
    element at xi_of(p_e), f = -laplace(u) and u_D = u of the spherical front, nodal."""
    degrees = front_degrees(ne, center=center, r0=r0)
    nbr, bc = box_topology(ne, ne, ne)
    X = element_coords_mixed(box_vertices(ne, ne, ne), degrees, xi_of)
    f = np.concatenate([front_source(x, alpha=alpha, r0=r0, center=center).ravel() for x in X])
    uD = np.concatenate([front_solution(x, alpha=alpha, r0=r0, center=center).ravel() for x in X])
    return degrees, X, nbr, bc, f, uD



# --- unstructured topology: face orientation and the extruded diamond mesh ----------------
#
# Face-node layout (first, second) of face phi: phi 0/1 -> (k, j), 2/3 -> (k, i), 4/5 -> (j, i).
# Orientation code o of a face seen from element e toward its neighbour's face nf: bit 0 = T,
# bit 1 = F1, bit 2 = F2.  The node (a, b) of e's face is the neighbour's face node (a', b') with
# (x, y) = (b, a) if T else (a, b), a' = n-1-x if F1 else x, b' = n-1-y if F2 else y.
# Aligned neighbours (the structured grids above) have nf = phi ^ 1 and o = 0.

def _rotations():
    """The 24 proper rotations of the reference cube as signed permutation matrices."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int64)
            for r in range(3):
                R[r, perm[r]] = signs[r]
            if round(np.linalg.det(R)) == 1:
                out.append(R)
    return out


ROTATIONS = _rotations()


def rotate_local_axes(X, rot):
    """Renumber every element's nodes by a proper rotation of its reference cube.

    X (E, 3, n, n, n) [e, coord, k, j, i]; rot (E,) indices into ROTATIONS.  The new node
    q' = (i', j', k') takes the old node q = R (q' - c) + c, c = (n - 1)/2, so the element, its
    geometry and the sign of its Jacobian are unchanged, only its local axes turn."""
    X = np.asarray(X)
    E, n = X.shape[0], X.shape[2]
    g = np.arange(n)
    K, J, I = np.meshgrid(g, g, g, indexing='ij')
    qp = np.stack([I, J, K], axis=-1).reshape(-1, 3)          # (n^3, 3) in (i, j, k)
    out = np.empty_like(X)
    for r, R in enumerate(ROTATIONS):
        sel = np.nonzero(np.asarray(rot) == r)[0]
        if len(sel) == 0:
            continue
        q = (qp * 2 - (n - 1)) @ R.T                            # 2 R (q' - c)
        q = (q + (n - 1)) // 2
        src = (q[:, 2] * n + q[:, 1]) * n + q[:, 0]
        flat = X[sel].reshape(len(sel), 3, n ** 3)
        out[sel] = flat[:, :, src].reshape(len(sel), 3, n, n, n)
    return out


def face_array(V, phi):
    """Face-phi node layer of V[..., k, j, i] in the layout (first, second) above."""
    s = 0 if phi % 2 == 0 else -1
    if phi < 2:
        return V[..., :, :, s]
    if phi < 4:
        return V[..., :, s, :]
    return V[..., s, :, :]


def orient_index(n, o):
    """Index arrays (ap, bp) with neighbour face node (ap[a, b], bp[a, b]) for our node (a, b)."""
    A, B = np.meshgrid(np.arange(n), np.arange(n), indexing='ij')
    x, y = (B, A) if o & 1 else (A, B)
    ap = n - 1 - x if o & 2 else x
    bp = n - 1 - y if o & 4 else y
    return ap, bp


def face_connectivity(X, period=None, bc_code=DIRICHLET, tol=1e-9):
    """Neighbour table from the element coordinates alone, by matching face nodes.

    X (E, 3, n, n, n); period: None, or the box side length(s) of a periodic domain (faces
    then match modulo the period).  Returns nbr (E, 6) int32 (-1 boundary), nbr_face (E, 6)
    int8, nbr_orient (E, 6) int8 and bc (E, 6) int8."""
    X = np.asarray(X, dtype=np.float64)
    E, n = X.shape[0], X.shape[2]
    per = None if period is None else np.broadcast_to(np.asarray(period, dtype=np.float64), (3,))
    scale = max(1.0, float(np.abs(X).max()))
    q = tol * scale * 1e3
    F = np.stack([face_array(X, phi) for phi in range(6)], axis=1)        # (E, 6, 3, n, n)
    # pair the faces by their centroids (faces of a valid mesh do not share one), wrapped
    c = F.reshape(E, 6, 3, -1).mean(axis=3)
    if per is not None:
        c = c - per * np.floor(c / per + 0.5 * q / per)
    key = np.round(c / q).astype(np.int64)
    if per is not None:
        key = key % np.round(per / q).astype(np.int64)
    flat = key.reshape(-1, 3)
    _, inv, cnt = np.unique(flat, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    if np.any(cnt > 2):
        raise ValueError('a face is shared by %d element faces' % cnt.max())
    order = np.argsort(inv, kind='stable')
    grp = inv[order]
    first = np.nonzero((grp[1:] == grp[:-1]))[0]
    a, b = order[first], order[first + 1]                                  # paired (e * 6 + phi)
    nbr = np.full(E * 6, -1, dtype=np.int32)
    nbf = np.full(E * 6, -1, dtype=np.int8)
    nbo = np.zeros(E * 6, dtype=np.int8)
    Ff = F.reshape(E * 6, 3, n, n)
    for x, y in ((a, b), (b, a)):
        Fa, Fb = Ff[x], Ff[y]
        code = np.full(len(x), -1)
        hits = np.zeros(len(x), dtype=int)
        for o in range(8):
            ap, bp = orient_index(n, o)
            d = Fa - Fb[:, :, ap, bp]
            if per is not None:
                d = d - per[None, :, None, None] * np.round(d / per[None, :, None, None])
            ok = np.abs(d).reshape(len(x), -1).max(axis=1) <= tol * scale * 1e2
            code = np.where(ok, o, code)
            hits += ok
        if np.any(hits != 1):
            k = int(np.nonzero(hits != 1)[0][0])
            raise ValueError('element %d face %d: %d orientations match' % (x[k] // 6, x[k] % 6, hits[k]))
        nbr[x] = y // 6
        nbf[x] = y % 6
        nbo[x] = code
    nbr, nbf, nbo = nbr.reshape(E, 6), nbf.reshape(E, 6), nbo.reshape(E, 6)
    bc = np.where(nbr < 0, bc_code, 0).astype(np.int8)
    return nbr, nbf, nbo, bc


def diamond_quads(nc, rho=0.3, angle=0.0, shift_seed=None):
    """2D diamond cells: the unit cell is split into a central quadrilateral (a square of
    half-diagonal rho, turned by `angle` from the axes: the "diamond") and four trapezoids, one
    per side, whose corner angles at the cell corners are 45 degrees (for angle 0); the cells are
    repeated nc x nc over [0, nc]^2.  Returns vertices (Nv, 2) and quads (Q, 4)
    counter-clockwise; with shift_seed every quad starts at a random corner (a rotation of its
    local axes).  Cell corners are shared by 8 quads, the diamond's corners by 3."""
    corner = {}
    verts = []

    def cvert(x, y):
        k = (x, y)
        if k not in corner:
            corner[k] = len(verts)
            verts.append((float(x), float(y)))
        return corner[k]

    quads = []
    for cy in range(nc):
        for cx in range(nc):
            c00, c10, c11, c01 = cvert(cx, cy), cvert(cx + 1, cy), cvert(cx + 1, cy + 1), cvert(cx, cy + 1)
            ins = []
            for kk in range(4):
                th = 1.25 * np.pi + kk * 0.5 * np.pi + angle
                ins.append(len(verts))
                verts.append((cx + 0.5 + rho * np.cos(th), cy + 0.5 + rho * np.sin(th)))
            i0, i1, i2, i3 = ins
            quads += [[i0, i1, i2, i3], [c00, c10, i1, i0], [c10, c11, i2, i1], [c11, c01, i3, i2],
                      [c01, c00, i0, i3]]
    quads = np.array(quads, dtype=np.int64)
    if shift_seed is not None:
        s = np.random.default_rng(shift_seed).integers(0, 4, size=len(quads))
        quads = np.stack([np.roll(qd, -int(k)) for qd, k in zip(quads, s)])
    return np.array(verts), quads


def diamond_coords(nc, layers, xi, length=1.0, height=1.0, shift_seed=None, rot_seed=None):
    """Coordinates (E, 3, n, n, n) of the extruded diamond mesh at tensor points xi.

    nc x nc diamond cells (5 quads each) over [0, length]^2, extruded into `layers` layers over
    [0, height]; element e = layer * Q + quad.  Each quad is bilinear in (xi_1, xi_2) through its
    corners (-,-), (+,-), (+,+), (-,+); xi_3 runs along x_3.  rot_seed turns every element's
    local axes by a random proper rotation (ROTATIONS)."""
    V, quads = diamond_quads(nc, shift_seed=shift_seed)
    V = V * (length / nc)
    xi = np.asarray(xi, dtype=np.float64)
    n = len(xi)
    lo, hi = 0.5 * (1 - xi), 0.5 * (1 + xi)
    Q = len(quads)
    c = V[quads]                                              # (Q, 4, 2)
    # [q, j, i, 2]: bilinear in (xi_1 = i, xi_2 = j)
    P = (c[:, 0, None, None, :] * (lo[None, None, :, None] * lo[None, :, None, None])
         + c[:, 1, None, None, :] * (hi[None, None, :, None] * lo[None, :, None, None])
         + c[:, 2, None, None, :] * (hi[None, None, :, None] * hi[None, :, None, None])
         + c[:, 3, None, None, :] * (lo[None, None, :, None] * hi[None, :, None, None]))
    dz = height / layers
    X = np.empty((layers * Q, 3, n, n, n))
    for l in range(layers):
        z = l * dz + dz * hi
        X[l * Q:(l + 1) * Q, 0] = P[:, None, :, :, 0]
        X[l * Q:(l + 1) * Q, 1] = P[:, None, :, :, 1]
        X[l * Q:(l + 1) * Q, 2] = z[None, :, None, None]
    if rot_seed is not None:
        rot = np.random.default_rng(rot_seed).integers(0, len(ROTATIONS), size=len(X))
        X = rotate_local_axes(X, rot)
    return X
