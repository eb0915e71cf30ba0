"""SIPG operator, right-hand side and dense assembly (oracle; test infrastructure only).

Follows eq. helmholtz:dgm (Sec. 2.2) with GLL quadrature on every volume and
face integral (Remark on basis functions):

  volume   sum_q w_q J_q [ nu grad(phi_i).grad(u) + kappa phi_i u ]
  interior mu max(nu) [v].[u] - {nu grad v}.[u] - [v].{nu grad u}
  Dirichlet mu nu v 2u - nu (d_n v) u - nu v d_n u
  rhs      int v f + Dirichlet: mu nu v 2 u_D - nu (d_n v) u_D ; Neumann: v q_N

with [u] = n^- u^- + n^+ u^+ and {w} = (w^- + w^+)/2 (Sec. 2.2).  Each
element assembles its own rows; on an interior face it uses its own outward
normal n and the jump j = u_own - u_nbr.  The term -{nu grad v}.[u] for the
test functions of one element is its transposed face gradient ("lifting").
nu is given per node: at a face node the average is (nu^- d_n u^- + nu^+ d_n u^+)/2 with
each side's own nodal value, the penalty takes max(nu^-, nu^+) there, and the lifting of an
element's test functions its own value.
"""
import numpy as np

from .mesh import d_ref, dT_ref, face_view


def _face_dn(mesh, gradf, phi):
    """n_out . grad u at the face nodes, with this element's outward normal."""
    return np.einsum('eaxy,eaxy->exy', mesh.face_n[phi], gradf)


def _add_lifting(mesh, lift, sigma, phi):
    """Accumulate sigma_f * (n . grad xi_c)(x_f) at the face nodes of lift[c].

    sum_c D_c^T lift[c] then equals sum_f sigma_f (n . grad phi_q)(x_f) for every q.
    """
    nvec = mesh.face_n[phi]
    for c in range(3):
        dxi_c = face_view(np.moveaxis(mesh.dxi[..., c, :], -1, 1), phi)   # (E, 3, n, n): d xi_c / d x_a
        coef = np.einsum('eaxy,eaxy->exy', nvec, dxi_c)
        fv = face_view(lift[c], phi)
        fv += sigma * coef


def apply(mesh, u):
    """A u for the SIPG operator (eq. helmholtz:system). u: (E, n, n, n)."""
    u = np.asarray(u, dtype=np.float64).reshape(mesh.E, mesh.n, mesh.n, mesh.n)
    kappa = mesh.kappa
    nu_v = mesh.nu_n
    grad = mesh.grad(u)
    # volume term: sum_b D_b^T [ w J nu grad(xi_b) . grad u ] + kappa w J u
    out = kappa * mesh.w3 * mesh.detJ * u
    for b in range(3):
        flux_b = nu_v * mesh.w3 * mesh.detJ * np.einsum('ekjia,eakji->ekji', mesh.dxi[..., b, :], grad)
        out = out + dT_ref(mesh.D, flux_b, b)
    lift = [np.zeros_like(u) for _ in range(3)]
    for phi in range(6):
        ws = mesh.face_ws[phi]
        uf = face_view(u, phi)
        dn_own = _face_dn(mesh, face_view(grad, phi), phi)
        nb = mesh.nbr[:, phi]
        row = np.zeros_like(uf)
        sigma = np.zeros_like(uf)
        nu_o = face_view(mesh.nu_n, phi)
        inter = nb >= 0
        if np.any(inter):
            u_nb = mesh.neighbour_face(u, phi, inter)
            g_nb = mesh.neighbour_face(grad, phi, inter)
            dn_nb = np.einsum('eaxy,eaxy->exy', mesh.face_n[phi][inter], g_nb)   # own normal
            jmp = uf[inter] - u_nb
            mu = mesh.mu[inter, phi][:, None, None]
            wsi = ws[inter]
            nu_i, nu_n = nu_o[inter], mesh.neighbour_face(mesh.nu_n, phi, inter)
            row[inter] = mu * np.maximum(nu_i, nu_n) * wsi * jmp - 0.5 * wsi * (nu_i * dn_own[inter] + nu_n * dn_nb)
            sigma[inter] = -0.5 * nu_i * wsi * jmp
        dir_ = (nb < 0) & (mesh.bc[:, phi] == 1)
        if np.any(dir_):
            mu = mesh.mu[dir_, phi][:, None, None]
            wsd = ws[dir_]
            nu_d = nu_o[dir_]
            row[dir_] = 2.0 * mu * nu_d * wsd * uf[dir_] - wsd * nu_d * dn_own[dir_]
            sigma[dir_] = -nu_d * wsd * uf[dir_]
        # Neumann faces contribute nothing to the operator
        fv = face_view(out, phi)
        fv += row
        _add_lifting(mesh, lift, sigma, phi)
    for c in range(3):
        out = out + dT_ref(mesh.D, lift[c], c)
    return out


def rhs(mesh, f, uD=None, qN=None):
    """Right-hand side b of eq. helmholtz:system from nodal f, u_D and q_N values."""
    f = np.asarray(f, dtype=np.float64).reshape(mesh.E, mesh.n, mesh.n, mesh.n)
    b = mesh.w3 * mesh.detJ * f
    lift = [np.zeros_like(b) for _ in range(3)]
    for phi in range(6):
        nb = mesh.nbr[:, phi]
        ws = mesh.face_ws[phi]
        row = np.zeros_like(ws)
        sigma = np.zeros_like(ws)
        dir_ = (nb < 0) & (mesh.bc[:, phi] == 1)
        if uD is not None and np.any(dir_):
            ud = face_view(np.asarray(uD, dtype=np.float64).reshape(b.shape), phi)
            mu = mesh.mu[dir_, phi][:, None, None]
            nu_d = face_view(mesh.nu_n, phi)[dir_]
            row[dir_] = 2.0 * mu * nu_d * ws[dir_] * ud[dir_]
            sigma[dir_] = -nu_d * ws[dir_] * ud[dir_]
        neu = (nb < 0) & (mesh.bc[:, phi] == 2)
        if qN is not None and np.any(neu):
            qn = face_view(np.asarray(qN, dtype=np.float64).reshape(b.shape), phi)
            row[neu] = ws[neu] * qn[neu]
        fv = face_view(b, phi)
        fv += row
        _add_lifting(mesh, lift, sigma, phi)
    for c in range(3):
        b = b + dT_ref(mesh.D, lift[c], c)
    return b


def assemble(mesh):
    """Dense A by applying the operator to unit vectors (tiny meshes only)."""
    N = mesh.n_dof()
    A = np.empty((N, N))
    e = np.zeros(N)
    for j in range(N):
        e[j] = 1.0
        A[:, j] = apply(mesh, e).ravel()
        e[j] = 0.0
    return A


def l2_error(mesh, u, u_exact):
    """Discrete L2 norm of u - u_exact with GLL quadrature (Sec. 6.1 error norm)."""
    d = np.asarray(u).reshape(mesh.E, mesh.n, mesh.n, mesh.n) - u_exact
    return float(np.sqrt(np.sum(mesh.w3 * mesh.detJ * d * d)))
