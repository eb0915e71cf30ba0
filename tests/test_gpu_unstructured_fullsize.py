"""The unstructured path at the diamond benchmark's size (periodic [0, 2 pi)^3, 16 x 16 diamond
cells x 24 layers, p = 4: 30,720 elements, 3.84M DOF; the launch configuration bench.py times):
the operator against the oracle's on the whole mesh; the Schwarz method on 48 sampled
subdomain neighbourhoods, with the oracle building only the subdomains that reach them; and a
FAS-MG-SCG(8,4) solve whose final residual the oracle's operator confirms."""
import numpy as np
import pytest

from oracle import operator as oop
from oracle.gll import gll as ogll
from oracle.mesh import Mesh
from oracle.unstructured import TopoSchwarz, vertex_star
from paper_2608_14123_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')

P, NC, LAYERS = 4, 16, 24


@pytest.fixture(scope='module')
def setup():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2608_14123_amd import binding as B
    print('diamond full size: building meshes', flush=True)
    L = 2 * np.pi
    Xo = W.diamond_coords(NC, LAYERS, ogll(P)[0], length=L, height=L, shift_seed=1, rot_seed=2)
    nbr, nf, no, bc = W.face_connectivity(Xo, period=L)
    mesh = Mesh(P, Xo, nbr, bc, kappa=0.0, mu_star=5.0, nbr_face=nf, nbr_orient=no)
    Xl = W.diamond_coords(NC, LAYERS, B.gll(P)[0], length=L, height=L, shift_seed=1, rot_seed=2)
    o = B.default_options(kappa=0.0, null_space=1, mu_star=5.0, root_rtol=0.1, smoother=B.SCG, ns1=8, ns2=4)
    lib = B.Solver(np.full(len(Xl), P, np.int32), Xl, nbr, bc, o, nbr_face=nf, nbr_orient=no)
    yield B, mesh, lib
    lib.close()


def test_operator_at_full_size(setup):
    B, mesh, lib = setup
    print('diamond full size: operator', flush=True)
    u = np.random.default_rng(21).standard_normal(mesh.n_dof())
    ref = oop.apply(mesh, u).ravel()
    out = torch.empty(mesh.n_dof(), dtype=torch.float64, device='cuda')
    lib.apply(lib.n_levels, torch.from_numpy(u).cuda(), out)
    err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err


def test_schwarz_on_sampled_subdomains(setup):
    B, mesh, lib = setup
    print('diamond full size: schwarz', flush=True)
    rng = np.random.default_rng(22)
    r = rng.standard_normal(mesh.n_dof())
    z = torch.empty(mesh.n_dof(), dtype=torch.float64, device='cuda')
    lib.schwarz(lib.n_levels, torch.from_numpy(r).cuda(), z)
    zg = z.cpu().numpy().reshape(mesh.E, -1)
    n = mesh.n
    sample = rng.choice(mesh.E, size=48, replace=False)
    reach = set()
    for e in sample:
        for c in range(8):
            reach |= set(vertex_star(mesh, int(e), (c & 1, (c >> 1) & 1, c >> 2)))
    T = TopoSchwarz(mesh, 1, subset=sorted(reach))
    zo = T.apply(r).reshape(mesh.E, -1)
    err = np.abs(zg[sample] - zo[sample]).max() / np.abs(zo[sample]).max()
    assert err < 1e-12, err


def test_solve_residual_confirmed_by_the_oracle(setup):
    B, mesh, lib = setup
    print('diamond full size: solve', flush=True)
    b = W.uniform_nodal(mesh.n_dof(), 11)
    b -= b.mean()
    u = torch.zeros(mesh.n_dof(), dtype=torch.float64, device='cuda')
    hist, ok = lib.solve(u, torch.from_numpy(b).cuda(), max_cycles=12, rtol=1e-10)
    assert ok and len(hist) - 1 <= 8, list(hist)
    res = b - oop.apply(mesh, u.cpu().numpy()).ravel()
    assert np.linalg.norm(res) <= 2e-10 * np.linalg.norm(b), np.linalg.norm(res) / np.linalg.norm(b)
