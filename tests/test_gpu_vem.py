"""Virtual element matrices on the GPU (Sec. 3, eqs. discreteA and
discreteF) against the generator's, element by element, through the C-ABI.

For degrees k = 2, 3, 4 on a jittered 3^3 mesh (27 general hexahedra with
planar faces, viscosity log-uniform in [0.1, 10] per element): the local
stiffness A^K, the divergence rows B^K and the load F^K of the manufactured
solution.  The two implementations share no code (their quadrature rules,
monomial tables and the Helmholtz split of the vector monomials are built
independently), so they agree to rounding: the element computation inverts
monomial mass matrices whose condition numbers grow with k, and the bar is
1e-12 of the largest entry for A^K and B^K and 1e-11 for F^K (measured
spread 1e-14 and 1e-13 at k = 4).  A second case spans two of the library's
element chunks (18^3 elements at k = 2) and compares elements sampled from
both."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs.mesh import CubeMesh
from inputs.vem import element_matrices
from inputs.assemble import load_vector, u_curl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def vb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09770_amd import binding
    binding.load()
    return binding


def _gpu(vb, mesh, k, nu):
    E = mesh.nK
    N, nP = vb.vb_vem_dofs(k)
    X8 = torch.tensor(np.ascontiguousarray(mesh.verts[mesh.elem_verts].reshape(E, 24)), device=DEV)
    nut = torch.tensor(np.ascontiguousarray(nu), device=DEV)
    A = torch.zeros((E, N, N), dtype=torch.float64, device=DEV)
    B = torch.zeros((E, nP, N), dtype=torch.float64, device=DEV)
    F = torch.zeros((E, N), dtype=torch.float64, device=DEV)
    ctx = vb.vb_create()
    try:
        vb.vb_vem_element_matrices(ctx, k, X8, nut, A, B, F)
        torch.cuda.synchronize()
    finally:
        vb.vb_destroy(ctx)
    return A.cpu().numpy(), B.cpu().numpy(), F.cpu().numpy()


def _ref(mesh, k, el, nu):
    out = element_matrices(mesh, k, el, nu, keep=True)
    force = lambda P, e: 1.5 * np.pi ** 2 * nu[e][:, None, None] * u_curl(P)
    return out["A"], out["B"], load_vector(mesh, k, el, out["P0"], force)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("k", [2, 3, 4])
def test_element_matrices_match_the_generator(vb, k):
    print("vem case k =", k, flush=True)
    mesh = CubeMesh(3, jitter=0.15, seed=1)
    nu = 10 ** np.random.default_rng(k).uniform(-1, 1, mesh.nK)
    A, B, F = _gpu(vb, mesh, k, nu)
    Ar, Br, Fr = _ref(mesh, k, np.arange(mesh.nK), nu)
    assert A.shape == Ar.shape and B.shape == Br.shape
    assert _rel(A, Ar) < 1e-12, _rel(A, Ar)
    assert _rel(B, Br) < 1e-12, _rel(B, Br)
    assert _rel(F, Fr) < 1e-11, _rel(F, Fr)
    # the stiffness is symmetric
    assert np.abs(A - A.transpose(0, 2, 1)).max() < 1e-12 * np.abs(A).max()


def test_element_matrices_across_chunks(vb):
    mesh = CubeMesh(18, jitter=0.15, seed=2)
    nu = np.ones(mesh.nK)
    A, B, F = _gpu(vb, mesh, 2, nu)
    el = np.array([0, 1, 2500, 5340, 5341, 5342, mesh.nK - 1])  # the first chunk holds 5,341
    Ar, Br, Fr = _ref(mesh, 2, el, nu)
    assert _rel(A[el], Ar) < 1e-12 and _rel(B[el], Br) < 1e-12 and _rel(F[el], Fr) < 1e-11


def test_element_matrices_argument_checks(vb):
    ctx = vb.vb_create()
    try:
        lib = vb.load()
        assert lib.vb_vem_element_matrices(ctx, 5, 1, None, None, 0, None, None, None) == -1
        assert lib.vb_vem_element_matrices(ctx, 2, 1, None, None, 0, None, None, None) == -1
        assert lib.vb_vem_element_matrices(ctx, 2, 0, None, None, 0, None, None, None) == 0
    finally:
        vb.vb_destroy(ctx)
