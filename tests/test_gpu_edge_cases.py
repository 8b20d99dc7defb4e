"""Degenerate inputs on the GPU: a mesh of one triangle (no interior edge,
one block), two triangles with Neumann data only, a zero load vector and a
non-finite one, through both solver paths and every Arnoldi block size."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1502_02941_amd import workloads as W
from tests import dgcases as DC

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_02941_amd import api as A
    A.lib()
    return A


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


ONE = W.MeshArrays(np.array([[0.0, 0.0], [1.0, 0.2], [0.3, 0.9]]), np.array([[0, 1, 2]], np.int32),
                   np.array([[0, 1], [1, 2]], np.int32), np.array([[2, 0]], np.int32))
TWO = W.MeshArrays(np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]]),
                   np.array([[0, 1, 2], [0, 2, 3]], np.int32), np.zeros((0, 2), np.int32),
                   np.array([[0, 1], [1, 2], [2, 3], [3, 0]], np.int32))


def _solve_both(api, mesh, vals, rhs, tol):
    """Both solver paths; the kernel-per-step one with 1 to 4 Arnoldi vectors
    per Gram-Schmidt pass (one triangle: the preconditioned operator is the
    identity, so every block breaks down at its first Cholesky pivot)."""
    out = []
    for persistent, block in (("auto", 0), (False, 1), (False, 2), (False, 3), (False, 4)):
        s = api.Solver(mesh, restart=16, max_iters=200, rel_tol=tol, persistent=persistent, block=block)
        s.setup(vals)
        x = torch.zeros_like(rhs)
        rep = s.solve(rhs, x)
        out.append((rep, x.cpu().numpy()))
    return out


@pytest.mark.parametrize("method", [1, 2, 3])
@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("mesh_name", ["one_triangle", "two_triangles_neumann"])
def test_tiny_meshes_match_oracle(api, mesh_name, k, method):
    m = ONE if mesh_name == "one_triangle" else TWO
    alpha = 0.5 if mesh_name == "one_triangle" else 1.0   # pure Neumann needs the reaction
    sigma = 3.0 if k == 0 else None
    case = DC.Case(mesh_name, m, k, method, 0.1, (0.8, -0.3), alpha, lambda x, y: 1.0 + x * y,
                   gD=lambda x, y: x - y, gN=lambda x, y, nx, ny: 0.3 * nx - 0.2 * ny + 0.0 * x, sigma=sigma)
    mesh = api.Mesh.from_arrays(m, k)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(case, mesh, api))
    M, B = DC.oracle_system(case)
    Ao = B.to_scipy()
    assert DC.rel_fro(api.bsr_to_scipy(mesh, vals).tocsr(), Ao) <= 1e-12
    assert DC.rel_fro(rhs.cpu().numpy(), B.rhs) <= 1e-12
    xd = np.linalg.solve(Ao.toarray(), B.rhs)
    for rep, x in _solve_both(api, mesh, vals, rhs, 1e-12):
        assert rep.converged
        assert np.linalg.norm(x - xd) <= 1e-9 * max(np.linalg.norm(xd), 1e-300)


@pytest.mark.parametrize("mixed", [False, True])
def test_zero_and_non_finite_load_vectors(api, mixed):
    """F = 0 gives x = 0 with status OK and no iteration; a NaN in F gives
    DG_ERR_NONFINITE, on both solver paths."""
    m = W.structured_mesh(4)
    mesh = api.Mesh.from_arrays(m, 1)
    case = DC.Case("zero", m, 1, 2, 0.1, (1.0, 0.0), 1.0, 0.0)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(case, mesh, api))
    assert float(rhs.abs().max()) == 0.0
    for persistent, block in (("auto", 0), (False, 1), (False, 2), (False, 3), (False, 4)):
        s = api.Solver(mesh, restart=16, rel_tol=1e-10, mixed=mixed, persistent=persistent, block=block)
        s.setup(vals)
        x = torch.full_like(rhs, 3.0)
        rep = s.solve(rhs, x)
        assert rep.status == 0 and rep.iters == 0 and rep.rel_res == 0.0
        assert float(x.abs().max()) == 0.0
        bad = rhs.clone()
        bad[5] = float("nan")
        with pytest.raises(api.DGError) as e:
            s.solve(bad, torch.zeros_like(rhs))
        assert e.value.status == -7  # DG_ERR_NONFINITE
