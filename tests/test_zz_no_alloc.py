"""dg_solve_small_noalloc (setup + one-workgroup GMRES with no allocation)
against dg_solver_setup + dg_solver_solve on the same path, through the C ABI:
two calls in a row, the second on a smaller system, each bitwise equal to the
allocating path and judged by the oracle's FP64 matrix."""
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


def _case(n, k):
    p = W.sinsin_problem()
    return DC.Case("sinsin_%dx%d_p%d" % (n, n, k), W.structured_mesh(n), k, 2, p.eps, p.b, p.alpha, p.f, tol=1e-11)


def _run_both(api, c, mixed, restart):
    M, B = DC.oracle_system(c)
    mesh = api.Mesh.from_arrays(c.mesh, c.k)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(c, mesh, api))
    s = api.Solver(mesh, restart=restart, rel_tol=c.tol, mixed=mixed, persistent=True)
    s.setup(vals)
    x_ref = torch.zeros_like(rhs)
    rep_ref = s.solve(rhs, x_ref)
    x = torch.zeros_like(rhs)
    rep = torch.zeros(api.REPORT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    api.solve_small_noalloc(mesh, vals, rhs, x, rep, restart=restart, rel_tol=c.tol, mixed=mixed)
    torch.cuda.synchronize()
    R = api.Batch.reports(rep)[0]
    A = B.to_scipy()
    xr = x.cpu().numpy()
    rr = float(np.linalg.norm(B.rhs - A @ xr) / np.linalg.norm(B.rhs))
    _say("  %s mixed=%s: no-alloc %d its rel-res %.2e (oracle-judged %.2e); allocating path %d its rel-res %.2e"
         % (c.name, mixed, R["iters"], R["rel_res"], rr, rep_ref.iters, rep_ref.rel_res))
    assert rep_ref.persistent == 1 and rep_ref.converged
    assert R["status"] == 0 and R["persistent"] == 1
    assert R["iters"] == rep_ref.iters and R["cycles"] == rep_ref.cycles and R["rel_res"] == rep_ref.rel_res
    assert torch.equal(x, x_ref)
    assert rr <= 1.01 * c.tol


@pytest.mark.parametrize("mixed", [False, True])
def test_noalloc_matches_allocating_solve_twice_then_smaller(api, mixed):
    """First call on a 7 x 7 P2 system (588 unknowns), the second on an 8 x 8
    P1 system (384 unknowns): the scratch array keeps the first call's larger
    contents, which the second must not read."""
    _run_both(api, _case(7, 2), mixed, 20)
    _run_both(api, _case(8, 1), mixed, 32)


def test_noalloc_rejects_what_does_not_fit(api):
    c = _case(40, 2)  # 19200 unknowns: the Krylov state does not fit LDS
    mesh = api.Mesh.from_arrays(c.mesh, c.k)
    vals, rhs = mesh.alloc_system()
    x = torch.zeros_like(rhs)
    rep = torch.zeros(api.REPORT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    with pytest.raises(api.DGError):
        api.solve_small_noalloc(mesh, vals, rhs, x, rep, restart=32)
    small = api.Mesh.from_arrays(W.structured_mesh(4), 1)
    v2, r2 = small.alloc_system()
    x2 = torch.zeros_like(r2)
    with pytest.raises(api.DGError):
        api.solve_small_noalloc(small, v2, r2, x2, rep, restart=129)  # above the LDS solver's restart cap
