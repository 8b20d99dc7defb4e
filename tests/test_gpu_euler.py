"""Backward Euler in time on the GPU (dg_implicit_euler, dg_euler_rhs; the
time discretisation that section 3 reads its reaction coefficient from)
against the oracle's backward Euler with direct solves."""
import math
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


def _mass(case):
    M = O.Mesh(case.mesh.nodes, case.mesh.elems, case.mesh.dirichlet, case.mesh.neumann)
    return M, O.assemble(M, case.k, sigma=1.0, kappa=-1.0, eps=0.0, bx=0.0, by=0.0, alpha=1.0, f=0.0,
                         parts=O.PART_R)


def _case(k, a0, inv_dt, eps=1e-2, b=(1.0, 0.5), n=8):
    m = W.structured_mesh(n, dirichlet=("left", "bottom"), neumann=("right", "top"), jitter=0.2, seed=11)
    prob = W.sinsin_problem()
    return DC.Case("euler_k%d" % k, m, k, 2, eps, b, a0 + inv_dt, prob.f, gD=prob.u)


@pytest.mark.parametrize("k", [1, 2])
def test_euler_rhs_is_F_plus_mass_times_u(api, k):
    case = _case(k, 0.5, 20.0)
    mesh = api.Mesh.from_arrays(case.mesh, k)
    M, Mass = _mass(case)
    g = np.random.default_rng(k)
    u = g.standard_normal(mesh.n_dofs)
    F = g.standard_normal(mesh.n_dofs)
    out = api.euler_rhs(mesh, torch.from_numpy(F).cuda(), torch.from_numpy(u).cuda(), 20.0).cpu().numpy()
    ref = F + 20.0 * (Mass.to_scipy() @ u)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("k", [1, 2])
def test_implicit_euler_matches_oracle(api, k, mixed):
    """Ten steps of dt = 0.05 on a convection-diffusion problem with mixed
    boundary conditions, from u^0 = 0: the GPU (GMRES to 1e-12 per step, warm
    started from the previous step) against direct solves."""
    a0, inv_dt, steps = 0.5, 20.0, 10
    case = _case(k, a0, inv_dt)
    mesh = api.Mesh.from_arrays(case.mesh, k)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(case, mesh, api))
    s = api.Solver(mesh, restart=40, max_iters=20000, rel_tol=1e-12, mixed=mixed)
    x = torch.zeros_like(rhs)
    rep = api.implicit_euler(mesh, s, vals, rhs, x, inv_dt, steps)
    _say("  k=%d mixed=%s: %s" % (k, mixed, rep))
    assert rep["status"] == 0 and rep["steps"] == steps and rep["newton_steps"] == 0
    M, B = DC.oracle_system(case)
    _, Mass = _mass(case)
    ref = O.implicit_euler(M, k, B, Mass, inv_dt, steps)
    assert np.linalg.norm(x.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)


def test_implicit_euler_nonlinear_matches_oracle(api):
    """r(u) = u^2: each step by Newton on the GPU (GMRES inside) against the
    oracle's Newton with direct solves, five steps from zero."""
    k, a0, inv_dt, steps = 1, 1.0, 10.0, 5
    case = _case(k, a0, inv_dt)
    mesh = api.Mesh.from_arrays(case.mesh, k)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(case, mesh, api))
    s = api.Solver(mesh, restart=40, max_iters=20000, rel_tol=1e-13)
    x = torch.zeros_like(rhs)
    rep = api.implicit_euler(mesh, s, vals, rhs, x, inv_dt, steps, c=[0.0, 1.0], tol=1e-12)
    _say("  nonlinear: %s" % rep)
    assert rep["status"] == 0 and rep["steps"] == steps and rep["newton_steps"] >= steps
    M, B = DC.oracle_system(case)
    _, Mass = _mass(case)
    ref = O.implicit_euler(M, k, B, Mass, inv_dt, steps, c=[0.0, 1.0], tol=1e-13)
    assert np.linalg.norm(x.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)


def test_implicit_euler_reaction_only_closed_form(api):
    """eps = 0, b = 0: every element follows the backward Euler recurrence of
    u_t + a0 u = f0, so the constant mode after N steps is
    (1 - (1 + a0 dt)^-N) f0 / a0 (times 1/sqrt(2))."""
    k, a0, f0, dt, steps = 2, 2.0, 1.5, 0.1, 7
    m = W.structured_mesh(6, jitter=0.2, seed=2)
    case = DC.Case("reaction_only", m, k, 2, 0.0, (0.0, 0.0), a0 + 1.0 / dt, f0, sigma=1.0)
    mesh = api.Mesh.from_arrays(m, k)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(case, mesh, api))
    s = api.Solver(mesh, restart=8, rel_tol=1e-14)
    x = torch.zeros_like(rhs)
    rep = api.implicit_euler(mesh, s, vals, rhs, x, 1.0 / dt, steps)
    assert rep["status"] == 0 and rep["steps"] == steps
    c = x.cpu().numpy().reshape(mesh.T, -1)
    exact = (1.0 - (1.0 + a0 * dt) ** -steps) * f0 / a0
    np.testing.assert_allclose(math.sqrt(2.0) * c[:, 0], exact, rtol=1e-12)
    assert np.abs(c[:, 1:]).max() <= 1e-12


def test_implicit_euler_stops_at_a_failing_step(api):
    """A step that cannot reach its tolerance ends the run: the report names
    the steps completed and the status (the host-side stop, no GPU fault)."""
    case = _case(1, 0.5, 20.0)
    mesh = api.Mesh.from_arrays(case.mesh, 1)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(case, mesh, api))
    s = api.Solver(mesh, restart=5, max_iters=3, rel_tol=1e-14)
    x = torch.zeros_like(rhs)
    rep = api.implicit_euler(mesh, s, vals, rhs, x, 20.0, 4)
    assert rep["status"] == api.DG_NOT_CONVERGED and rep["steps"] == 0
