"""Non-linear reaction and Newton's method (section 3) on the GPU vs the
oracle, through the C ABI."""
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


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_reaction_terms_match_oracle(api, k):
    m = W.structured_mesh(7, dirichlet=("bottom", "left"), neumann=("top", "right"), jitter=0.2, seed=k)
    mesh = api.Mesh.from_arrays(m, k)
    M = O.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann)
    c = [0.3, 1.0, 0.5]
    x = np.random.default_rng(k).standard_normal(mesh.n_dofs) * 0.8
    h, hj = api.reaction_terms(mesh, c, torch.from_numpy(x).cuda())
    ho, hjo = O.reaction_terms(M, k, c, x)
    assert DC.rel_fro(h.cpu().numpy(), ho) <= 1e-12
    assert DC.rel_fro(hj.cpu().numpy(), hjo) <= 1e-12


def _shifted_polynomial(k, seed):
    prob = W.polynomial_problem(k, 0.05, (0.6, -0.4), 0.3, seed=seed)
    g = np.linspace(0, 1, 41)
    shift = 0.2 - min(0.0, prob.u(*np.meshgrid(g, g)).min())
    u = lambda X, Y: prob.u(X, Y) + shift
    f = lambda X, Y: prob.f(X, Y) + prob.alpha * shift + u(X, Y) ** 2
    return prob, u, f


def _oracle_nonlinear_residual(case, k, c, x):
    M, B = DC.oracle_system(case)
    h, _ = O.reaction_terms(M, k, c, x)
    return float(np.linalg.norm(B.to_scipy() @ x + h - B.rhs) / np.linalg.norm(B.rhs))


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("method", [1, 2, 3])
def test_newton_reproduces_polynomial_solution(api, k, method):
    """r(u) = u^2 with f built from a positive global u in P_k: the GPU Newton
    iterate reaches u itself; the oracle's assembly and reaction terms judge the
    residual."""
    prob, u, f = _shifted_polynomial(k, 40 + k)
    m = W.structured_mesh(6, dirichlet=("bottom", "left"), neumann=("top", "right"), jitter=0.2, seed=k)
    case = DC.Case("poly_nl", m, k, method, prob.eps, (0.6, -0.4), prob.alpha, f, gD=u, gN=prob.gN)
    mesh = api.Mesh.from_arrays(m, k)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(case, mesh, api))
    s = api.Solver(mesh, restart=120, max_iters=5000, rel_tol=1e-13)
    x = torch.zeros_like(rhs)
    rep = api.newton_solve(mesh, s, vals, rhs, x, [0.0, 1.0], tol=1e-12, max_newton=30)
    _say("k=%d method %d: %s" % (k, method, rep))
    assert rep["status"] == 0 and rep["newton_steps"] <= 12
    xs = x.cpu().numpy()
    assert _oracle_nonlinear_residual(case, k, [0.0, 1.0], xs) <= 1.01e-12
    M = O.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann)
    pts = M.volume_points(k + 2)
    X, Y = pts[..., 0].ravel(), pts[..., 1].ravel()
    uh = O.eval_solution(M, k, xs, np.repeat(np.arange(M.T), (k + 2) ** 2), np.stack([X, Y], 1))
    assert np.abs(uh - u(X, Y)).max() <= 1e-9 * np.abs(u(X, Y)).max()


def test_newton_paper_example_matches_oracle_newton(api):
    """The paper's example with r(u) = u^2 (section 4: eps = 1e-6, b = (1, 2)/sqrt(5),
    alpha = 1, u = (1 - tanh((2x - y - 1/4)/sqrt(5 eps)))/2) on the paper's mesh
    refined three times, P1 SIPG: GPU Newton and the oracle's Newton (direct
    linear solves) reach the same discrete solution."""
    tl = W.tanh_layer_problem()
    fnl = lambda X, Y: tl.f(X, Y) + tl.u(X, Y) ** 2
    m = W.uniform_refine(W.uniform_refine(W.uniform_refine(W.paper_mesh())))
    case = DC.Case("paper_nl", m, 1, 2, tl.eps, tl.b, tl.alpha, fnl, gD=tl.u)
    mesh = api.Mesh.from_arrays(m, 1)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(case, mesh, api))
    s = api.Solver(mesh, restart=200, max_iters=20000, rel_tol=1e-13)
    x = torch.zeros_like(rhs)
    rep = api.newton_solve(mesh, s, vals, rhs, x, [0.0, 1.0], tol=1e-11, max_newton=50)
    _say("paper example: %s" % rep)
    assert rep["status"] == 0
    M, B = DC.oracle_system(case)
    xo, its, rel, conv = O.newton(M, 1, B, [0.0, 1.0], tol=1e-12, max_newton=50)
    assert conv
    xs = x.cpu().numpy()
    assert np.linalg.norm(xs - xo) <= 1e-8 * np.linalg.norm(xo)
    assert _oracle_nonlinear_residual(case, 1, [0.0, 1.0], xs) <= 1.01e-11


def test_newton_reports_non_convergence_and_invalidates_the_solver(api):
    prob, u, f = _shifted_polynomial(2, 7)
    m = W.structured_mesh(5)
    case = DC.Case("poly_nl", m, 2, 2, prob.eps, (0.6, -0.4), prob.alpha, f, gD=u)
    mesh = api.Mesh.from_arrays(m, 2)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(case, mesh, api))
    s = api.Solver(mesh, restart=80, max_iters=5000, rel_tol=1e-12)
    x = torch.zeros_like(rhs)
    rep = api.newton_solve(mesh, s, vals, rhs, x, [0.0, 1.0], tol=1e-14, max_newton=1)
    assert rep["status"] == api.DG_NOT_CONVERGED and rep["newton_steps"] == 1 and rep["rel_res"] > 1e-14
    with pytest.raises(api.DGError):
        s.solve(rhs, torch.zeros_like(rhs))
    s.setup(vals)
    assert s.solve(rhs, torch.zeros_like(rhs)).converged
