"""Uniform refinement on the GPU (dg_mesh_refine, the refinement step of the
paper's driver in section 2.1) against the oracle's refinement, bit for bit,
and an h-convergence study whose meshes are refined on the device."""
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


def _shuffled(m, seed):
    """The same triangulation with the elements permuted and each element's
    vertex list rotated (still counter-clockwise)."""
    rng = np.random.default_rng(seed)
    e = m.elems[rng.permutation(len(m.elems))]
    rot = rng.integers(0, 3, len(e))
    e = np.stack([np.roll(r, -s) for r, s in zip(e, rot)]).astype(np.int32)
    return W.MeshArrays(m.nodes, e, m.dirichlet, m.neumann)


MESHES = {
    "paper_2x2": lambda: W.paper_mesh(),
    "structured_8": lambda: W.structured_mesh(8),
    "jittered_9_mixed": lambda: W.structured_mesh(9, dirichlet=("left", "bottom"), neumann=("right", "top"),
                                                  jitter=0.2, seed=4),
    "shuffled_7_neumann": lambda: _shuffled(W.structured_mesh(7, dirichlet=("top",),
                                                              neumann=("left", "right", "bottom")), 5),
    "jittered_128": lambda: W.structured_mesh(128, jitter=0.2, seed=0),
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_refinement_matches_oracle_bitwise(api, name):
    m = MESHES[name]()
    _say("refine %s (%d triangles)" % (name, len(m.elems)))
    mesh = api.Mesh.from_arrays(m, 1)
    r = mesh.refine()
    torch.cuda.synchronize()
    got = r.host()
    ref = O.uniform_refine(m.nodes, m.elems, m.dirichlet, m.neumann)
    for g, o in zip((got.nodes, got.elems, got.dirichlet, got.neumann), ref):
        assert g.shape == o.reshape(g.shape).shape
        np.testing.assert_array_equal(g, o.reshape(g.shape))
    # the refined arrays are a valid mesh for the library
    fine = api.Mesh(r.nodes, r.elems, r.dirichlet, r.neumann, 1)
    assert fine.T == 4 * mesh.T


def test_refining_the_paper_mesh_twice_gives_the_8x8_solution(api):
    """The paper's 2x2 mesh refined twice on the GPU and the structured 8x8
    grid carry the same triangles: the P1 SIPG solutions of the C1 problem
    have the same L2 error up to quadrature error (the collapsed-coordinate
    rule follows each triangle's vertex order, which differs between the two
    meshes, so f is sampled at other points: 2e-7 relative here)."""
    prob = W.sinsin_problem()
    pm = W.paper_mesh()
    mesh = api.Mesh.from_arrays(pm, 1)
    for _ in range(2):
        r = mesh.refine()
        mesh = api.Mesh(r.nodes, r.elems, r.dirichlet, r.neumann, 1)
    errs = []
    for mm in (mesh, api.Mesh.from_arrays(W.structured_mesh(8), 1)):
        vol = mm.qpoints()[0].cpu().numpy()
        gd = mm.qpoints()[1].cpu().numpy()
        f = api.Field.qpoints(torch.from_numpy(np.ascontiguousarray(prob.f(vol[..., 0], vol[..., 1]))).cuda())
        gD = api.Field.qpoints(torch.from_numpy(np.ascontiguousarray(prob.u(gd[..., 0], gd[..., 1]))).cuda())
        sigma, _ = api.default_penalty(api.SIPG, 1)
        P = api.Problem(api.SIPG, 1, sigma, eps=prob.eps, bx=prob.b[0], by=prob.b[1], alpha=prob.alpha, f=f, gD=gD)
        vals, rhs = api.assemble(mm, P)
        s = api.Solver(mm, restart=32, rel_tol=1e-13)
        s.setup(vals)
        x = torch.zeros_like(rhs)
        assert s.solve(rhs, x).converged
        errs.append(api.l2_error(mm, x, prob.u)[0])
    _say("  L2 errors %.15e %.15e" % tuple(errs))
    assert abs(errs[0] - errs[1]) <= 1e-5 * errs[1]


@pytest.mark.parametrize("k", [1, 2])
def test_convergence_order_with_gpu_refinement(api, k):
    """SIPG on the sin(pi x) sin(pi y) problem from a 4x4 mesh refined three
    times on the GPU: assembly, GMRES, L2 error and refinement all on the
    device; the observed order on the finest pair is k + 1 within 0.3."""
    prob = W.sinsin_problem()
    m = W.structured_mesh(4)
    arrays = (m.nodes, m.elems, m.dirichlet, m.neumann)
    errs, hs = [], []
    for level in range(4):
        mesh = api.Mesh(*arrays, k)
        # the problem data are evaluated at the library's points of this mesh
        case = DC.Case("refined_%d" % level, m, k, 2, prob.eps, prob.b, prob.alpha, prob.f)
        vals, rhs = api.assemble(mesh, DC.gpu_problem(case, mesh, api))
        s = api.Solver(mesh, restart=min(16 * 2 ** level + 64, 512), max_iters=20000, rel_tol=1e-12)
        s.setup(vals)
        x = torch.zeros_like(rhs)
        assert s.solve(rhs, x).converged
        l2, hmax = api.l2_error(mesh, x, prob.u)
        errs.append(l2)
        hs.append(hmax)
        r = mesh.refine()
        arrays = (r.nodes, r.elems, r.dirichlet, r.neumann)
    rates = [math.log(errs[i] / errs[i + 1]) / math.log(hs[i] / hs[i + 1]) for i in range(3)]
    _say("  k=%d errors %s rates %s" % (k, ["%.3e" % e for e in errs], ["%.2f" % q for q in rates]))
    assert abs(rates[-1] - (k + 1)) <= 0.3
