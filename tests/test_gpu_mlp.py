"""MLP kernels (BF16 MFMA products, FP32 accumulation) vs the MLP oracle, and
the P0 -> P1 prolongation, through the C ABI."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import mlp as OM
from paper_1502_02941_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_02941_amd import api as A
    A.lib()
    return A


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.mark.parametrize("widths,B", [([23, 256, 256, 256, 1024], 300), ([5, 33, 17, 40], 45), ([64, 64], 32)])
def test_forward_backward_match_oracle(api, widths, B):
    p0 = W.mlp_init(widths, seed=7)
    p0 = p0 + np.float32(0.01) * np.random.default_rng(1).standard_normal(p0.size).astype(np.float32)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((B, widths[0])).astype(np.float32)
    T = rng.standard_normal((B, widths[-1])).astype(np.float32)
    net = api.MLP(widths, max_batch=512, init_params=p0)
    y = net.forward(torch.from_numpy(X).cuda())
    loss, dy = net.loss_mse(torch.from_numpy(T).cuda())
    net.backward(dy)
    p, g = net.params()
    torch.cuda.synchronize()
    Yo, cache = OM.forward(p0, widths, X, bf16_round=True)
    lo, dYo = OM.mse(Yo, T)
    go = OM.backward(p0, widths, cache, dYo, bf16_round=True)
    ey, el = rel(y.cpu().numpy(), Yo), abs(float(loss.item()) - lo) / lo
    ed, eg = rel(dy.cpu().numpy(), dYo), rel(g.cpu().numpy(), go)
    print("widths %s, B %d: Y %.2e, loss %.2e, dY %.2e, gradients %.2e" % (widths, B, ey, el, ed, eg), flush=True)
    assert ey <= 1e-3 and el <= 1e-3 and ed <= 1e-3 and eg <= 1e-3
    np.testing.assert_array_equal(p.cpu().numpy(), p0)


def test_adam_step_matches_oracle(api):
    widths = [8, 16, 4]
    p0 = W.mlp_init(widths, seed=1)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((20, 8)).astype(np.float32)
    T = rng.standard_normal((20, 4)).astype(np.float32)
    net = api.MLP(widths, max_batch=64, init_params=p0)
    m1 = np.zeros(p0.size)
    m2 = np.zeros(p0.size)
    pref = p0.astype(np.float64)
    for t in range(1, 4):
        net.forward(torch.from_numpy(X).cuda())
        _, dy = net.loss_mse(torch.from_numpy(T).cuda())
        net.backward(dy)
        _, g = net.params()
        net.adam_step(1e-3)
        pref, m1, m2 = OM.adam(pref, g.cpu().numpy().astype(np.float64), m1, m2, t, 1e-3)
        p, _ = net.params()
        torch.cuda.synchronize()
        assert np.abs(p.cpu().numpy() - pref).max() <= 1e-6


def test_training_reduces_loss(api):
    widths = [6, 64, 64, 10]
    rng = np.random.default_rng(4)
    X = rng.standard_normal((256, 6)).astype(np.float32)
    A = rng.standard_normal((6, 10))
    T = np.tanh(X @ A).astype(np.float32)
    net = api.MLP(widths, max_batch=256, init_params=W.mlp_init(widths, seed=2))
    Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    losses = []
    for _ in range(300):
        net.forward(Xt)
        loss, dy = net.loss_mse(Tt)
        losses.append(float(loss.item()))
        net.backward(dy)
        net.adam_step(3e-3)
    assert losses[-1] < 0.1 * losses[0]


def test_prolongation_injection_and_bilinear(api):
    n, nc = 16, 8
    m = W.structured_mesh(n)
    mesh = api.Mesh.from_arrays(m, 1)
    rng = np.random.default_rng(5)
    coarse = rng.standard_normal((3, nc * nc)).astype(np.float32)
    x = torch.zeros(3, mesh.n_dofs, dtype=torch.float64, device="cuda")
    api.warmstart_prolong(mesh, torch.from_numpy(coarse).cuda(), nc, 0, x)
    xs = x.cpu().numpy().reshape(3, m.T, 3)
    cent = m.nodes[m.elems].mean(axis=1)
    ci = np.clip((cent[:, 0] * nc).astype(int), 0, nc - 1)
    cj = np.clip((cent[:, 1] * nc).astype(int), 0, nc - 1)
    np.testing.assert_allclose(xs[:, :, 0] * math.sqrt(2.0), coarse[:, cj * nc + ci], rtol=1e-6)
    assert np.abs(xs[:, :, 1:]).max() == 0.0
    # bilinear: coarse values of an affine function are reproduced exactly away
    # from the boundary strip, and the result is continuous (u_h from both sides agrees)
    cc = (np.arange(nc) + 0.5) / nc
    CX, CY = np.meshgrid(cc, cc, indexing="xy")
    f = lambda X_, Y_: 0.3 + 1.2 * X_ - 0.7 * Y_
    lin = f(CX, CY).ravel()[None].astype(np.float32)
    x1 = torch.zeros(1, mesh.n_dofs, dtype=torch.float64, device="cuda")
    api.warmstart_prolong(mesh, torch.from_numpy(lin).cuda(), nc, 1, x1)
    M = O.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann)
    coef = x1.cpu().numpy()[0]
    inner = [e for e in range(m.T) if (m.nodes[m.elems[e]].min() >= 1.0 / nc - 1e-12 and
                                       m.nodes[m.elems[e]].max() <= 1 - 1.0 / nc + 1e-12)]
    pts = cent[inner]
    uh = O.eval_solution(M, 1, coef, np.array(inner), pts)
    np.testing.assert_allclose(uh, f(pts[:, 0], pts[:, 1]), atol=1e-6)
    # continuity at the vertices of an interior edge
    e0, e1 = M.int_el[len(M.int_el) // 2]
    a, b = M.int_v[len(M.int_el) // 2]
    for v in (a, b):
        u0 = O.eval_solution(M, 1, coef, np.array([e0]), m.nodes[v][None])
        u1 = O.eval_solution(M, 1, coef, np.array([e1]), m.nodes[v][None])
        assert abs(u0[0] - u1[0]) <= 1e-6
