"""Learned initial guess on the GPU: training with the library's kernels on
solves the method generates, what the trained network gains (the error of the
initial guess), and the residual judge that falls back to the zero guess."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_1502_02941_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL = os.path.join(ROOT, "paper_1502_02941_amd", "data", "c5_mlp.npz")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_02941_amd import api as A
    A.lib()
    from paper_1502_02941_amd import learned
    return learned


@pytest.fixture(scope="module")
def held_out(L):
    """64 held-out instances (seed 2), solved from zero: features, solutions, reports."""
    insts = L.instances(64, seed=2)
    fam = L.Family(insts, mixed=True)
    x, rep = fam.solve()
    torch.cuda.synchronize()
    return insts, x.clone(), fam.batch.reports(rep).copy()


def test_training_on_method_solves_reduces_validation_error(L):
    X, Y, its = L.generate(1024, seed=7, chunk=1024, log=_say)
    assert (its > 0).all()
    m0 = L.train(X, Y, epochs=1, batch=64, n_val=128, log=_say)
    m1 = L.train(X, Y, epochs=60, batch=64, n_val=128, log=_say)
    v0, v1 = m0["history"][-1][2], m1["history"][-1][2]
    _say("validation mse after 1 epoch %.4f, after 60 epochs %.4f" % (v0, v1))
    assert v1 < 0.85 * v0


def test_trained_network_gains_guess_accuracy(L, held_out):
    """The committed network (20000 training solves) predicts the coarse cell
    means of held-out solutions with a median relative error well below the
    zero guess's (which is 1)."""
    insts, x, R = held_out
    truth = L.coarse_means(x.cpu().numpy())
    ws = L.WarmStart(L.load(MODEL), len(insts))
    pred = ws.coarse(torch.from_numpy(L.features(insts)).cuda()).cpu().numpy()
    err = np.linalg.norm(pred - truth, axis=1) / np.linalg.norm(truth, axis=1)
    _say("coarse relative error: median %.3f p90 %.3f" % (np.median(err), np.percentile(err, 90)))
    assert np.median(err) <= 0.6
    # the prolonged guess, measured against the fine solution (L2 of coefficients)
    g = ws.guess(torch.from_numpy(L.features(insts)).cuda())
    fe = ((g - x).norm(dim=1) / x.norm(dim=1)).cpu().numpy()
    _say("prolonged guess relative error: median %.3f" % np.median(fe))
    assert np.median(fe) < 0.9


def test_judged_learned_solve_converges_and_never_costs_iterations(L, held_out):
    """Learned guess + mixed solve with the default judge: every instance
    reaches 1e-10 (checked against the oracle's assembly for two of them);
    a rejected guess restarts from zero."""
    insts, x0, R0 = held_out
    ws = L.WarmStart(L.load(MODEL), len(insts))
    fam = L.Family(insts, mixed=True)
    x = ws.guess(torch.from_numpy(L.features(insts)).cuda())
    x, rep = fam.solve(x)
    torch.cuda.synchronize()
    R = fam.batch.reports(rep)
    assert (R["status"] == 0).all() and (R["rel_res"] <= 1e-10).all()
    rej = R["guess_rejected"] == 1
    _say("rejected %d of %d guesses; rel-res0 median %.3g" % (rej.sum(), len(insts), np.median(R["rel_res0"])))
    assert (R["rel_res0"][rej] > 1.0).all() and (R["rel_res0"][~rej] <= 1.0 + 1e-8).all()
    assert (np.abs(R["iters"][rej].astype(int) - R0["iters"][rej].astype(int)) <= 1).all()
    m = W.structured_mesh(L.FINE)
    M = O.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann)
    xs = x.cpu().numpy()
    for i in (0, 1):
        inst = insts[i]
        sigma, kappa = O.default_penalty(O.SIPG, 1)
        B = O.assemble(M, 1, sigma=sigma, kappa=kappa, eps=inst.eps, bx=inst.b[0], by=inst.b[1], alpha=inst.alpha,
                       f=O.Field.gauss_sum([tuple(t) for t in inst.gauss]), gD=0.0)
        r = np.linalg.norm(B.rhs - B.to_scipy() @ xs[i]) / np.linalg.norm(B.rhs)
        assert r <= 1.01e-10, (i, r)
