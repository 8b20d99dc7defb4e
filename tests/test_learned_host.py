"""Host logic of the learned initial guess: folding the standardisation into
the network, and the coarse cell means used as training targets."""
import math

import numpy as np

from oracle import mlp as OM
from paper_1502_02941_amd import learned as L
from paper_1502_02941_amd import workloads as W


def test_folded_network_equals_standardised_network():
    widths = [5, 16, 16, 7]
    rng = np.random.default_rng(0)
    p = W.mlp_init(widths, seed=3) + 0.05 * rng.standard_normal(sum(
        widths[l] * widths[l + 1] + widths[l + 1] for l in range(3))).astype(np.float32)
    X = rng.standard_normal((40, 5)) * [1, 10, 0.1, 3, 1] + [0, 5, -2, 1, 0]
    mu, sd, ys = X.mean(0), X.std(0), 2.5
    ref, _ = OM.forward(p.astype(np.float64), widths, (X - mu) / sd, bf16_round=False)
    folded = L.fold_standardisation(p, widths, mu, sd, ys)
    got, _ = OM.forward(folded.astype(np.float64), widths, X, bf16_round=False)
    np.testing.assert_allclose(got, ys * ref, rtol=2e-5, atol=2e-5 * np.abs(ys * ref).max())


def test_coarse_means_of_piecewise_constants_and_linears():
    n, nc = 8, 4
    m = W.structured_mesh(n)
    T = m.T
    cent = m.nodes[m.elems].mean(axis=1)
    # mean of u_h over a triangle is sqrt(2) c0 with the orthonormal basis
    vals = 1.0 + 2.0 * cent[:, 0] - 3.0 * cent[:, 1]
    x = np.zeros((1, T * 3))
    x[0, 0::3] = vals / math.sqrt(2.0)
    got = L.coarse_means(x, n, nc)[0]
    cc = (np.arange(nc) + 0.5) / nc
    CX, CY = np.meshgrid(cc, cc, indexing="xy")
    np.testing.assert_allclose(got, (1.0 + 2.0 * CX - 3.0 * CY).ravel(), atol=1e-12)
    x[0, 1::3] = 7.0  # higher modes have zero mean
    x[0, 2::3] = -4.0
    np.testing.assert_allclose(L.coarse_means(x, n, nc)[0], got, atol=1e-12)
