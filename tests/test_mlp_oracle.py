"""Pins of the MLP oracle: finite differences, BF16 rounding, Adam's first step."""
import math

import numpy as np
import pytest

from oracle import mlp as OM
from paper_1502_02941_amd import workloads as W


def test_bf16_rounding_values():
    one = 1.0
    ulp = 2.0 ** -7  # spacing of BF16 just above 1
    x = np.array([one, one + ulp / 2, one + 1.5 * ulp, one + ulp / 4, -3.0, 1e-40, 65504.0])
    r = OM.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                 # tie -> even (1.0)
    assert r[2] == one + 2 * ulp       # tie -> even (1 + 2 ulp)
    assert r[3] == 1.0
    assert r[4] == -3.0
    assert r[6] == 65536.0             # 65504 rounds up to 2^16 in BF16
    # representable values are fixed points
    v = OM.bf16(np.random.default_rng(0).standard_normal(1000))
    assert np.array_equal(OM.bf16(v), v)


def test_oracle_gradients_match_central_differences():
    widths = [5, 7, 6, 4]
    p = W.mlp_init(widths, seed=3).astype(np.float64)
    p[p == 0] = 0.05  # nonzero biases
    rng = np.random.default_rng(1)
    X = rng.standard_normal((9, 5))
    T = rng.standard_normal((9, 4))

    def loss(q):
        Y, _ = OM.forward(q, widths, X, bf16_round=False)
        return OM.mse(Y, T)[0]

    Y, cache = OM.forward(p, widths, X, bf16_round=False)
    _, dY = OM.mse(Y, T)
    g = OM.backward(p, widths, cache, dY, bf16_round=False)
    h = 1e-6
    fd = np.array([(loss(p + h * e) - loss(p - h * e)) / (2 * h) for e in np.eye(len(p))])
    assert np.abs(fd - g).max() <= 1e-6 * max(1.0, np.abs(g).max())


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3])
    p, _, _ = OM.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-12)


# A 2-3-2 network whose hidden pre-activations are ln 3, 0 and -ln 3, where
# the logistic function takes the values 3/4, 1/2 and 1/4, so every value
# below is worked out by hand from silu(z) = z / (1 + e^{-z}):
#   x = (1, 2);  W1 = [[0.5, -0.25], [1, 1], [-2, 0.5]],  W1 x = (0, 3, -1)
#   b1 = (ln 3, -3, 1 - ln 3)                 ->  z = (ln 3, 0, -ln 3)
#   h = silu(z) = (3/4 ln 3, 0, -1/4 ln 3)      (no activation on the last layer)
#   W2 = [[1, 5, 2], [-1, 0.5, 4]], b2 = (1/8, -1)
#   y = W2 h + b2 = (1/4 ln 3 + 1/8, -7/4 ln 3 - 1)
# Every input and weight is a BF16 number.  With BF16 rounding of the hidden
# activations: 3/4 ln 3 = 0.8239592... = 1.6479184... * 2^-1 and 1.6479184 * 128
# = 210.93 rounds to 211, so bf16(h_0) = 211/256; -1/4 ln 3 = -1.0986123 * 2^-2
# and 1.0986123 * 128 = 140.62 rounds to 141, so bf16(h_2) = -141/512; then
# y = (211/256 - 282/512 + 1/8, -211/256 - 564/512 - 1) = (0.3984375, -2.92578125).
LN3 = math.log(3.0)
HAND_WIDTHS = [2, 3, 2]
HAND_X = np.array([[1.0, 2.0]])
HAND_W1 = np.array([[0.5, -0.25], [1.0, 1.0], [-2.0, 0.5]])
HAND_B1 = np.array([LN3, -3.0, 1.0 - LN3])
HAND_W2 = np.array([[1.0, 5.0, 2.0], [-1.0, 0.5, 4.0]])
HAND_B2 = np.array([0.125, -1.0])


def _hand_params():
    return np.concatenate([HAND_W1.ravel(), HAND_B1, HAND_W2.ravel(), HAND_B2])


def test_forward_matches_hand_computed_network():
    Y, (H, Z) = OM.forward(_hand_params(), HAND_WIDTHS, HAND_X, bf16_round=False)
    np.testing.assert_allclose(Z[0], [[LN3, 0.0, -LN3]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(H[1], [[0.75 * LN3, 0.0, -0.25 * LN3]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(Y, [[0.25 * LN3 + 0.125, -1.75 * LN3 - 1.0]], rtol=0, atol=1e-15)


def test_bf16_forward_matches_hand_rounded_network():
    Y, (H, _) = OM.forward(_hand_params(), HAND_WIDTHS, HAND_X, bf16_round=True)
    assert H[1][0, 0] == 211.0 / 256.0 and H[1][0, 1] == 0.0 and H[1][0, 2] == -141.0 / 512.0
    np.testing.assert_allclose(Y, [[0.3984375, -2.92578125]], rtol=0, atol=1e-15)


def test_backward_matches_hand_computed_gradients():
    """Gradients of y_0 (dY = (1, 0)) in closed form: dW2[0] = h, db2 = (1, 0),
    dh = W2[0] = (1, 5, 2), dz = dh * silu'(z) with silu'(z) = s (1 + z (1 - s)),
    s = 3/4, 1/2, 1/4; dW1 = dz x^T, db1 = dz."""
    p = _hand_params()
    Y, cache = OM.forward(p, HAND_WIDTHS, HAND_X, bf16_round=False)
    g = OM.backward(p, HAND_WIDTHS, cache, np.array([[1.0, 0.0]]), bf16_round=False)
    dz = np.array([0.75 * (1.0 + LN3 * 0.25), 5.0 * 0.5, 2.0 * 0.25 * (1.0 - LN3 * 0.75)])
    want = np.concatenate([np.outer(dz, HAND_X[0]).ravel(), dz,
                           np.array([[0.75 * LN3, 0.0, -0.25 * LN3], [0.0, 0.0, 0.0]]).ravel(), [1.0, 0.0]])
    np.testing.assert_allclose(g, want, rtol=0, atol=1e-14)
