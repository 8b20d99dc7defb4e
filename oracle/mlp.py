"""MLP oracle -- TEST INFRASTRUCTURE.

Plain FP64 NumPy forward / backward of the perceptron Z_l = H_{l-1} W_l^T + b_l,
H_l = silu(Z_l) (identity on the last layer), mean-squared-error loss and one
Adam step.  With bf16=True the operands of every product (input, weights,
hidden activations, the dZ factors of the backward products) are rounded to
BF16 (round to nearest even) at the points where the GPU kernels round them;
with bf16=False everything stays FP64 (for finite-difference checks).
"""
import numpy as np


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unflatten(params, widths):
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for l in range(len(widths) - 1):
        n, k = widths[l + 1], widths[l]
        W = p[o:o + n * k].reshape(n, k)
        o += n * k
        b = p[o:o + n]
        o += n
        out.append((W, b))
    assert o == len(p)
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_d(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, widths, X, bf16_round=True):
    r = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unflatten(params, widths)
    H = [r(X)]
    Z = []
    for l, (W, b) in enumerate(layers):
        z = H[-1] @ r(W).T + b
        Z.append(z)
        if l < len(layers) - 1:
            H.append(r(silu(z)))
    return Z[-1], (H, Z)


def mse(Y, T):
    n = Y.size
    return float(np.sum((Y - T) ** 2) / n), 2.0 * (Y - T) / n


def backward(params, widths, cache, dY, bf16_round=True):
    r = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unflatten(params, widths)
    H, Z = cache
    grads = []
    d = np.asarray(dY, dtype=np.float64)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        dz = d if l == len(layers) - 1 else d * silu_d(Z[l])
        grads.append((r(dz).T @ H[l], dz.sum(axis=0)))
        if l > 0:
            d = r(dz) @ r(W)
    grads.reverse()
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adam(params, grads, m1, m2, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m1 = b1 * m1 + (1 - b1) * grads
    m2 = b2 * m2 + (1 - b2) * grads * grads
    mh = m1 / (1 - b1 ** t)
    vh = m2 / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m1, m2
