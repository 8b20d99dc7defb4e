"""Seeded synthetic inputs: meshes, coefficients and manufactured solutions.

This module describes *problems*, not the method: mesh arrays in the form of
section 2.1 of Uzunca & Karasozen (nodes, counter-clockwise elements,
Dirichlet and Neumann edge lists, 0-based here), coefficient values and exact
solutions with their derivatives.  It holds none of the discretisation's
arithmetic, so both the GPU path and the CPU oracle take their inputs from it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SIDES = ("bottom", "right", "top", "left")  # y=0, x=1, y=1, x=0


@dataclass
class MeshArrays:
    nodes: np.ndarray       # float64 [n_nodes, 2]
    elems: np.ndarray       # int32 [T, 3], counter-clockwise
    dirichlet: np.ndarray   # int32 [n_dir, 2] (start, end node)
    neumann: np.ndarray     # int32 [n_neu, 2]

    @property
    def T(self):
        return len(self.elems)


def structured_mesh(n: int, dirichlet=SIDES, neumann=(), jitter: float = 0.0, seed: int = 0) -> MeshArrays:
    """Unit square split into n x n squares, each cut by its '/' diagonal into the
    counter-clockwise triangles (ll, lr, ur) and (ll, ur, ul), as in the paper's
    figure 2.  Nodes are numbered row by row (node (i,j) -> j*(n+1)+i).
    ``jitter`` > 0 moves every interior node by independent uniform(-jitter*h,
    jitter*h) offsets in x and y, drawn with numpy default_rng(seed) in node order."""
    h = 1.0 / n
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    nodes = np.stack([i.ravel() * h, j.ravel() * h], axis=1).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        off = rng.uniform(-jitter * h, jitter * h, size=nodes.shape)
        ii, jj = i.ravel(), j.ravel()
        interior = (ii > 0) & (ii < n) & (jj > 0) & (jj < n)
        nodes[interior] += off[interior]
    idx = lambda a, b: b * (n + 1) + a
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci, cj = ci.ravel(), cj.ravel()
    ll, lr, ur, ul = idx(ci, cj), idx(ci + 1, cj), idx(ci + 1, cj + 1), idx(ci, cj + 1)
    t1 = np.stack([ll, lr, ur], axis=1)
    t2 = np.stack([ll, ur, ul], axis=1)
    elems = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int32)
    k = np.arange(n)
    side_edges = {
        "bottom": np.stack([idx(k, 0), idx(k + 1, 0)], axis=1),
        "right": np.stack([idx(n, k), idx(n, k + 1)], axis=1),
        "top": np.stack([idx(k + 1, n), idx(k, n)], axis=1),
        "left": np.stack([idx(0, k + 1), idx(0, k)], axis=1),
    }
    for s in tuple(dirichlet) + tuple(neumann):
        if s not in side_edges:
            raise ValueError("unknown side %r" % (s,))
    d = [side_edges[s] for s in dirichlet]
    nm = [side_edges[s] for s in neumann]
    dirr = np.concatenate(d).astype(np.int32) if d else np.zeros((0, 2), np.int32)
    neu = np.concatenate(nm).astype(np.int32) if nm else np.zeros((0, 2), np.int32)
    return MeshArrays(nodes, elems, dirr, neu)


def paper_mesh() -> MeshArrays:
    """The initial 2x2 mesh of the paper's figure 2 (9 nodes, 8 triangles, all
    boundary edges Dirichlet), converted from 1-based to 0-based indices."""
    nodes = np.array([[0, 0], [0.5, 0], [1, 0], [0, 0.5], [0.5, 0.5], [1, 0.5], [0, 1], [0.5, 1], [1, 1]],
                     dtype=np.float64)
    elems = np.array([[4, 1, 5], [1, 2, 5], [5, 2, 6], [2, 3, 6], [7, 4, 8], [4, 5, 8], [8, 5, 9], [5, 6, 9]],
                     dtype=np.int32) - 1
    dirichlet = np.array([[1, 2], [2, 3], [1, 4], [3, 6], [4, 7], [6, 9], [7, 8], [8, 9]], dtype=np.int32) - 1
    return MeshArrays(nodes, elems, dirichlet, np.zeros((0, 2), np.int32))


def uniform_refine(m: MeshArrays) -> MeshArrays:
    """Red refinement: every triangle (a, b, c) is split at its edge midpoints
    into (a, ab, ca), (ab, b, bc), (ca, bc, c) and (ab, bc, ca); boundary edges
    are split in two, keeping their Dirichlet / Neumann type."""
    nodes = [tuple(p) for p in m.nodes]
    mid = {}

    def midpoint(a, b):
        key = (min(a, b), max(a, b))
        if key not in mid:
            mid[key] = len(nodes)
            nodes.append(tuple(0.5 * (m.nodes[a] + m.nodes[b])))
        return mid[key]

    elems = []
    for a, b, c in m.elems:
        ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
        elems += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]

    def split(edges):
        out = []
        for a, b in edges:
            mm = midpoint(a, b)
            out += [(a, mm), (mm, b)]
        return np.array(out, dtype=np.int32).reshape(-1, 2)

    return MeshArrays(np.array(nodes, dtype=np.float64), np.array(elems, dtype=np.int32),
                      split(m.dirichlet), split(m.neumann))


# ----------------------------------------------------------------------------
# Manufactured solutions: u and the data f = alpha u - eps Lap u + b . grad u,
# g^D = u, g^N = eps grad u . n  (section 1, eq. 1).
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    eps: float
    b: tuple                 # (bx, by) constants, or ("affine", (c0,c1,c2), (c0,c1,c2))
    alpha: float
    u: object = None         # u(x, y) or None
    grad_u: object = None    # (ux, uy)(x, y)
    f: object = None         # f(x, y)
    meta: dict = field(default_factory=dict)

    def b_at(self, x, y):
        if self.b[0] == "affine":
            cx, cy = self.b[1], self.b[2]
            return cx[0] + cx[1] * x + cx[2] * y, cy[0] + cy[1] * x + cy[2] * y
        return self.b[0] + 0 * x, self.b[1] + 0 * x

    def gN(self, x, y, nx, ny):
        ux, uy = self.grad_u(x, y)
        return self.eps * (ux * nx + uy * ny)


def sinsin_problem(eps=1e-2, b=(1.0, 1.0), alpha=1.0) -> Problem:
    """u = sin(pi x) sin(pi y) (zero on the boundary of the unit square)."""
    pi = math.pi
    u = lambda x, y: np.sin(pi * x) * np.sin(pi * y)
    gu = lambda x, y: (pi * np.cos(pi * x) * np.sin(pi * y), pi * np.sin(pi * x) * np.cos(pi * y))

    def f(x, y):
        ux, uy = gu(x, y)
        return alpha * u(x, y) + 2.0 * eps * pi * pi * u(x, y) + b[0] * ux + b[1] * uy

    return Problem("sinsin", eps, tuple(b), alpha, u, gu, f)


def boundary_layer_problem(eps=1e-6, b=(1.0, 0.0), alpha=0.0) -> Problem:
    """u = x y (1 - exp((x-1)/eps)) (1 - exp((y-1)/eps)): layers at x=1 and y=1,
    zero on the whole boundary of the unit square."""

    def g(s):
        E = np.exp((s - 1.0) / eps)
        return s * (1.0 - E), 1.0 - E - s * E / eps, -2.0 * E / eps - s * E / (eps * eps)

    def u(x, y):
        return g(x)[0] * g(y)[0]

    def gu(x, y):
        gx, gy = g(x), g(y)
        return gx[1] * gy[0], gx[0] * gy[1]

    def f(x, y):
        gx, gy = g(x), g(y)
        lap = gx[2] * gy[0] + gx[0] * gy[2]
        return alpha * gx[0] * gy[0] - eps * lap + b[0] * gx[1] * gy[0] + b[1] * gx[0] * gy[1]

    return Problem("boundary_layer", eps, tuple(b), alpha, u, gu, f)


def tanh_layer_problem(eps=1e-6, b=(1.0 / math.sqrt(5.0), 2.0 / math.sqrt(5.0)), alpha=1.0) -> Problem:
    """The paper's example (section 4), linear part only: u = (1 - tanh(z))/2 with
    z = (2x - y - 0.25)/sqrt(5 eps); f = alpha u - eps Lap u + b . grad u."""
    s5 = math.sqrt(5.0 * eps)

    def u(x, y):
        return 0.5 * (1.0 - np.tanh((2 * x - y - 0.25) / s5))

    def sech2(z):  # 1 / cosh(z)^2 without overflow
        e = np.exp(-2.0 * np.abs(z))
        return 4.0 * e / (1.0 + e) ** 2

    def gu(x, y):
        s2 = sech2((2 * x - y - 0.25) / s5)
        return -s2 / s5, 0.5 * s2 / s5

    def f(x, y):
        z = (2 * x - y - 0.25) / s5
        s2 = sech2(z)
        uxx = (0.8 / eps) * np.tanh(z) * s2
        uyy = (0.2 / eps) * np.tanh(z) * s2
        ux, uy = -s2 / s5, 0.5 * s2 / s5
        return alpha * u(x, y) - eps * (uxx + uyy) + b[0] * ux + b[1] * uy

    return Problem("tanh_layer", eps, tuple(b), alpha, u, gu, f)


def polynomial_problem(deg: int, eps: float, b, alpha: float, seed: int = 0) -> Problem:
    """A random global polynomial u of total degree <= deg (coefficients N(0,1)).
    With a constant or affine b, f is a polynomial too."""
    rng = np.random.default_rng(seed)
    coef = {(i, j): rng.standard_normal() for i in range(deg + 1) for j in range(deg + 1 - i)}

    def u(x, y):
        return sum(c * x ** i * y ** j for (i, j), c in coef.items())

    def gu(x, y):
        ux = sum(c * i * x ** (i - 1) * y ** j for (i, j), c in coef.items() if i > 0)
        uy = sum(c * j * x ** i * y ** (j - 1) for (i, j), c in coef.items() if j > 0)
        return ux + 0 * x, uy + 0 * x

    def lap(x, y):
        s = 0 * x
        for (i, j), c in coef.items():
            if i > 1:
                s = s + c * i * (i - 1) * x ** (i - 2) * y ** j
            if j > 1:
                s = s + c * j * (j - 1) * x ** i * y ** (j - 2)
        return s

    prob = Problem("poly%d" % deg, eps, b if b[0] == "affine" else tuple(b), alpha, u, gu, None,
                   meta={"coef": coef})

    def f(x, y):
        bx, by = prob.b_at(x, y)
        ux, uy = gu(x, y)
        return alpha * u(x, y) - eps * lap(x, y) + bx * ux + by * uy

    prob.f = f
    return prob


def rotating_b():
    """b = (-(y - 1/2), x - 1/2) as affine coefficients."""
    return ("affine", (0.5, 0.0, -1.0), (-0.5, 1.0, 0.0))


# ----------------------------------------------------------------------------
# Batched workload: many instances with random coefficients and uneven sizes.
# ----------------------------------------------------------------------------
@dataclass
class Instance:
    k: int
    N: int
    eps: float
    theta: float
    bnorm: float
    alpha: float
    gauss: np.ndarray  # [4, 4]: (cx, cy, width, amplitude)

    @property
    def b(self):
        return (self.bnorm * math.cos(self.theta), self.bnorm * math.sin(self.theta))

    def features(self) -> np.ndarray:
        """23 parameters: log10 eps, cos theta, sin theta, |b|, b_x, b_y, alpha, then
        (c_x, c_y, width, amplitude) of the 4 Gaussians."""
        bx, by = self.b
        head = [math.log10(self.eps), math.cos(self.theta), math.sin(self.theta), self.bnorm, bx, by, self.alpha]
        return np.array(head + list(self.gauss.ravel()), dtype=np.float64)

    def f(self, x, y):
        s = 0 * x
        for cx, cy, w, a in self.gauss:
            s = s + a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * w * w))
        return s


def sample_instances(count: int, seed: int = 0, k_choices=(1, 2), n_range=(16, 128), fixed_N=None,
                     fixed_k=None):
    """Draws `count` instances: k uniform over k_choices, N ~ U{n_range}, log10 eps ~
    U[-6,-1], angle ~ U[0, 2 pi], |b| ~ U[0.5, 2], alpha ~ U[0, 1], and 4 Gaussians
    with centres ~ U[0.1, 0.9]^2, widths ~ U[0.02, 0.1], amplitudes ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = int(rng.choice(k_choices)) if fixed_k is None else fixed_k
        N = int(rng.integers(n_range[0], n_range[1] + 1)) if fixed_N is None else fixed_N
        eps = 10.0 ** rng.uniform(-6.0, -1.0)
        theta = rng.uniform(0.0, 2.0 * math.pi)
        bnorm = rng.uniform(0.5, 2.0)
        alpha = rng.uniform(0.0, 1.0)
        c = rng.uniform(0.1, 0.9, size=(4, 2))
        w = rng.uniform(0.02, 0.1, size=(4, 1))
        a = rng.standard_normal(size=(4, 1))
        out.append(Instance(k, N, eps, theta, bnorm, alpha, np.concatenate([c, w, a], axis=1)))
    return out


# ----------------------------------------------------------------------------
# Learned initial guess: seeded initial weights of the multilayer perceptron.
# ----------------------------------------------------------------------------
def mlp_widths():
    """23 instance parameters -> 3 hidden layers of 256 -> 32 x 32 coarse values."""
    return [23, 256, 256, 256, 1024]


def mlp_init(widths, seed=0):
    """Flat FP32 parameter vector W_1, b_1, W_2, b_2, ...: weights ~ N(0, 1/fan_in)
    (the last layer scaled by 0.1), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        fan_in, fan_out = widths[l], widths[l + 1]
        scale = (1.0 if l < len(widths) - 2 else 0.1) / math.sqrt(fan_in)
        parts.append((rng.standard_normal((fan_out, fan_in)) * scale).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)
