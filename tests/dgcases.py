"""Test cases shared by the parity tests: one problem description turned into
inputs for the GPU library and for the CPU oracle.  Each side evaluates the
problem's functions at its own quadrature points."""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

import oracle as O
from paper_1502_02941_amd import workloads as W


@dataclass
class Case:
    name: str
    mesh: W.MeshArrays
    k: int
    method: int          # 1 NIPG, 2 SIPG, 3 IIPG
    eps: float
    b: object            # (bx, by) or ("affine", (c0,c1,c2), (c0,c1,c2))
    alpha: float
    f: object            # float, callable(x, y) or ("gauss", terms)
    gD: object = 0.0     # float or callable(x, y)
    gN: object = 0.0     # float or callable(x, y, nx, ny)
    sigma: float | None = None
    sigma_D: float | None = None
    tol: float = 1e-10
    b0: float = 1.0      # superpenalty exponent: h_e = |e|^b0

    def penalty(self):
        if self.sigma is not None:
            return self.sigma, {1: 1.0, 2: -1.0, 3: 0.0}[self.method]
        return O.default_penalty(self.method, self.k)


def oracle_system(c: Case, basis=O.DUBINER):
    M = O.Mesh(c.mesh.nodes, c.mesh.elems, c.mesh.dirichlet, c.mesh.neumann)
    q = c.k + 2
    sigma, kappa = c.penalty()
    kw = {}
    if callable(c.f):
        pts = M.volume_points(q)
        kw["f"] = O.Field.points(c.f(pts[..., 0], pts[..., 1]))
    elif isinstance(c.f, tuple):
        kw["f"] = O.Field.gauss_sum(c.f[1])
    else:
        kw["f"] = O.Field.const(c.f)
    if callable(c.gD) or callable(c.gN):
        bp, nrm = M.boundary_points(q)
    kw["gD"] = O.Field.points(c.gD(bp[..., 0], bp[..., 1])) if callable(c.gD) else O.Field.const(c.gD)
    kw["gN"] = (O.Field.points(c.gN(bp[..., 0], bp[..., 1], nrm[:, None, 0], nrm[:, None, 1]))
                if callable(c.gN) else O.Field.const(c.gN))
    if c.b[0] == "affine":
        bx, by = O.Field.affine(*c.b[1]), O.Field.affine(*c.b[2])
    else:
        bx, by = O.Field.const(c.b[0]), O.Field.const(c.b[1])
    B = O.assemble(M, c.k, sigma=sigma, kappa=kappa, sigma_D=c.sigma_D, b0=c.b0, eps=c.eps, bx=bx, by=by, alpha=c.alpha,
                   basis=basis, **kw)
    return M, B


def gpu_problem(c: Case, mesh, api):
    """Problem object for the GPU library; QPOINTS data evaluated on the host at
    the library's own points and uploaded."""
    import torch
    sigma, _ = c.penalty()
    F = api.Field
    vol, bnd, nrm, _typ = mesh.qpoints()
    torch.cuda.synchronize()
    if callable(c.f):
        v = vol.cpu().numpy()
        f = F.qpoints(torch.from_numpy(np.ascontiguousarray(c.f(v[..., 0], v[..., 1]))).cuda())
    elif isinstance(c.f, tuple):
        f = F.gauss_sum(c.f[1])
    else:
        f = F.const(c.f)
    b_ = bnd.cpu().numpy()
    n_ = nrm.cpu().numpy()
    gD = F.qpoints(torch.from_numpy(np.ascontiguousarray(c.gD(b_[..., 0], b_[..., 1]))).cuda()) \
        if callable(c.gD) else F.const(c.gD)
    gN = F.qpoints(torch.from_numpy(np.ascontiguousarray(c.gN(b_[..., 0], b_[..., 1], n_[:, None, 0],
                                                               n_[:, None, 1]))).cuda()) \
        if callable(c.gN) else F.const(c.gN)
    if c.b[0] == "affine":
        bx, by = F.affine(*c.b[1]), F.affine(*c.b[2])
    else:
        bx, by = F.const(c.b[0]), F.const(c.b[1])
    return api.Problem(method=c.method, degree=c.k, sigma=sigma, sigma_D=c.sigma_D or 0.0, b0=c.b0,
                       eps=F.const(c.eps), bx=bx, by=by, alpha=F.const(c.alpha), f=f, gD=gD, gN=gN)


def _gauss_terms(seed):
    inst = W.sample_instances(1, seed=seed)[0]
    return inst, [tuple(t) for t in inst.gauss]


def small_cases():
    """Cases the oracle finishes in well under a second; they span several
    workgroups and leave a ragged last workgroup."""
    cases = []
    p1 = W.sinsin_problem()
    cases.append(Case("c1_8x8_p1_sipg", W.structured_mesh(8), 1, 2, p1.eps, p1.b, p1.alpha, p1.f, tol=1e-12))
    for k in (0, 1, 2, 3, 4):
        for meth in (1, 2, 3):
            if k == 0 and meth != 1:
                continue
            pr = W.polynomial_problem(max(k, 1) + 1, 0.05, W.rotating_b(), 0.4, seed=10 * k + meth)
            m = W.structured_mesh(13, dirichlet=("bottom", "left"), neumann=("top", "right"), jitter=0.2,
                                  seed=k + meth)
            cases.append(Case("jit13_p%d_m%d_mixedbc_rot" % (k, meth), m, k, meth, pr.eps, pr.b, pr.alpha, pr.f,
                              gD=pr.u, gN=pr.gN))
    # constant eps, b, alpha: the reference-tensor assembly path (k <= 3) on jittered meshes with
    # mixed boundaries (b enters through Dirichlet and Neumann sides)
    for k in (0, 1, 2, 3, 4):
        for meth in (1, 2, 3):
            if k == 0 and meth != 1:
                continue
            pr = W.polynomial_problem(max(k, 1) + 1, 0.03, (0.8, -0.5), 0.3, seed=100 + 10 * k + meth)
            m = W.structured_mesh(11, dirichlet=("top", "right"), neumann=("bottom", "left"), jitter=0.2,
                                  seed=50 + k + meth)
            cases.append(Case("jit11_p%d_m%d_mixedbc_const" % (k, meth), m, k, meth, pr.eps, pr.b, pr.alpha, pr.f,
                              gD=pr.u, gN=pr.gN))
    bl = W.boundary_layer_problem()
    for meth in (1, 2):
        cases.append(Case("c2like_32_p2_m%d" % meth, W.structured_mesh(32), 2, meth, bl.eps, bl.b, bl.alpha, bl.f))
    cases.append(Case("c3like_24_p3_iipg", W.structured_mesh(24, dirichlet=("left", "bottom"),
                                                              neumann=("right", "top"), jitter=0.2, seed=0),
                      3, 3, 1e-4, W.rotating_b(), 0.5, 1.0))
    inst, terms = _gauss_terms(3)
    cases.append(Case("c4like_20_p%d_gauss" % inst.k, W.structured_mesh(20), inst.k, 2, inst.eps, inst.b,
                      inst.alpha, ("gauss", terms)))
    tl = W.tanh_layer_problem()
    cases.append(Case("paper_e1_linear_p1", W.uniform_refine(W.uniform_refine(W.paper_mesh())), 1, 2, tl.eps, tl.b,
                      tl.alpha, tl.f, gD=tl.u))
    return cases


def superpenalty_cases():
    """b0 != 1 (h_e = |e|^b0): reference-tensor path with constant and with
    rotating b, and the point path (P4)."""
    out = []
    for k, b, b0 in ((2, (0.8, -0.5), 2.0), (3, W.rotating_b(), 1.5), (4, (0.3, 0.9), 2.0)):
        pr = W.polynomial_problem(k + 1, 0.02, b, 0.5, seed=200 + k)
        m = W.structured_mesh(9, dirichlet=("top", "left"), neumann=("bottom", "right"), jitter=0.2, seed=70 + k)
        out.append(Case("jit9_p%d_sipg_b0_%g" % (k, b0), m, k, 2, pr.eps, pr.b, pr.alpha, pr.f, gD=pr.u, gN=pr.gN,
                        b0=b0))
    return out


def c2_full(method=2):
    bl = W.boundary_layer_problem()
    return Case("c2_256_p2_m%d" % method, W.structured_mesh(256), 2, method, bl.eps, bl.b, bl.alpha, bl.f)


def c3_full():
    return Case("c3_512_p3_iipg", W.structured_mesh(512, dirichlet=("left", "bottom"), neumann=("right", "top"),
                                                    jitter=0.2, seed=0), 3, 3, 1e-4, W.rotating_b(), 0.5, 1.0)


def rel_fro(a, b):
    """||a - b||_F / ||b||_F for dense arrays or scipy sparse matrices."""
    import scipy.sparse as sp
    if sp.issparse(a):
        d = (a.tocsr() - b.tocsr()).tocsr()
        return float(np.linalg.norm(d.data) / max(np.linalg.norm(b.tocsr().data), 1e-300))
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_abs_diff(a, b):
    import scipy.sparse as sp
    if sp.issparse(a):
        d = (a.tocsr() - b.tocsr()).tocsr()
        return float(np.abs(d.data).max()) if d.nnz else 0.0, float(np.abs(b.tocsr().data).max())
    return float(np.abs(a - b).max()), float(np.abs(b).max())
